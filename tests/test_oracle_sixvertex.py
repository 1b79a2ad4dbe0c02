"""Pins for the six-vertex oracle (domain-wall boundary, N x N).

* Section 1.2 (c-flips connect the configurations with fixed boundary):
  breadth-first search through the oracle's flip primitive from h_min reaches
  exactly the alternating-sign-matrix numbers 1, 2, 7, 42, 429, and the
  2-enumeration sum 2^{N_-} equals 2^{N(N-1)/2} (N_- = (#c - N)/2).
* Figure "sixvertexh": the printed heights follow from the printed paths by the
  +-1 rule, and the oracle's c-vertex rule marks exactly the vertices where a
  printed path turns.
* Vertex weights (Figure "sixvertex"(A)): visit frequencies match prod w(v)/Z
  with vertex types read off the edge occupancy, for a = b and for a != b.
* Monotone coupling for a, b <= c; colour-order independence; resume.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def thr(a, b, c2, metropolis=False):
    return oracle.table_from_ratios(oracle.sixv_ratios(a, b, c2), metropolis)


def enumerate_states(N):
    ch = oracle.SixVertexOracle(N, thr(1, 1, 1))
    get = lambda: ch.h.copy()

    def put(s):
        ch.h[:] = s

    seen = bfs(ch, get, put, lambda: ch.export().tobytes())
    out = {}
    for k, s in seen.items():
        put(s)
        out[k] = ch.export()
    return out


def edges_from_heights(h):
    """Occupancy from face heights (Figure "sixvertexh" rule): the vertical edge
    between faces (I-1, J) and (I, J) is occupied iff h rises by 1 in +x; the
    horizontal edge between (I, J-1) and (I, J) iff h rises by 1 in +y."""
    vert = (h[:, 1:] - h[:, :-1]) == 1    # [J, I-1]
    horz = (h[1:, :] - h[:-1, :]) == 1    # [J-1, I]
    return vert, horz


def vertex_weight_product(h, a, b, c):
    """prod over the N x N vertices of a (types a1, a2), b (b1, b2), c (c1, c2)
    read off the edges around each vertex: a1 none, a2 all four, b1 left+right,
    b2 bottom+top, c1 bottom+left, c2 right+top."""
    vert, horz = edges_from_heights(h)
    N = h.shape[0] - 1
    w = Fraction(1)
    for j in range(1, N + 1):
        for i in range(1, N + 1):
            # vertex between faces (i-1, j-1), (i, j-1), (i-1, j), (i, j)
            bottom = vert[j - 1, i - 1]
            top = vert[j, i - 1]
            left = horz[j - 1, i - 1]
            right = horz[j - 1, i]
            e = (bool(left), bool(right), bool(bottom), bool(top))
            if e in ((False, False, False, False), (True, True, True, True)):
                w *= a
            elif e in ((True, True, False, False), (False, False, True, True)):
                w *= b
            elif e in ((True, False, True, False), (False, True, False, True)):
                w *= c
            else:
                raise AssertionError("not one of the six vertex types: %r" % (e,))
    return w


@pytest.mark.parametrize("N,count", [(1, 1), (2, 2), (3, 7), (4, 42), (5, 429)])
def test_bfs_count_is_asm(N, count):
    states = enumerate_states(N)
    assert len(states) == count
    ch = oracle.SixVertexOracle(N, thr(1, 1, 1))
    total = 0
    for h in states.values():
        ch.load(h)
        nc, _ = ch.observe(1)
        assert (nc - N) % 2 == 0
        total += 2 ** ((nc - N) // 2)
    assert total == 2 ** (N * (N - 1) // 2)


def test_fig_sixvertexh():
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "fig_sixvertexh.txt"))
             if l.strip() and not l.startswith("#")]
    k = lines.index("paths")
    heights = np.array([list(map(int, l.split())) for l in lines[1:k]], dtype=np.int64)  # [J][I]
    paths = [[tuple(map(float, p.split(","))) for p in l.split()] for l in lines[k + 1:]]
    occupied = set()
    for pl in paths:
        for (x1, y1), (x2, y2) in zip(pl, pl[1:]):
            steps = int(round(max(abs(x2 - x1), abs(y2 - y1)) / 0.5))
            for s in range(steps):
                p = (x1 + (x2 - x1) * s / steps, y1 + (y2 - y1) * s / steps)
                q = (x1 + (x2 - x1) * (s + 1) / steps, y1 + (y2 - y1) * (s + 1) / steps)
                occupied.add(tuple(sorted([(round(p[0], 2), round(p[1], 2)), (round(q[0], 2), round(q[1], 2))])))
    fx = lambda I: -1.75 + 0.5 * I
    fy = lambda J: -1.25 + 0.5 * J
    # heights follow from the paths by the +-1 rule, bottom-left face = 0
    H = np.zeros_like(heights)
    for J in range(5):
        for I in range(7):
            if I == 0 and J == 0:
                continue
            if I > 0:   # vertical edge on x = fx(I) - 0.25 between y = fy(J) -+ 0.25
                x = round(fx(I) - 0.25, 2)
                e = tuple(sorted([(x, round(fy(J) - 0.25, 2)), (x, round(fy(J) + 0.25, 2))]))
                H[J, I] = H[J, I - 1] + (1 if e in occupied else -1)
            else:
                y = round(fy(J) - 0.25, 2)
                e = tuple(sorted([(round(fx(I) - 0.25, 2), y), (round(fx(I) + 0.25, 2), y)]))
                H[J, I] = H[J - 1, I] + (1 if e in occupied else -1)
    assert (H == heights).all()
    # the oracle's c-vertex rule on the printed heights marks the turning points
    N = 6
    h = np.zeros((N + 1, N + 1), dtype=np.int32)
    h[:5, :] = heights
    ch = oracle.SixVertexOracle(N, thr(1, 1, 1))
    ch.load(h)
    _, per_vertex = ch.observe(1)
    per_vertex = per_vertex.reshape(N, N)      # [j-1][i-1]
    for j in range(1, 5):
        for i in range(1, 7):
            vx, vy = round(-2 + 0.5 * i, 2), round(-1.5 + 0.5 * j, 2)
            e = lambda p, q: tuple(sorted([p, q])) in occupied
            left = e((round(vx - 0.5, 2), vy), (vx, vy))
            right = e((vx, vy), (round(vx + 0.5, 2), vy))
            bottom = e((vx, round(vy - 0.5, 2)), (vx, vy))
            top = e((vx, vy), (vx, round(vy + 0.5, 2)))
            turn = (left and bottom and not right and not top) or (right and top and not left and not bottom)
            assert bool(per_vertex[j - 1, i - 1]) == turn, (i, j)


@pytest.mark.parametrize("metropolis", [False, True])
@pytest.mark.parametrize("a,b,c2", [(1, 1, 1), (1, 1, 2), (2, 1, 4)])
def test_stationary_vertex_weights(a, b, c2, metropolis):
    # weights enter squared (c = sqrt(2) is irrational): w = sqrt(prod w(v)^2)
    states = enumerate_states(4)
    w2 = {k: vertex_weight_product(h, Fraction(a * a), Fraction(b * b), Fraction(c2))
          for k, h in states.items()}
    w = {k: math.sqrt(v) for k, v in w2.items()}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    ch = oracle.SixVertexOracle(4, thr(a, b, c2, metropolis), metropolis=metropolis, seed=41)
    assert chi_square_pvalue(ch, probs, 12000, 8) > 1e-3


def test_a_b_corner_assignment_detected():
    # with a != b, swapping the a and b corners gives a different law
    states = enumerate_states(4)
    w = {k: vertex_weight_product(h, Fraction(1), Fraction(2), Fraction(2)) for k, h in states.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.SixVertexOracle(4, thr(2, 1, 4), seed=41)
    assert chi_square_pvalue(ch, probs, 12000, 8) < 1e-6


def test_monotone_coupling_and_ice_rule():
    N = 12
    t = thr(1, 1, 2)
    top = oracle.SixVertexOracle(N, t, seed=5, init="max")
    bot = oracle.SixVertexOracle(N, t, seed=5, init="min")
    for _ in range(40):
        top.sweep(1)
        bot.sweep(1)
        assert (top.export() >= bot.export()).all()
        for hh in (top.export(), bot.export()):
            assert (np.abs(np.diff(hh, axis=0)) == 1).all() and (np.abs(np.diff(hh, axis=1)) == 1).all()
    top.sweep(4000)
    bot.sweep(4000)
    assert (top.export() == bot.export()).all()


def test_order_independence_and_resume():
    t = thr(1, 1, 2)
    a = oracle.SixVertexOracle(10, t, seed=9)
    a.sweep(30)
    oracle.set_reverse_order(True)
    try:
        b = oracle.SixVertexOracle(10, t, seed=9)
        b.sweep(11)
        b.sweep(19)
    finally:
        oracle.set_reverse_order(False)
    assert (a.export() == b.export()).all()


# ------------------------------------------------------ six vertex weights
def vertex_weight_product6(h, wts):
    """prod over the N x N vertices of the weight of the vertex type read off
    the edges (a1 none, a2 all four, b1 left+right, b2 bottom+top, c1
    bottom+left, c2 right+top); wts = (a1, a2, b1, b2, c1, c2)."""
    vert, horz = edges_from_heights(h)
    N = h.shape[0] - 1
    kinds = {(False, False, False, False): 0, (True, True, True, True): 1, (True, True, False, False): 2,
             (False, False, True, True): 3, (True, False, True, False): 4, (False, True, False, True): 5}
    w = Fraction(1)
    for j in range(1, N + 1):
        for i in range(1, N + 1):
            e = (bool(horz[j - 1, i - 1]), bool(horz[j - 1, i]), bool(vert[j - 1, i - 1]), bool(vert[j, i - 1]))
            w *= Fraction(wts[kinds[e]])
    return w


WTS6 = (1, 2, Fraction(3, 2), Fraction(1, 2), 1, 3)


def test_six_weights_reduce_to_three():
    for a, b, c in ((1, 1, 1), (2, 3, 5), (Fraction(1, 2), 3, 7)):
        assert oracle.sixv_ratios6(a, a, b, b, c, c) == oracle.sixv_ratios(a, b, c * c)


def test_six_weights_enter_through_products():
    # a corner of a flipped face moves between two types whose weights
    # multiply to a1 a2, b1 b2 or c1 c2: only those products matter
    base = oracle.sixv_ratios6(*WTS6)
    a1, a2, b1, b2, c1, c2 = [Fraction(x) for x in WTS6]
    for x, y, z in ((Fraction(1, 3), 5, Fraction(7, 2)), (2, Fraction(1, 9), 1)):
        assert oracle.sixv_ratios6(x, a1 * a2 / x, y, b1 * b2 / y, z, c1 * c2 / z) == base
    assert oracle.sixv_ratios6(2, 1, 1, 1, 1, 1) != oracle.sixv_ratios6(1, 1, 1, 1, 1, 1)


def test_six_weight_table_matches_whole_configurations():
    # every flip of every DWBC N = 4 state: the ratio of the two full
    # configuration weights equals the table entry of the flip's mask
    R = oracle.sixv_ratios6(*WTS6)
    states = enumerate_states(4)
    seen = set()
    for h in states.values():
        for J in range(1, 4):
            for I in range(1, 4):
                m = h[J, I + 1]
                if not (h[J, I - 1] == m and h[J + 1, I] == m and h[J - 1, I] == m):
                    continue
                mask = sum(1 << k for k, (dI, dJ) in enumerate(((1, 1), (-1, 1), (-1, -1), (1, -1)))
                           if h[J + dJ, I + dI] == m + 1)
                up, down = h.copy(), h.copy()
                up[J, I], down[J, I] = m + 1, m - 1
                assert vertex_weight_product6(up, WTS6) / vertex_weight_product6(down, WTS6) == R[mask]
                seen.add(mask)
    assert len(seen) >= 8


@pytest.mark.parametrize("metropolis", [False, True])
def test_stationary_six_weights(metropolis):
    states = enumerate_states(4)
    w = {k: vertex_weight_product6(h, WTS6) for k, h in states.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    t6 = oracle.table_from_ratios(oracle.sixv_ratios6(*WTS6), metropolis)
    ch = oracle.SixVertexOracle(4, t6, metropolis=metropolis, seed=43)
    assert chi_square_pvalue(ch, probs, 12000, 8) > 1e-3
