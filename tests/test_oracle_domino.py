"""Pins for the domino oracle (Aztec diamond).

* Figure "tilestate" (Section 2.2): the oracle's tilestates reproduce the printed
  matrix, and the printed Update formula maps the printed T_w onto T_b.
* Section 1.1.2 (connectivity by rotations): breadth-first search through the
  oracle's rotation primitive from the brick tiling reaches exactly the
  2^(n(n+1)/2) tilings of the order-n Aztec diamond.
* Section 1.1.1 / 1.1.3 (stationary law): visit frequencies match the uniform
  law and the two-periodic edge-weight law P ~ prod w_e (heat-bath and lazy
  Metropolis) in a chi-square test.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_matrix(name):
    rows = [l.split() for l in open(os.path.join(GOLDEN, name)) if l.strip() and not l.startswith("#")]
    return np.array(rows, dtype=np.int64)


def uniform_thr(metropolis=False):
    return oracle.table_from_ratios(oracle.domino_ratios(), metropolis)


def two_periodic_thr(a, b, metropolis=False):
    return oracle.table_from_ratios(oracle.domino_ratios("two", a, b), metropolis)


def chain(n, thr, metropolis=False, seed=1, **kw):
    return oracle.DominoOracle(n, thr, metropolis=metropolis, seed=seed, **kw)


def enumerate_tilings(n):
    d = chain(n, uniform_thr())
    get = lambda: (d.Tb.copy(), d.Tw.copy())

    def put(s):
        d.Tb[:] = s[0]
        d.Tw[:] = s[1]

    seen = bfs(d, get, put, lambda: d.export().tobytes())
    faces = {}
    for k, st in seen.items():
        put(st)
        faces[k] = d.export()
    return faces


def two_periodic_weight(f, n, a, b):
    """prod over dominoes of the weight of the crossed edge: a if the edge's
    even endpoint (x+y even, centred) has x even, b otherwise."""
    w = Fraction(1)
    H, W = f.shape
    for Y in range(H):
        for X in range(W):
            d = f[Y, X]
            if d == 2:      # horizontal domino; crossed edge (X+1,Y)-(X+1,Y+1)
                ends = [(X + 1, Y), (X + 1, Y + 1)]
            elif d == 0:    # vertical domino; crossed edge (X,Y+1)-(X+1,Y+1)
                ends = [(X, Y + 1), (X + 1, Y + 1)]
            else:
                continue
            ex, ey = [(p, q) for (p, q) in ends if (p + q) % 2 == 0][0]
            w *= Fraction(a) if (ex - n) % 2 == 0 else Fraction(b)
    return w


def test_fig_tilestate_matrix_from_oracle_states():
    # The figure's tiling of the 4x4 square (Figure "tilestate"), embedded in the
    # Aztec diamond of order 4 (the square is faces X, Y in [2, 5]); the outer
    # ring is tiled so that no domino crosses the square's boundary.
    M = load_matrix("fig_tilestate.txt")
    n = 4
    f = np.full((8, 8), 255, dtype=np.uint8)

    def dom(p, q):
        (x1, y1), (x2, y2) = p, q
        if x2 == x1 + 1:
            f[y1 + 4, x1 + 4], f[y2 + 4, x2 + 4] = 2, 3
        else:
            f[y1 + 4, x1 + 4], f[y2 + 4, x2 + 4] = 0, 1

    # square (centred face coordinates)
    dom((-2, 0), (-2, 1)); dom((-2, -2), (-2, -1)); dom((1, 0), (1, 1)); dom((1, -2), (1, -1))
    dom((-1, 1), (0, 1)); dom((-1, -2), (0, -2)); dom((-1, -1), (-1, 0)); dom((0, -1), (0, 0))
    # outside ring
    dom((-1, 3), (0, 3)); dom((-2, 2), (-1, 2)); dom((0, 2), (1, 2))
    dom((-2, -3), (-1, -3)); dom((0, -3), (1, -3)); dom((-1, -4), (0, -4))
    dom((-3, 0), (-3, 1)); dom((-4, -1), (-4, 0)); dom((-3, -2), (-3, -1))
    dom((2, 0), (2, 1)); dom((3, -1), (3, 0)); dom((2, -2), (2, -1))
    d = chain(n, uniform_thr())
    d.load(f)

    def internal(X, Y, bit):
        # edge of vertex (X, Y) lies between two faces of the square [2,5]^2
        if bit == 1:   # N: faces (X-1, Y), (X, Y)
            return 3 <= X <= 5 and 2 <= Y <= 5
        if bit == 2:   # S: faces (X-1, Y-1), (X, Y-1)
            return 3 <= X <= 5 and 3 <= Y <= 6
        if bit == 4:   # E: faces (X, Y-1), (X, Y)
            return 2 <= X <= 5 and 3 <= Y <= 5
        return 3 <= X <= 6 and 3 <= Y <= 5   # W: faces (X-1, Y-1), (X-1, Y)

    got = np.zeros((5, 5), dtype=np.int64)
    for row in range(5):
        for col in range(5):
            # printed rows run north to south; printed columns are read as
            # running from east to west (the paper's "E" is column - 1)
            X, Y = 6 - col, 6 - row
            s = d.vertex_state(X, Y)
            got[row, col] = sum(b for b in (1, 2, 4, 8) if s & b and internal(X, Y, b))
    assert (got == M).all(), got


def test_fig_tilestate_update_formula_as_printed():
    # Split the printed matrix (zero padded to an even size) into T_b and T_w
    # and apply the printed UpdateBlack formula to T_w: it must give T_b.
    M = load_matrix("fig_tilestate.txt")
    P = 2
    N = 10
    T = np.zeros((N, N), dtype=np.int64)
    T[P:P + 5, P:P + 5] = M
    Tb = np.zeros((N, N // 2), dtype=np.int64)
    Tw = np.zeros((N, N // 2), dtype=np.int64)
    for i in range(N):
        for j in range(N // 2):
            Tb[i, j] = T[i, 2 * j + i % 2]
            Tw[i, j] = T[i, 2 * j + 1 - i % 2]

    def g(A, i, j):
        return A[i, j] if 0 <= i < N and 0 <= j < N // 2 else 0

    for i in range(1, N - 1):
        for j in range(N // 2):
            p = i % 2
            s = (g(Tw, i - 1, j) & 2) // 2 + 2 * (g(Tw, i + 1, j) & 1) \
                + (g(Tw, i, j + p - 1) & 8) // 2 + 2 * (g(Tw, i, j + p) & 4)
            assert s == Tb[i, j], (i, j)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_rotation_bfs_counts_aztec(n):
    assert len(enumerate_tilings(n)) == 2 ** (n * (n + 1) // 2)


def test_brick_is_all_horizontal_and_valid():
    for n in (1, 2, 5, 8):
        d = chain(n, uniform_thr())
        f = d.export()
        inside = d.in_domain_cells()
        assert set(np.unique(f[inside])) <= {2, 3}
        assert (f[~inside] == 255).all()
        v, _ = d.observe(1)
        assert v == 2 * n * (n + 1)


def test_tiling_valid_after_sweeps_and_resume():
    n = 6
    a = chain(n, uniform_thr(), seed=5)
    a.sweep(7)
    a.sweep(9)
    b = chain(n, uniform_thr(), seed=5)
    b.sweep(16)
    assert (a.export() == b.export()).all()
    c = chain(n, uniform_thr(), seed=5)
    c.load(a.export())   # the export is a valid tiling
    assert (c.export() == a.export()).all()
    d = chain(n, uniform_thr(), seed=6)
    d.sweep(16)
    assert (d.export() != a.export()).any()


@pytest.mark.parametrize("n,samples,thin", [(2, 8000, 8), (3, 16000, 12)])
def test_uniform_stationary(n, samples, thin):
    faces = enumerate_tilings(n)
    probs = {k: 1.0 / len(faces) for k in faces}
    assert chi_square_pvalue(chain(n, uniform_thr(), seed=11), probs, samples, thin) > 1e-3


@pytest.mark.parametrize("metropolis", [False, True])
@pytest.mark.parametrize("n,samples,thin", [(2, 8000, 8), (3, 16000, 12)])
def test_two_periodic_stationary(n, samples, thin, metropolis):
    a, b = Fraction(1), Fraction(1, 2)
    faces = enumerate_tilings(n)
    w = {k: two_periodic_weight(f, n, a, b) for k, f in faces.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = chain(n, two_periodic_thr(a, b, metropolis), metropolis=metropolis, seed=23)
    assert chi_square_pvalue(ch, probs, samples, thin) > 1e-3


def test_two_periodic_orientation_matters():
    # swapping a and b must be detected: the law with a<->b differs at n=3
    a, b = Fraction(1), Fraction(1, 2)
    faces = enumerate_tilings(3)
    w = {k: two_periodic_weight(f, 3, b, a) for k, f in faces.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = chain(3, two_periodic_thr(a, b), seed=23)
    assert chi_square_pvalue(ch, probs, 16000, 12) < 1e-6


def test_observables_accumulate_per_sample():
    n, B = 5, 3
    d = chain(n, uniform_thr(), seed=3, obs_every=2, bin_=B)
    d.sweep(9)
    e = chain(n, uniform_thr(), seed=3)
    acc = np.zeros_like(d.bin_sum)
    tot = 0
    nb = -(-2 * n // B)
    for t in range(9):
        e.sweep(1)
        if (t + 1) % 2 == 0:
            f = e.export()
            hz = (f == 2) | (f == 3)
            tot += int(hz.sum())
            for Y, X in zip(*np.nonzero(hz)):
                acc[(Y // B) * nb + X // B] += 1
    assert int(d.samples[0]) == 4
    assert int(d.scalar_sum[0]) == tot
    assert (d.bin_sum == acc).all()


# ---------------------------------------------------------------- volume weights
# Face (X, Y) of the box is black iff X + Y is even, i.e. iff its south-west
# corner is a black vertex.  With this colouring Thurston's rule makes the
# vertical pair the higher state at black vertices (the up direction of the
# rotations, reading C4).
BLACK_FACE_PARITY = 0


def face_heights(f, n):
    """Height function of a tiling (canonical export, row 0 southmost) by
    Thurston's rule (Section 1.1, Figure "hf"): along an edge with a black face
    on its left the height rises by 1, or falls by 3 if a domino covers the
    edge; with a white face on the left the signs flip.  Returns {vertex: h}
    with h = 0 at the south corner (vertex (n - 1, 0))."""
    W = 2 * n
    inside = lambda X, Y: 0 <= X < W and 0 <= Y < W and f[Y, X] != 255
    black = lambda X, Y: (X + Y) % 2 == BLACK_FACE_PARITY

    def step(u, v):
        (X, Y), (X2, Y2) = u, v
        if X2 == X + 1:        # east: left face (X, Y), right face (X, Y-1)
            left, right = (X, Y), (X, Y - 1)
            crossed = inside(*left) and inside(*right) and f[Y - 1, X] == 0
        elif Y2 == Y + 1:      # north: left face (X-1, Y), right face (X, Y)
            left, right = (X - 1, Y), (X, Y)
            crossed = inside(*left) and inside(*right) and f[Y, X - 1] == 2
        else:
            back = step(v, u)
            return None if back is None else -back
        if not (inside(*left) or inside(*right)):
            return None
        d = 1 if black(*left) else -1
        return -3 * d if crossed else d

    h = {(n - 1, 0): 0}
    todo = [(n - 1, 0)]
    while todo:
        u = todo.pop()
        X, Y = u
        for v in ((X + 1, Y), (X - 1, Y), (X, Y + 1), (X, Y - 1)):
            dh = step(u, v)
            if dh is None:
                continue
            if v in h:
                assert h[v] == h[u] + dh, "inconsistent heights"
            else:
                h[v] = h[u] + dh
                todo.append(v)
    return h


def volume_thr(a, b, metropolis=False):
    return oracle.table_from_ratios(oracle.domino_ratios("volume", a, b), metropolis)


def test_height_rule_and_rotation_sign():
    # every rotation changes the height at its own vertex only, by 4, and the
    # vertical pair is the higher state exactly at black (x+y even) vertices
    n = 3
    faces = enumerate_tilings(n)
    d = chain(n, uniform_thr())
    checked = 0
    for f in faces.values():
        h0 = face_heights(f, n)
        for (X, Y) in d.sites():
            d.load(f)
            if not d.flip(X, Y, 1):
                continue
            h1 = face_heights(d.export(), n)
            diff = {v: h1[v] - h0[v] for v in h0 if h1[v] != h0[v]}
            even = (X - n + Y - n) % 2 == 0
            assert diff == {(X, Y): 4 if even else -4}
            checked += 1
    assert checked > 50


def volume_law(n, a, b):
    faces = enumerate_tilings(n)
    w = {}
    for k, f in faces.items():
        h = face_heights(f, n)
        p = Fraction(1)
        for (X, Y), v in h.items():
            q = a if (X + Y - 2 * n) % 2 == 0 else b
            p *= q ** v
        w[k] = p
    Z = sum(w.values())
    return {k: float(v / Z) for k, v in w.items()}


@pytest.mark.parametrize("metropolis", [False, True])
@pytest.mark.parametrize("n,samples,thin", [(2, 8000, 8), (3, 16000, 12)])
def test_volume_weights_stationary(n, samples, thin, metropolis):
    a, b = Fraction(5, 4), Fraction(2, 3)
    probs = volume_law(n, a, b)
    ch = chain(n, volume_thr(a, b, metropolis), metropolis=metropolis, seed=29)
    assert chi_square_pvalue(ch, probs, samples, thin) > 1e-3


def test_volume_weights_colours_matter():
    a, b = Fraction(5, 4), Fraction(2, 3)
    probs = volume_law(3, b, a)   # black and white weights swapped
    ch = chain(3, volume_thr(a, b), seed=29)
    assert chi_square_pvalue(ch, probs, 16000, 12) < 1e-6
