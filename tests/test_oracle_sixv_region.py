"""Pins for the oracle's six-vertex model on general domains (Section 1.2 with
the domains of Section 1.1; the L-shaped example with domain-wall type
boundary).

* on the N x N square the boundary heights are the domain-wall ones, the
  extremes are |I - J| and N - |I + J - N|, and the chain equals the
  domain-wall oracle bit for bit (same draws, moves and contexts);
* a brute-force enumerator of height functions (checked against the ASM
  numbers on squares) decides which domains admit a configuration, and the
  extremes are the pointwise max / min over everything it finds;
* flips from either extreme reach every enumerated configuration, the
  chain's law on an L-shape is prod w(vertex) (chi-square), and coupling
  from the past coalesces from every state.
"""
import math
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue
from test_oracle_cftp import chi_square_of_samples, run_from
from test_oracle_region import accepted, l_shape, ones, random_domain
import test_oracle_sixvertex as tos

I32MIN = np.iinfo(np.int32).min


def enumerate_configs(mask, free_north=False, free_side=None):
    """Every height function of the domain (brute force): sites (and free
    points) in row-major order take a value one away from their west or
    south neighbour (one of them is known: a free point of a south or west
    side may lack it, then both values one away from its known neighbour are
    tried), and a complete assignment is kept if every cell side joins
    heights one apart."""
    side = free_side or ("north" if free_north else None)
    pts, sites = oracle.sixv_points(mask)
    hb = oracle.sixv_boundary_heights(mask, free_side=side)
    H = np.full(pts.shape, I32MIN, dtype=np.int64)
    for (I, J), v in hb.items():
        H[J, I] = v
    free = oracle.sixv_free_points(mask, side) if side else np.zeros_like(pts)
    order = [(I, J) for J in range(pts.shape[0]) for I in range(pts.shape[1]) if sites[J, I] or free[J, I]]
    fixed = {(I, J) for (I, J) in hb}
    out = []

    m = np.asarray(mask, dtype=bool)

    def valid():
        # every side of every cell of the domain joins heights one apart
        for y, x in zip(*np.nonzero(m)):
            c = H[y:y + 2, x:x + 2]
            if abs(c[0, 0] - c[0, 1]) != 1 or abs(c[1, 0] - c[1, 1]) != 1 or abs(c[0, 0] - c[1, 0]) != 1 \
                    or abs(c[0, 1] - c[1, 1]) != 1:
                return False
        return True

    def rec(i):
        if i == len(order):
            if valid():
                out.append(H.copy())
            return
        I, J = order[i]

        def known(a, b):
            return 0 <= b < H.shape[0] and 0 <= a < H.shape[1] and H[b, a] != I32MIN

        base = H[J, I - 1] if known(I - 1, J) else H[J - 1, I]
        for v in (base - 1, base + 1):
            if known(I - 1, J) and abs(v - H[J, I - 1]) != 1:
                continue
            if known(I, J - 1) and abs(v - H[J - 1, I]) != 1:
                continue
            if (I + 1, J) in fixed and abs(v - H[J, I + 1]) != 1:
                continue
            if (I, J + 1) in fixed and abs(v - H[J + 1, I]) != 1:
                continue
            H[J, I] = v
            rec(i + 1)
        H[J, I] = I32MIN

    rec(0)
    return out


def vertex_weight(mask, H, a, b, c):
    """prod over the domain's cells of a, b or c by the vertex type read off
    the edge occupancy (a: none or all four, b: left+right or bottom+top,
    c: bottom+left or right+top)."""
    vert = (H[:, 1:] - H[:, :-1]) == 1
    horz = (H[1:, :] - H[:-1, :]) == 1
    w = Fraction(1)
    for y, x in zip(*np.nonzero(mask)):
        e = (bool(horz[y, x]), bool(horz[y, x + 1]), bool(vert[y, x]), bool(vert[y + 1, x]))
        if e in ((False, False, False, False), (True, True, True, True)):
            w *= a
        elif e in ((True, True, False, False), (False, False, True, True)):
            w *= b
        elif e in ((True, False, True, False), (False, True, False, True)):
            w *= c
        else:
            raise AssertionError("not a six-vertex configuration")
    return w


def chain(mask, thr=None, seed=1, init="min", **kw):
    return oracle.SixVertexRegionOracle(mask, thr if thr is not None else tos.thr(1, 1, 1), seed=seed, init=init,
                                        **kw)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 9])
def test_square_is_the_domain_wall_square(N):
    m = ones(N, N)
    hmax, hmin = oracle.sixv_extremal_heights(m)
    I, J = np.meshgrid(np.arange(N + 1), np.arange(N + 1))
    assert (hmin == np.abs(I - J)).all() and (hmax == N - np.abs(I + J - N)).all()
    d = oracle.SixVertexOracle(N, tos.thr(1, 1, 1))
    hb = oracle.sixv_boundary_heights(m)
    for (i, j), v in hb.items():
        assert d.export()[j, i] == v


@pytest.mark.parametrize("w2,metro,random", [((1, 1, 2), False, False), ((4, 1, 4), True, False),
                                             ((1, 1, 1), False, True)])
def test_square_chain_equals_the_domain_wall_chain(w2, metro, random):
    N = 12
    thr = oracle.table_from_ratios(oracle.sixv_ratios(int(round(w2[0] ** 0.5)), int(round(w2[1] ** 0.5)), w2[2]),
                                   metro)
    for init in ("min", "max"):
        a = chain(ones(N, N), thr, seed=5, init=init, metropolis=metro, random_colours=random)
        b = oracle.SixVertexOracle(N, thr, metropolis=metro, seed=5, init=init, random_colours=random)
        for k in (1, 3, 8):
            a.sweep(k)
            b.sweep(k)
            assert (a.export() == b.export()).all()


@pytest.mark.parametrize("N,asm", [(1, 1), (2, 2), (3, 7), (4, 42), (5, 429)])
def test_enumerator_counts_alternating_sign_matrices(N, asm):
    assert len(enumerate_configs(ones(N, N))) == asm


def check_against_enumeration(m):
    try:
        hmax, hmin = oracle.sixv_extremal_heights(m)
    except oracle.Untileable:
        try:
            configs = enumerate_configs(m)
        except oracle.Untileable:
            return 0
        assert configs == []
        return 0
    configs = enumerate_configs(m)
    assert configs
    stack = np.stack(configs)
    pts = hmax != I32MIN
    assert (stack.max(axis=0)[pts] == hmax[pts]).all() and (stack.min(axis=0)[pts] == hmin[pts]).all()
    keys = {c.tobytes() for c in configs}
    assert hmax.tobytes() in keys and hmin.tobytes() in keys
    # flips from either extreme reach every configuration
    for init in ("min", "max"):
        ch = chain(m, init=init)
        get = lambda: ch.H.copy()

        def put(s):
            ch.H[:] = s

        seen = bfs(ch, get, put, lambda: ch.export().astype(np.int64).tobytes())
        assert set(seen) == keys
    return len(configs)


@pytest.mark.parametrize("name", ["l4", "l5", "l6b", "rect3x5", "rect4x2", "t"])
def test_named_domains(name):
    t = ones(4, 5)
    t[:2, :2] = False
    t[:2, 3:] = False
    m = {"l4": l_shape(4, 2, 2), "l5": l_shape(5, 2, 3), "l6b": l_shape(6, 3, 3), "rect3x5": ones(3, 5),
         "rect4x2": ones(4, 2), "t": t}[name]
    check_against_enumeration(m)


def test_l_shapes():
    # square minus a corner block: thick arms admit configurations, thin ones
    # (fewer cells to route the entering paths through) may not
    counts = {}
    for a in range(2, 7):
        for b in range(1, a):
            for c in range(1, a):
                counts[(a, b, c)] = check_against_enumeration(l_shape(a, b, c))
    assert counts[(4, 2, 2)] > 0 and counts[(6, 3, 3)] > 0 and counts[(3, 2, 2)] == 0


@pytest.mark.parametrize("seed", range(10))
def test_random_domains(seed):
    rng = np.random.default_rng(seed)
    m = random_domain(rng, 4 + seed % 3, 4, 0.7)
    check_against_enumeration(m)


def test_some_domains_have_no_configuration():
    found = 0
    for bits in range(1, 1 << 9):
        m = np.array([(bits >> i) & 1 for i in range(9)], dtype=bool).reshape(3, 3)
        if not accepted(m):
            continue
        try:
            oracle.sixv_extremal_heights(m)
        except oracle.Untileable:
            found += 1
            continue
    assert found > 0
    # a 2 x 1 domino of cells: two paths enter (south, west) but three legs leave
    with pytest.raises(oracle.Untileable):
        oracle.sixv_extremal_heights(ones(1, 2))


def test_law_on_an_l_shape():
    m = l_shape(5, 2, 3)
    configs = enumerate_configs(m)
    w = {c.astype(np.int64).tobytes(): math.sqrt(vertex_weight(m, c, 1, 1, 2)) for c in configs}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    ch = chain(m, tos.thr(1, 1, 2), seed=31)

    class View:
        def sweep(self, n):
            ch.sweep(n)

        def export(self):
            return ch.export().astype(np.int64)

    assert chi_square_pvalue(View(), probs, 8000, 4) > 1e-3


def test_cftp_on_an_l_shape():
    m = l_shape(5, 2, 3)
    states = enumerate_configs(m)
    for seed in range(4):
        make = lambda init, s=seed: chain(m, tos.thr(1, 1, 2), seed=s, init=init)
        R, sample = oracle.cftp(make)
        for st in states:
            assert np.array_equal(run_from(make, st, R), sample)


def test_observables_on_a_domain():
    m = l_shape(8, 3, 4)
    ch = chain(m, seed=2, obs_every=2, bin_=3)
    ch.sweep(9)
    v, bs = ch.observe()
    assert v == int(oracle.sixv_c_vertices(m, ch.export()).sum()) and bs.sum() == v
    assert int(ch.samples[0]) == 4


# ------------------------------------------------------------ free north edge

STOCH = (1, 1, Fraction(3, 10), Fraction(7, 10), Fraction(3, 10), Fraction(7, 10))


def weight6(mask, H, wts):
    """prod over the domain's cells of the weight of the vertex type read off
    the corner heights (a1 none, a2 all four, b1 left+right, b2 bottom+top,
    c1 bottom+left, c2 right+top)."""
    names = ("a1", "a2", "b1", "b2", "c1", "c2")
    w = dict(zip(names, [Fraction(x) for x in wts]))
    p = Fraction(1)
    for y, x in zip(*np.nonzero(mask)):
        p *= w[oracle.sixv_vertex_type(H[y, x], H[y, x + 1], H[y + 1, x], H[y + 1, x + 1])]
    return p


def free_chain(mask, wts, seed=1, init="min", **kw):
    thr = oracle.table_from_ratios(oracle.sixv_ratios6(*wts), False)
    thr_free = oracle.table_from_ratios(oracle.sixv_free_ratios6(*wts), False)
    return oracle.SixVertexRegionOracle(mask, thr, seed=seed, init=init, free_north=True, thr_free=thr_free, **kw)


@pytest.mark.parametrize("hw", [(3, 4), (2, 5), (4, 4), (3, 6)])
def test_free_north_extremes_and_connectivity(hw):
    m = ones(*hw)
    configs = enumerate_configs(m, free_north=True)
    assert configs
    hmax, hmin = oracle.sixv_extremal_heights(m, free_north=True)
    stack = np.stack(configs)
    pts = hmax != I32MIN
    assert (stack.max(axis=0)[pts] == hmax[pts]).all() and (stack.min(axis=0)[pts] == hmin[pts]).all()
    keys = {c.tobytes() for c in configs}
    for init in ("min", "max"):
        ch = free_chain(m, STOCH, init=init)
        get = lambda: ch.H.copy()

        def put(s):
            ch.H[:] = s

        seen = bfs(ch, get, put, lambda: ch.export().astype(np.int64).tobytes())
        assert set(seen) == keys
    # on the square the fixed west and east sides force the free top edge
    # (N steps from N down to 0): the configurations are the domain-wall ones
    if hw[0] == hw[1]:
        assert {c.tobytes() for c in enumerate_configs(m)} == keys


def test_free_table_is_the_configuration_weight_ratio():
    # every flip at a free point of every configuration changes the weight by
    # the table entry of its context
    m = ones(3, 5)
    wts = (2, 1, Fraction(3, 10), Fraction(7, 10), Fraction(1, 2), 3)
    R = oracle.sixv_free_ratios6(*wts)
    free = oracle.sixv_free_points(m)
    checked = 0
    for H in enumerate_configs(m, free_north=True):
        for J, I in np.argwhere(free):
            e, w_, s = H[J, I + 1], H[J, I - 1], H[J - 1, I]
            if not (e == w_ == s) or H[J, I] != e - 1:
                continue
            ctx = (1 if H[J - 1, I - 1] == e + 1 else 0) | (2 if H[J - 1, I + 1] == e + 1 else 0)
            up = H.copy()
            up[J, I] = e + 1
            assert weight6(m, up, wts) / weight6(m, H, wts) == R[ctx]
            checked += 1
    assert checked > 20


@pytest.mark.parametrize("wts", [STOCH, (1, 2, 1, Fraction(1, 2), 3, 1)])
def test_free_north_law(wts):
    m = ones(3, 4)
    configs = enumerate_configs(m, free_north=True)
    w = {c.astype(np.int64).tobytes(): float(weight6(m, c, wts)) for c in configs}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    ch = free_chain(m, wts, seed=41)

    class View:
        def sweep(self, n):
            ch.sweep(n)

        def export(self):
            return ch.export().astype(np.int64)

    assert chi_square_pvalue(View(), probs, 12000, 3) > 1e-3


def test_free_north_law_needs_the_free_table():
    # negative control: flipping free points with the interior table's
    # product form (a2 = a1 a2, ...) gives another law
    m = ones(3, 4)
    wts = STOCH
    configs = enumerate_configs(m, free_north=True)
    w = {c.astype(np.int64).tobytes(): float(weight6(m, c, wts)) for c in configs}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    thr = oracle.table_from_ratios(oracle.sixv_ratios6(*wts), False)
    wrong = oracle.table_from_ratios(oracle.sixv_free_ratios6(1, 1, Fraction(21, 100), 1, Fraction(21, 100), 1),
                                     False)
    ch = oracle.SixVertexRegionOracle(m, thr, seed=41, free_north=True, thr_free=wrong)

    class View:
        def sweep(self, n):
            ch.sweep(n)

        def export(self):
            return ch.export().astype(np.int64)

    assert chi_square_pvalue(View(), probs, 12000, 3) < 1e-6


def test_free_north_refuses_split_boundaries():
    # an L-shape's free north edges cut its fixed boundary in two
    with pytest.raises(ValueError):
        oracle.sixv_extremal_heights(l_shape(6, 3, 3), free_north=True)


# ------------------------------------------------- free south, east, west sides
# The same pins for a free side anywhere: the enumerated configurations are
# what the chain's flips reach from either extreme, every flip at a free point
# changes the configuration weight by the free table's entry, and the chain's
# law is the weight product (chi-square, with the interior table's product
# form as a negative control).  Wide boxes for north / south, tall for east /
# west (the others have no configuration).

SIDE_BOXES = {"north": (3, 4), "south": (3, 4), "east": (4, 3), "west": (4, 3)}


def side_chain(mask, wts, side, seed=1, init="min", thr_free=None, **kw):
    thr = oracle.table_from_ratios(oracle.sixv_ratios6(*wts), False)
    if thr_free is None:
        thr_free = oracle.table_from_ratios(oracle.sixv_free_ratios6(*wts, side=side), False)
    return oracle.SixVertexRegionOracle(mask, thr, seed=seed, init=init, free_side=side, thr_free=thr_free, **kw)


class _View:
    def __init__(self, ch):
        self.ch = ch

    def sweep(self, n):
        self.ch.sweep(n)

    def export(self):
        return self.ch.export().astype(np.int64)


@pytest.mark.parametrize("side", ["north", "south", "east", "west"])
def test_free_side_extremes_and_connectivity(side):
    m = ones(*SIDE_BOXES[side])
    configs = enumerate_configs(m, free_side=side)
    assert len(configs) > 3
    hmax, hmin = oracle.sixv_extremal_heights(m, free_side=side)
    stack = np.stack(configs)
    pts = hmax != I32MIN
    assert (stack.max(axis=0)[pts] == hmax[pts]).all() and (stack.min(axis=0)[pts] == hmin[pts]).all()
    free = oracle.sixv_free_points(m, side)
    assert free.sum() == (SIDE_BOXES[side][1] - 1 if side in ("north", "south") else SIDE_BOXES[side][0] - 1)
    keys = {c.tobytes() for c in configs}
    for init in ("min", "max"):
        ch = side_chain(m, STOCH, side, init=init)
        get = lambda: ch.H.copy()

        def put(s_):
            ch.H[:] = s_

        seen = bfs(ch, get, put, lambda: ch.export().astype(np.int64).tobytes())
        assert set(seen) == keys


@pytest.mark.parametrize("side", ["north", "south", "east", "west"])
def test_free_side_table_is_the_configuration_weight_ratio(side):
    m = ones(*SIDE_BOXES[side])
    wts = (2, 1, Fraction(3, 10), Fraction(7, 10), Fraction(1, 2), 3)
    R = oracle.sixv_free_ratios6(*wts, side=side)
    free = oracle.sixv_free_points(m, side)
    miss = oracle.FREE_SIDES[side]["missing"]
    d0, d1 = oracle.FREE_SIDES[side]["diag"]
    nbrs = [d for d in ((1, 0), (-1, 0), (0, 1), (0, -1)) if d != miss]
    checked = 0
    for H in enumerate_configs(m, free_side=side):
        for J, I in np.argwhere(free):
            vals = [H[J + dj, I + di] for di, dj in nbrs]
            if len(set(vals)) != 1 or H[J, I] != vals[0] - 1:
                continue
            e = vals[0]
            ctx = (1 if H[J + d0[1], I + d0[0]] == e + 1 else 0) | (2 if H[J + d1[1], I + d1[0]] == e + 1 else 0)
            up = H.copy()
            up[J, I] = e + 1
            assert weight6(m, up, wts) / weight6(m, H, wts) == R[ctx]
            checked += 1
    assert checked > 5


@pytest.mark.parametrize("side", ["south", "east", "west"])
def test_free_side_law(side):
    m = ones(*SIDE_BOXES[side])
    wts = STOCH
    configs = enumerate_configs(m, free_side=side)
    w = {c.astype(np.int64).tobytes(): float(weight6(m, c, wts)) for c in configs}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    assert chi_square_pvalue(_View(side_chain(m, wts, side, seed=41)), probs, 12000, 3) > 1e-3
    # negative control: the north table on this side gives another law
    wrong = oracle.table_from_ratios(oracle.sixv_free_ratios6(*wts, side="north"), False)
    if list(wrong) != list(oracle.table_from_ratios(oracle.sixv_free_ratios6(*wts, side=side), False)):
        assert chi_square_pvalue(_View(side_chain(m, wts, side, seed=41, thr_free=wrong)), probs, 12000, 3) < 1e-6


def test_free_side_tables_differ_by_side():
    # the four sides change different cells, so their tables differ for
    # generic weights; the north one has the closed form of its two cells
    wts = (2, 1, Fraction(3, 10), Fraction(7, 10), Fraction(1, 2), 3)
    tabs = {s_: oracle.sixv_free_ratios6(*wts, side=s_) for s_ in ("north", "south", "east", "west")}
    assert len({tuple(v) for v in tabs.values()}) == 4
    # a closed form for the north table (two cells below the point)
    a1, a2, b1, b2, c1, c2 = [Fraction(x) for x in wts]
    north = [(c2 / a1 if ctx & 1 else a2 / c1) * (c1 / b2 if ctx & 2 else b1 / c2) for ctx in range(4)]
    assert tabs["north"] == north


@pytest.mark.parametrize("side", ["north", "south", "east", "west"])
def test_free_side_draws_use_offsets(side):
    # a free south (west) side keys the draws two rows (columns) up (right):
    # the chain equals a step-by-step replay of two sweeps, in plain Python,
    # with those keys, the side's neighbours and contexts, and the tables
    m = ones(*SIDE_BOXES[side])
    wts = STOCH
    ch = side_chain(m, wts, side, seed=9, init="max")
    ox, oy = (2, 0) if side == "west" else (0, 2) if side == "south" else (0, 0)
    assert (ch.ox, ch.oy) == (ox, oy)
    thr = oracle.table_from_ratios(oracle.sixv_ratios6(*wts), False)
    thr_free = oracle.table_from_ratios(oracle.sixv_free_ratios6(*wts, side=side), False)
    miss = oracle.FREE_SIDES[side]["missing"]
    d0, d1 = oracle.FREE_SIDES[side]["diag"]
    H = ch.H.astype(np.int64).copy()
    site = ch.site
    for t in range(2):
        for c in range(4):
            for J in range(H.shape[0]):
                for I in range(H.shape[1]):
                    if not site[J, I] or (I & 1) + 2 * (J & 1) != c:
                        continue
                    nb = [d for d in ((1, 0), (-1, 0), (0, 1), (0, -1)) if site[J, I] == 1 or d != miss]
                    vals = {H[J + dj, I + di] for di, dj in nb}
                    if len(vals) != 1:
                        continue
                    e = vals.pop()
                    if site[J, I] == 1:
                        k = sum(bit for (di, dj), bit in (((1, 1), 1), ((-1, 1), 2), ((-1, -1), 4), ((1, -1), 8))
                                if H[J + dj, I + di] == e + 1)
                        T = thr[k]
                    else:
                        k = (1 if H[J + d0[1], I + d0[0]] == e + 1 else 0) | (2 if H[J + d1[1], I + d1[0]] == e + 1
                                                                              else 0)
                        T = thr_free[k]
                    u = oracle.site_uniform(9, J + oy, (I + ox) >> 1, t, c)
                    H[J, I] = e + 1 if u < T else e - 1
    ch.sweep(2)
    assert (ch.H.astype(np.int64) == H).all()
