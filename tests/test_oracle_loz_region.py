"""Pins for the oracle's lozenge tilings of general domains (Section 1.1
domains on the triangular lattice of Section 1.2).

* hexagons: the extremes equal the empty and full boxes, and the chain on the
  hexagon's triangle mask equals the hexagon oracle bit for bit;
* a brute-force enumerator of lozenge tilings (MacMahon's formula on
  hexagons) decides tileability of random domains and gives, through the
  heights of every tiling, the pointwise extremes;
* rotations from either extreme reach every tiling, the chain follows the
  q^volume law on a partial hexagon (chi-square), and coupling from the past
  coalesces from every state.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue
from test_oracle_cftp import run_from

I32MIN = np.iinfo(np.int32).min


def macmahon(a, b, c):
    p = Fraction(1)
    for i in range(1, a + 1):
        for j in range(1, b + 1):
            for k in range(1, c + 1):
                p *= Fraction(i + j + k - 1, i + j + k - 2)
    return int(p)


def nbrs(x, y, t):
    if t == 0:
        return ((x, y, 1), (x, y - 1, 1), (x + 1, y, 1))
    return ((x, y, 0), (x, y + 1, 0), (x - 1, y, 0))


def enumerate_tilings(mask):
    """Every lozenge tiling (a perfect matching of edge-adjacent triangles),
    by exhaustive search over the first unmatched triangle."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape[:2]
    tris = [(x, y, t) for y in range(h) for x in range(w) for t in (0, 1) if m[y, x, t]]
    inside = set(tris)
    partner = {}
    out = []

    def rec(i):
        while i < len(tris) and tris[i] in partner:
            i += 1
        if i == len(tris):
            out.append(dict(partner))
            return
        a = tris[i]
        for b in nbrs(*a):
            if b in inside and b not in partner:
                partner[a], partner[b] = b, a
                rec(i + 1)
                del partner[a], partner[b]

    rec(0)
    return out


def steps(X, Y):
    return (((X + 1, Y), (X, Y, 0), (X, Y - 1, 1)), ((X, Y + 1), (X - 1, Y, 0), (X, Y, 1)),
            ((X + 1, Y + 1), (X, Y, 1), (X, Y, 0)), ((X - 1, Y), (X - 1, Y - 1, 1), (X - 1, Y, 0)),
            ((X, Y - 1), (X, Y - 1, 1), (X - 1, Y - 1, 0)), ((X - 1, Y - 1), (X - 1, Y - 1, 0), (X - 1, Y - 1, 1)))


def tiling_heights(mask, partner):
    """H of a tiling relative to its lowest, then leftmost, vertex, from
    Thurston's rule: along an edge with a lower-right triangle on the left
    h' = 3H + X + Y rises by 1, or falls by 2 if a lozenge covers the edge;
    with an upper-left triangle on the left the signs flip."""
    m = np.asarray(mask, dtype=bool)
    h, w = m.shape[:2]
    inside = lambda t: 0 <= t[0] < w and 0 <= t[1] < h and m[t[1], t[0], t[2]]
    pts, _ = oracle.loz_points(m)
    start = next((X, Y) for Y in range(h + 1) for X in range(w + 1) if pts[Y, X])
    hp = {start: start[0] + start[1]}
    stack = [start]
    while stack:
        u = stack.pop()
        for v, left, right in steps(*u):
            if not (inside(left) or inside(right)):
                continue
            covered = inside(left) and inside(right) and partner.get(left) == right
            d = 1 if left[2] == 0 else -1
            hv = hp[u] + (-2 * d if covered else d)
            if v in hp:
                assert hp[v] == hv, "inconsistent heights"
            else:
                hp[v] = hv
                stack.append(v)
    H = np.full((h + 1, w + 1), I32MIN, dtype=np.int64)
    for (X, Y), x in hp.items():
        H[Y, X] = (x - X - Y) // 3
    H[pts] -= H[start[1], start[0]]
    return H


def thr_q(q, metro=False):
    return oracle.table_from_ratios(oracle.lozenge_ratios(q), metro)


@pytest.mark.parametrize("abc", [(1, 1, 1), (2, 3, 2), (3, 2, 4), (6, 5, 4)])
def test_hexagon_extremes_are_the_boxes(abc):
    m = oracle.hexagon_mask(*abc)
    Hmax, Hmin = oracle.loz_extremal_heights(m)
    assert (Hmin == oracle.LozengeOracle(*abc, [0, 0]).export()).all()
    assert (Hmax == oracle.LozengeOracle(*abc, [0, 0], init="max").export()).all()


@pytest.mark.parametrize("q,metro,random", [(Fraction(1, 2), False, False), (Fraction(1), True, False),
                                            (Fraction(3, 2), False, True)])
def test_hexagon_chain_equals_the_hexagon_oracle(q, metro, random):
    abc = (5, 6, 4)
    m = oracle.hexagon_mask(*abc)
    for init in ("min", "max"):
        a = oracle.LozengeRegionOracle(m, thr_q(q, metro), metropolis=metro, seed=3, init=init,
                                       random_colours=random)
        b = oracle.LozengeOracle(*abc, thr_q(q, metro), metropolis=metro, seed=3, init=init,
                                 random_colours=random)
        for k in (1, 3, 7):
            a.sweep(k)
            b.sweep(k)
            assert (a.export() == b.export()).all()


@pytest.mark.parametrize("abc", [(1, 1, 1), (2, 2, 2), (2, 3, 2), (3, 3, 2), (3, 3, 3)])
def test_enumerator_matches_macmahon(abc):
    assert len(enumerate_tilings(oracle.hexagon_mask(*abc))) == macmahon(*abc)


def random_tri_domain(rng, w, h, fill):
    while True:
        m = np.zeros((h, w, 2), dtype=bool)
        m[rng.integers(h), rng.integers(w), rng.integers(2)] = True
        target = max(2, int(fill * 2 * w * h))
        for _ in range(60 * w * h):
            if m.sum() >= target:
                break
            ys, xs, ts = np.nonzero(m)
            k = rng.integers(len(xs))
            x, y, t = nbrs(xs[k], ys[k], ts[k])[rng.integers(3)]
            if 0 <= x < w and 0 <= y < h and not m[y, x, t]:
                m[y, x, t] = True
                try:
                    oracle.check_loz_region(m)
                except ValueError:
                    m[y, x, t] = False
        try:
            oracle.check_loz_region(m)
            return m
        except ValueError:
            continue


def check_against_enumeration(m):
    tilings = enumerate_tilings(m)
    if not tilings:
        with pytest.raises(oracle.Untileable):
            oracle.loz_extremal_heights(m)
        return 0
    Hmax, Hmin = oracle.loz_extremal_heights(m)
    pts, _ = oracle.loz_points(m)
    hs = np.stack([tiling_heights(m, p) for p in tilings])
    # compare up to the common constant (both are heights of tilings of m)
    Y0, X0 = np.argwhere(pts)[0]
    off = Hmin[Y0, X0]
    assert (hs.max(axis=0)[pts] + off == Hmax[pts]).all()
    assert (hs.min(axis=0)[pts] + off == Hmin[pts]).all()
    keys = {np.where(pts, h_ + off, I32MIN).tobytes() for h_ in hs}
    for init in ("min", "max"):
        ch = oracle.LozengeRegionOracle(m, thr_q(1), init=init)
        get = lambda: ch.H.copy()

        def put(s):
            ch.H[:] = s

        seen = bfs(ch, get, put, lambda: ch.export().astype(np.int64).tobytes())
        assert set(seen) == keys
    return len(tilings)


@pytest.mark.parametrize("seed", range(12))
def test_random_domains_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    m = random_tri_domain(rng, 3 + seed % 2, 3, 0.7)
    check_against_enumeration(m)


def test_partial_hexagons():
    found = 0
    for abc in ((2, 2, 2), (3, 2, 2), (2, 3, 3)):
        m = oracle.hexagon_mask(*abc)
        h, w = m.shape[:2]
        for cut in range(1, 4):
            mm = m.copy()
            mm[h - cut:, w - cut:, :] = False     # a corner cut off
            try:
                oracle.check_loz_region(mm)
            except ValueError:
                continue
            found += check_against_enumeration(mm) > 0
    assert found > 0


def test_untileable_domains_are_refused():
    with pytest.raises(oracle.Untileable):
        m = np.zeros((1, 1, 2), dtype=bool)
        m[0, 0, 0] = True                          # a single triangle
        oracle.loz_extremal_heights(m)
    m = np.zeros((2, 2, 2), dtype=bool)
    m[0, 0, :] = True
    m[1, 0, 0] = True                              # three triangles in a row
    with pytest.raises(oracle.Untileable):
        oracle.loz_extremal_heights(m)


def test_law_on_a_partial_hexagon():
    q = Fraction(1, 2)
    m = oracle.hexagon_mask(2, 2, 2)
    m[3, 3, :] = False
    tilings = enumerate_tilings(m)
    Hmax, Hmin = oracle.loz_extremal_heights(m)
    pts, _ = oracle.loz_points(m)
    Y0, X0 = np.argwhere(pts)[0]
    w = {}
    for p in tilings:
        H = tiling_heights(m, p) + Hmin[Y0, X0]
        H[~pts] = I32MIN
        w[H.tobytes()] = q ** int((H - Hmin)[pts].sum())
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.LozengeRegionOracle(m, thr_q(q), seed=17)

    class View:
        def sweep(self, n):
            ch.sweep(n)

        def export(self):
            return ch.export().astype(np.int64)

    assert chi_square_pvalue(View(), probs, 8000, 4) > 1e-3


def test_cftp_on_a_partial_hexagon():
    m = oracle.hexagon_mask(2, 2, 2)
    m[3, 3, :] = False
    states = []
    Hmax, Hmin = oracle.loz_extremal_heights(m)
    pts, _ = oracle.loz_points(m)
    Y0, X0 = np.argwhere(pts)[0]
    for p in enumerate_tilings(m):
        H = tiling_heights(m, p) + Hmin[Y0, X0]
        H[~pts] = I32MIN
        states.append(H)
    for seed in range(4):
        make = lambda init, s=seed: oracle.LozengeRegionOracle(m, thr_q(Fraction(1, 3)), seed=s, init=init)
        R, sample = oracle.cftp(make)
        for st in states:
            assert np.array_equal(run_from(make, st, R), sample)


def test_observables_on_a_domain():
    m = oracle.hexagon_mask(4, 5, 3)
    m[-2:, -3:, :] = False
    ch = oracle.LozengeRegionOracle(m, thr_q(Fraction(2, 3)), seed=2, obs_every=2, bin_=3)
    ch.sweep(9)
    v, bs = ch.observe()
    pts, _ = oracle.loz_points(m)
    assert v == int((ch.export().astype(np.int64) - ch.Hmin)[pts].sum()) and bs.sum() == v
    assert int(ch.samples[0]) == 4
