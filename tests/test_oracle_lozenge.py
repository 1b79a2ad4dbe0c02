"""Pins for the lozenge oracle (a x b x c hexagon).

* Section 1.2 (lozenge tilings are connected by rotations at triangular
  vertices): breadth-first search through the oracle's rotation primitive from
  the empty box reaches exactly MacMahon's number of boxed plane partitions, and
  the volume generating function equals MacMahon's q-product.
* Section 1.1.1 volume weights: visit frequencies match q^volume / Z.
* Section 1.1.4 monotone coupling: chains from the maximal and minimal tilings on
  the same draws stay ordered.
* Proper 3-colouring (Section 1.2): the visiting order inside a colour class does
  not change the result.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle_helpers import bfs, chi_square_pvalue


def macmahon(a, b, c):
    p = Fraction(1)
    for i in range(1, a + 1):
        for j in range(1, b + 1):
            for k in range(1, c + 1):
                p *= Fraction(i + j + k - 1, i + j + k - 2)
    return p


def q_macmahon(a, b, c, q):
    p = Fraction(1)
    for i in range(1, a + 1):
        for j in range(1, b + 1):
            for k in range(1, c + 1):
                p *= (1 - q ** (i + j + k - 1)) / (1 - q ** (i + j + k - 2))
    return p


def thr(q, metropolis=False):
    return oracle.table_from_ratios(oracle.lozenge_ratios(q), metropolis)


def enumerate_states(a, b, c):
    ch = oracle.LozengeOracle(a, b, c, thr(1))
    get = lambda: ch.Hs.copy()

    def put(s):
        ch.Hs[:] = s

    seen = bfs(ch, get, put, lambda: ch.export().tobytes())
    vols = {}
    for k, s in seen.items():
        put(s)
        vols[k] = ch.observe(1)[0]
    return vols


@pytest.mark.parametrize("abc", [(1, 1, 1), (1, 2, 3), (2, 2, 2), (2, 3, 3), (3, 3, 3)])
def test_bfs_count_is_macmahon(abc):
    vols = enumerate_states(*abc)
    assert len(vols) == macmahon(*abc)
    q = Fraction(1, 3)
    assert sum(q ** v for v in vols.values()) == q_macmahon(*abc, q)


def test_extremes_and_site_count():
    a = b = c = 5
    lo = oracle.LozengeOracle(a, b, c, thr(1))
    hi = oracle.LozengeOracle(a, b, c, thr(1), init="max")
    assert lo.observe(1)[0] == 0
    assert hi.observe(1)[0] == a * b * c
    assert len(lo.sites()) == 3 * a * a - 3 * a + 1
    assert int(lo.in_domain_cells().sum()) == 3 * a * a + 3 * a + 1


@pytest.mark.parametrize("metropolis", [False, True])
@pytest.mark.parametrize("q", [Fraction(1), Fraction(1, 2)])
def test_stationary_q_volume(q, metropolis):
    vols = enumerate_states(2, 2, 2)
    w = {k: q ** v for k, v in vols.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.LozengeOracle(2, 2, 2, thr(q, metropolis), metropolis=metropolis, seed=31)
    assert chi_square_pvalue(ch, probs, 12000, 8) > 1e-3


def test_wrong_q_detected():
    vols = enumerate_states(2, 2, 2)
    q = Fraction(1, 2)
    w = {k: (1 / q) ** v for k, v in vols.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.LozengeOracle(2, 2, 2, thr(q), seed=31)
    assert chi_square_pvalue(ch, probs, 12000, 8) < 1e-6


def test_monotone_coupling():
    a, b, c = 4, 5, 6
    t = thr(Fraction(3, 4))
    top = oracle.LozengeOracle(a, b, c, t, seed=77, init="max")
    bot = oracle.LozengeOracle(a, b, c, t, seed=77, init="min")
    inside = top.in_domain_cells()
    for _ in range(60):
        top.sweep(1)
        bot.sweep(1)
        assert (top.export()[inside] >= bot.export()[inside]).all()
    top.sweep(3000)
    bot.sweep(3000)
    assert (top.export() == bot.export()).all()   # coalesced


def test_order_independence_and_resume():
    t = thr(Fraction(1999, 2000))
    a = oracle.LozengeOracle(6, 7, 5, t, seed=11)
    a.sweep(25)
    oracle.set_reverse_order(True)
    try:
        b = oracle.LozengeOracle(6, 7, 5, t, seed=11)
        b.sweep(10)
        b.sweep(15)
    finally:
        oracle.set_reverse_order(False)
    assert (a.export() == b.export()).all()


def test_valid_heights_after_sweeps():
    ch = oracle.LozengeOracle(5, 6, 7, thr(Fraction(1, 2)), seed=3)
    ch.sweep(40)
    H = ch.export().astype(np.int64)
    inside = ch.in_domain_cells()
    for dy, dx in ((0, 1), (1, 0), (1, 1)):
        a = H[:H.shape[0] - dy, :H.shape[1] - dx]
        b = H[dy:, dx:]
        m = inside[:H.shape[0] - dy, :H.shape[1] - dx] & inside[dy:, dx:]
        d = (b - a)[m]
        assert set(np.unique(d)) <= {0, -1}
