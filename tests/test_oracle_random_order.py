"""Pins for the random colour order (the paper's RandomWalk of Section 2.2
picks the colour of every step at random).

* the step colours are uniform over the K colours, and consecutive pairs are
  uniform over the K^2 pairs (chi-square);
* one sweep of the C oracle equals K single colour steps rebuilt here from the
  site draws and the oracle's own flip primitive (so each step updates the
  drawn colour with the draws of its own step counter);
* the stationary laws are unchanged (chi-square against the exact laws used
  for the fixed order), and coupling from the past still coalesces from every
  state.
"""
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle_helpers import chi_square_pvalue
import test_oracle_cftp as toc
import test_oracle_domino as tod
import test_oracle_sixvertex as tos


@pytest.mark.parametrize("K", [2, 3, 4])
def test_step_colours_are_uniform_and_independent(K):
    seq = [oracle.step_colour(12345, s, K) for s in range(60000)]
    assert set(seq) == set(range(K))
    counts = np.bincount(seq, minlength=K)
    assert stats.chisquare(counts).pvalue > 1e-3
    pairs = np.bincount([K * a + b for a, b in zip(seq[:-1], seq[1:])], minlength=K * K)
    assert stats.chisquare(pairs).pvalue > 1e-3
    other = [oracle.step_colour(54321, s, K) for s in range(2000)]
    assert other != seq[:2000]


def step_by_flips(ch, sites, colour_of, rk_of, seed, step, K):
    """One uniform-weight heat-bath colour step of the drawn colour, site by
    site through the oracle's flip primitive (sites of one colour do not
    interact, so their order does not matter)."""
    c = oracle.step_colour(seed, step, K)
    for site in sites:
        if colour_of(site) != c:
            continue
        r, k = rk_of(site)
        up = oracle.site_uniform(seed, r, k, step, c) < (1 << 31)
        ch.flip(*site, up)


def test_domino_sweep_is_k_drawn_steps():
    n, seed = 5, 77
    thr = tod.uniform_thr()
    a = oracle.DominoOracle(n, thr, seed=seed, random_colours=True)
    b = oracle.DominoOracle(n, thr, seed=seed)
    sites = b.sites()
    colour_of = lambda s: (s[0] - n + s[1] - n) % 2
    rk_of = lambda s: ((s[0] - n + s[1] - n + n - 1) // 2, (s[1] - n - (s[0] - n) + n - 1) // 2)
    for t in range(6):
        a.sweep(1)
        for i in range(2):
            step_by_flips(b, sites, colour_of, rk_of, seed, 2 * t + i, 2)
        assert (a.export() == b.export()).all(), t


def test_lozenge_sweep_is_k_drawn_steps():
    abc, seed = (3, 2, 4), 5
    thr = oracle.table_from_ratios(oracle.lozenge_ratios(1), False)
    a = oracle.LozengeOracle(*abc, thr, seed=seed, random_colours=True)
    b = oracle.LozengeOracle(*abc, thr, seed=seed)
    sites = b.sites()
    for t in range(6):
        a.sweep(1)
        for i in range(3):
            step_by_flips(b, sites, lambda s: (s[0] + s[1]) % 3, lambda s: (s[1], s[0] // 3), seed, 3 * t + i, 3)
        assert (a.export() == b.export()).all(), t


def test_sixvertex_sweep_is_k_drawn_steps():
    N, seed = 6, 9
    a = oracle.SixVertexOracle(N, tos.thr(1, 1, 1), seed=seed, random_colours=True)
    b = oracle.SixVertexOracle(N, tos.thr(1, 1, 1), seed=seed)
    sites = b.sites()
    for t in range(6):
        a.sweep(1)
        for i in range(4):
            step_by_flips(b, sites, lambda s: (s[0] & 1) + 2 * (s[1] & 1), lambda s: (s[1], s[0] >> 1), seed,
                          4 * t + i, 4)
        assert (a.export() == b.export()).all(), t


def test_random_order_differs_from_fixed_and_splits():
    thr = tod.uniform_thr()
    a = oracle.DominoOracle(6, thr, seed=3, random_colours=True)
    b = oracle.DominoOracle(6, thr, seed=3)
    a.sweep(10)
    b.sweep(10)
    assert (a.export() != b.export()).any()
    c = oracle.DominoOracle(6, thr, seed=3, random_colours=True)
    c.sweep(4)
    c.sweep(6)
    assert (a.export() == c.export()).all()


def test_domino_law_with_random_order():
    probs = {k: 1.0 / 64 for k in tod.enumerate_tilings(3)}
    ch = oracle.DominoOracle(3, tod.uniform_thr(), seed=21, random_colours=True)
    assert chi_square_pvalue(ch, probs, 12000, 6) > 1e-3


def test_two_periodic_law_with_random_order():
    a, b = Fraction(1), Fraction(1, 2)
    faces = tod.enumerate_tilings(3)
    w = {k: tod.two_periodic_weight(f, 3, a, b) for k, f in faces.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.DominoOracle(3, tod.two_periodic_thr(a, b), seed=22, random_colours=True)
    assert chi_square_pvalue(ch, probs, 12000, 6) > 1e-3


def test_lozenge_law_with_random_order():
    q = Fraction(1, 3)
    thr = oracle.table_from_ratios(oracle.lozenge_ratios(q), False)
    make0 = toc.lozenge_make((2, 2, 2), thr, 0)
    states = toc.states_of("lozenge", (2, 2, 2), make0)
    probe = make0("min")
    w = {}
    for st in states:
        probe.load(st)
        w[st.tobytes()] = q ** probe.observe(1)[0]
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    ch = oracle.LozengeOracle(2, 2, 2, thr, seed=23, random_colours=True)
    assert chi_square_pvalue(ch, probs, 10000, 4) > 1e-3


def test_sixvertex_law_with_random_order():
    import math
    states = tos.enumerate_states(4)
    w2 = {k: tos.vertex_weight_product(h, Fraction(1), Fraction(1), Fraction(2)) for k, h in states.items()}
    w = {k: math.sqrt(v) for k, v in w2.items()}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    ch = oracle.SixVertexOracle(4, tos.thr(1, 1, 2), seed=24, random_colours=True)
    assert chi_square_pvalue(ch, probs, 10000, 4) > 1e-3


@pytest.mark.parametrize("kind", ["domino", "lozenge", "sixv"])
def test_cftp_with_random_order_coalesces_from_every_state(kind):
    if kind == "domino":
        factory = lambda s: (lambda init: oracle.DominoOracle(3, tod.uniform_thr(), seed=s, init=init,
                                                              random_colours=True))
        size = 3
    elif kind == "lozenge":
        thr = oracle.table_from_ratios(oracle.lozenge_ratios(Fraction(1, 3)), False)
        factory = lambda s: (lambda init: oracle.LozengeOracle(2, 2, 2, thr, seed=s, init=init,
                                                               random_colours=True))
        size = (2, 2, 2)
    else:
        factory = lambda s: (lambda init: oracle.SixVertexOracle(4, tos.thr(1, 1, 2), seed=s, init=init,
                                                                 random_colours=True))
        size = 4
    states = toc.states_of(kind, size, factory(0))
    for seed in range(4):
        make = factory(seed)
        R, sample = oracle.cftp(make)
        for st in states:
            assert np.array_equal(toc.run_from(make, st, R), sample)
