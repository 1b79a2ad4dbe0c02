"""Pins for the oracle's coupling from the past (Section 1.1.4; the CFTP host
function of Section 2.2).

* the sweep counters of every time step are the same in every round;
* brute force on tiny domains: started from EVERY state (enumerated by single
  flips), the chain driven by the same draws from time -2^R reaches the state
  CFTP returns -- which holds only if the moves are monotone and the two
  starting states are the extremes (negative control: six-vertex weights with
  a > c, where the order is not preserved, Section 1.2.4);
* the CFTP output over many seeds follows the exact stationary law
  (chi-square against enumerated weights).
"""
import math
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle_helpers import bfs
import test_oracle_domino as tod
import test_oracle_sixvertex as tos


def domino_make(n, thr, seed):
    return lambda init: oracle.DominoOracle(n, thr, seed=seed, init=init)


def lozenge_make(abc, thr, seed):
    return lambda init: oracle.LozengeOracle(*abc, thr, seed=seed, init=init)


def sixv_make(N, thr, seed):
    return lambda init: oracle.SixVertexOracle(N, thr, seed=seed, init=init)


def all_exports(ch, arrays):
    """Exports of every state reachable from the chain's state by single flips
    (arrays: the chain's state arrays, restored around each flip)."""
    get = lambda: tuple(a.copy() for a in arrays)

    def put(s):
        for a, v in zip(arrays, s):
            a[:] = v

    seen = bfs(ch, get, put, lambda: ch.export().tobytes())
    out = []
    for s in seen.values():
        put(s)
        out.append(ch.export())
    return out


def run_from(make, state, R):
    ch = make("min")
    ch.load(state)
    for t0, count in oracle.cftp_segments(R):
        ch.t = t0
        ch.sweep(count)
    return ch.export()


def test_segments_fix_the_draws_of_each_time_step():
    def counters(R):
        out = []
        for t0, count in oracle.cftp_segments(R):
            out.extend(range(t0, t0 + count))
        return out   # counter of times -2^R, ..., -1
    for R in range(1, 14):
        c = counters(R)
        assert sorted(c) == list(range(1 << R))
        # the last 2^(R-1) time steps of round R are the whole of round R-1
        if R > 1:
            assert c[-(1 << (R - 1)):] == counters(R - 1)
        # time tau in [-2^r, -2^(r-1)) -> counter tau + 3 * 2^(r-1)
        for i, t in enumerate(c):
            tau = i - (1 << R)
            if tau == -1:
                assert t == 0
            else:
                r = (-tau - 1).bit_length()
                assert -(1 << r) <= tau < -(1 << (r - 1)) and t == tau + 3 * (1 << (r - 1))


CASES = [
    ("aztec2-uniform", lambda s: domino_make(2, tod.uniform_thr(), s), "domino", 2),
    ("aztec3-uniform", lambda s: domino_make(3, tod.uniform_thr(), s), "domino", 3),
    ("aztec3-two", lambda s: domino_make(3, tod.two_periodic_thr(1, Fraction(1, 2)), s), "domino", 3),
    ("hex222-q", lambda s: lozenge_make((2, 2, 2), oracle.table_from_ratios(oracle.lozenge_ratios(Fraction(1, 3)),
                                                                            False), s), "lozenge", (2, 2, 2)),
    ("hex232-uniform", lambda s: lozenge_make((2, 3, 2), oracle.table_from_ratios(oracle.lozenge_ratios(1), False),
                                              s), "lozenge", (2, 3, 2)),
    ("dwbc4-uniform", lambda s: sixv_make(4, tos.thr(1, 1, 1), s), "sixv", 4),
    ("dwbc5-sqrt2", lambda s: sixv_make(5, tos.thr(1, 1, 2), s), "sixv", 5),
]


def states_of(kind, size, make):
    ch = make("min")
    if kind == "domino":
        return all_exports(ch, [ch.Tb, ch.Tw])
    if kind == "lozenge":
        return all_exports(ch, [ch.Hs])
    return all_exports(ch, [ch.h])


@pytest.mark.parametrize("name,factory,kind,size", CASES, ids=[c[0] for c in CASES])
def test_every_state_coalesces_to_the_cftp_output(name, factory, kind, size):
    states = states_of(kind, size, factory(0))
    assert len(states) > 1
    for seed in range(4):
        make = factory(seed)
        R, sample = oracle.cftp(make)
        for st in states:
            assert np.array_equal(run_from(make, st, R), sample), (name, seed)


def test_non_monotone_weights_break_coalescence():
    # a = 2 > c = 1: the top and bottom chains can meet while other states
    # have not (Section 1.2.4: the order is preserved only for a, b <= c)
    thr = tos.thr(2, 1, 1)
    states = None
    broken = 0
    for seed in range(40):
        make = sixv_make(4, thr, seed)
        if states is None:
            states = states_of("sixv", 4, make)
        R, sample = oracle.cftp(make)
        broken += any(not np.array_equal(run_from(make, st, R), sample) for st in states)
    assert broken > 0


def chi_square_of_samples(samples, probs):
    counts = Counter(s.tobytes() for s in samples)
    assert set(counts) <= set(probs)
    keys = list(probs)
    obs = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    exp = np.array([probs[k] for k in keys], dtype=np.float64) * len(samples)
    return float(stats.chi2.sf(float(((obs - exp) ** 2 / exp).sum()), len(keys) - 1))


def test_cftp_law_aztec_two_periodic():
    a, b = Fraction(1), Fraction(1, 2)
    faces = tod.enumerate_tilings(3)
    w = {k: tod.two_periodic_weight(f, 3, a, b) for k, f in faces.items()}
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    thr = tod.two_periodic_thr(a, b)
    samples = [oracle.cftp(domino_make(3, thr, s))[1] for s in range(6000)]
    assert chi_square_of_samples(samples, probs) > 1e-3


def test_cftp_law_hexagon_q_volume():
    q = Fraction(1, 3)
    thr = oracle.table_from_ratios(oracle.lozenge_ratios(q), False)
    make0 = lozenge_make((2, 2, 2), thr, 0)
    states = states_of("lozenge", (2, 2, 2), make0)
    probe = make0("min")
    w = {}
    for st in states:
        probe.load(st)
        w[st.tobytes()] = q ** probe.observe(1)[0]
    Z = sum(w.values())
    probs = {k: float(v / Z) for k, v in w.items()}
    samples = [oracle.cftp(lozenge_make((2, 2, 2), thr, s))[1] for s in range(4000)]
    assert chi_square_of_samples(samples, probs) > 1e-3


def test_cftp_law_dwbc_sqrt2():
    states = tos.enumerate_states(4)
    w2 = {k: tos.vertex_weight_product(h, Fraction(1), Fraction(1), Fraction(2)) for k, h in states.items()}
    w = {k: math.sqrt(v) for k, v in w2.items()}
    Z = sum(w.values())
    probs = {k: v / Z for k, v in w.items()}
    thr = tos.thr(1, 1, 2)
    samples = [oracle.cftp(sixv_make(4, thr, s))[1] for s in range(4000)]
    assert chi_square_of_samples(samples, probs) > 1e-3
