"""GPU coupling from the past against the oracle's: the same round R, the same
exact sample bit for bit, and the same continuation afterwards."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def case(tl, kind, size, weights):
    if kind == "domino":
        dom = tl.domain(tl.TL_DOMINO, n=size)
        if weights == "uniform":
            w, thr = tl.weights(tl.TL_W_UNIFORM), oracle.table_from_ratios(oracle.domino_ratios(), False)
        elif weights == "volume":
            w = tl.weights(tl.TL_W_VOLUME_BW, 5.0, 4.0, 2.0, 3.0)
            thr = oracle.table_from_ratios(oracle.domino_ratios("volume", Fraction(5, 4), Fraction(2, 3)), False)
        else:
            w = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)
            thr = oracle.table_from_ratios(oracle.domino_ratios("two", 1, Fraction(1, 2)), False)
        make = lambda seed: (lambda init: oracle.DominoOracle(size, thr, seed=seed, init=init))
    elif kind == "lozenge":
        dom = tl.domain(tl.TL_LOZENGE, a=size[0], b=size[1], c=size[2])
        q = weights
        w = tl.weights(tl.TL_W_VOLUME, q.numerator, q.denominator)
        thr = oracle.table_from_ratios(oracle.lozenge_ratios(q), False)
        make = lambda seed: (lambda init: oracle.LozengeOracle(*size, thr, seed=seed, init=init))
    elif len(weights) == 6:
        dom = tl.domain(tl.TL_SIXVERTEX, n=size)
        w = tl.weights(tl.TL_W_SIXVERTEX6, *[float(x) for x in weights])
        thr = oracle.table_from_ratios(oracle.sixv_ratios6(*weights), False)
        make = lambda seed: (lambda init: oracle.SixVertexOracle(size, thr, seed=seed, init=init))
    else:
        dom = tl.domain(tl.TL_SIXVERTEX, n=size)
        a2, b2, c2 = weights
        w = tl.weights(tl.TL_W_SIXVERTEX, float(a2), float(b2), float(c2))
        thr = oracle.table_from_ratios(oracle.sixv_ratios(int(round(a2 ** 0.5)), int(round(b2 ** 0.5)), c2), False)
        make = lambda seed: (lambda init: oracle.SixVertexOracle(size, thr, seed=seed, init=init))
    return dom, w, make


CASES = [("domino", 1, "uniform", {}), ("domino", 2, "uniform", {}), ("domino", 7, "uniform", {}),
         ("domino", 24, "two", {}), ("domino", 32, "uniform", {"tile_rows": 8, "sweeps_per_launch": 5}),
         ("domino", 12, "volume", {}),
         ("lozenge", (3, 4, 5), Fraction(1, 2), {}), ("lozenge", (12, 10, 8), Fraction(1999, 2000), {}),
         ("lozenge", (30, 30, 30), Fraction(1), {"tile_rows": 16, "sweeps_per_launch": 3}),
         ("sixv", 5, (1, 1, 1), {}), ("sixv", 16, (1, 1, 2), {}),
         ("sixv", 48, (1, 1, 1), {"tile_rows": 16, "sweeps_per_launch": 4}),
         ("sixv", 40, (1, 1, 4), {"tile_rows": 12, "sweeps_per_launch": 2}),
         ("sixv", 20, (1, 2, 1, 1, 4, 4), {})]


@pytest.mark.parametrize("kind,size,weights,opts", CASES, ids=["%s-%s-%s" % c[:3] for c in CASES])
def test_cftp_equals_oracle(kind, size, weights, opts):
    tl = need_gpu()
    say("cftp %s %s %s %s" % (kind, size, weights, opts))
    dom, w, make = case(tl, kind, size, weights)
    for seed in (3, 4):
        s = tl.Sampler(dom, w, seed, tl.options(**opts))
        info = s.cftp(24)
        R, sample = oracle.cftp(make(seed), max_log2=24)
        assert info["log2_sweeps"] == R and info["sweeps"] == 1 << R
        assert info["total_sweeps"] == sum(2 << r for r in range(1, R + 1))
        assert (s.export() == sample).all()
        # later sweeps use the counters after 2^R
        o = make(seed)("min")
        o.load(sample)
        o.t = 1 << R
        s.sweep(3)
        o.sweep(3)
        assert (s.export() == o.export()).all()
        assert s.observables()["sweeps"] == (1 << R) + 3


def test_cftp_not_met_leaves_the_minimal_chain():
    tl = need_gpu()
    dom, w, make = case(tl, "domino", 30, "uniform")
    s = tl.Sampler(dom, w, 9)
    with pytest.raises(tl.TlError) as e:
        s.cftp(2)
    assert e.value.status == tl.TL_EBUSY
    o = make(9)("min")
    for t0, count in oracle.cftp_segments(2):
        o.t = t0
        o.sweep(count)
    assert (s.export() == o.export()).all()


def test_cftp_rejects_non_monotone_settings():
    tl = need_gpu()
    metro = tl.weights(tl.TL_W_UNIFORM)
    metro.rule = tl.TL_METROPOLIS
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=4), metro, 1)
    with pytest.raises(tl.TlError) as e:
        s.cftp(10)
    assert e.value.status == tl.TL_EINVAL
    s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=6), tl.weights(tl.TL_W_SIXVERTEX, 4.0, 1.0, 1.0), 1)
    with pytest.raises(tl.TlError) as e:
        s.cftp(10)
    assert e.value.status == tl.TL_EINVAL
    # six weights that do not keep the order (a2 > c2)
    s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=6), tl.weights(tl.TL_W_SIXVERTEX6, 1.0, 5.0, 1.0, 1.0, 1.0, 1.0), 1)
    with pytest.raises(tl.TlError) as e:
        s.cftp(10)
    assert e.value.status == tl.TL_EINVAL
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=4), tl.weights(tl.TL_W_UNIFORM), 1)
    for bad in (0, 32):
        with pytest.raises(tl.TlError) as e:
            s.cftp(bad)
        assert e.value.status == tl.TL_EINVAL


@pytest.mark.parametrize("model", ["domino", "sixv", "lozenge"])
def test_rounds_side_by_side_equal_rounds_in_turn(model):
    # One-tile states run consecutive rounds side by side; a tile option
    # forces the rounds one after the other: R, the sample and the reported
    # sweeps must agree.
    tl = need_gpu()
    say("cftp side by side vs in turn: %s" % model)
    if model == "domino":
        dom, w = tl.domain(tl.TL_DOMINO, n=20), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)
    elif model == "sixv":
        dom, w = tl.domain(tl.TL_SIXVERTEX, n=24), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)
    else:
        dom, w = tl.domain(tl.TL_LOZENGE, a=8, b=9, c=7), tl.weights(tl.TL_W_VOLUME, 2.0, 3.0)
    for seed in (11, 12, 13):
        a = tl.Sampler(dom, w, seed)
        b = tl.Sampler(dom, w, seed, tl.options(kernel=2, sweeps_per_launch=64))
        ia, ib = a.cftp(24), b.cftp(24)
        assert ia == ib
        assert (a.export() == b.export()).all()
        a.sweep(3)
        b.sweep(3)
        assert (a.export() == b.export()).all()       # both continue from counter 2^R
