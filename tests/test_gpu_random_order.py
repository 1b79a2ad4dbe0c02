"""GPU parity under the random colour order (Section 2.2's RandomWalk draws the
colour of every step): every kernel form of the three models against the
oracle's chains with random colours, bit for bit, and coupling from the past."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say
from test_oracle_region import l_shape

pytestmark = pytest.mark.gpu

KERNELS = {"auto": {}, "step": {"kernel": 1}, "tiled": {"kernel": 2, "tile_rows": 8, "sweeps_per_launch": 3}}


def domino_pair(tl, n, seed, kind, metro, **kw):
    if kind == "uniform":
        w, R = tl.weights(tl.TL_W_UNIFORM), oracle.domino_ratios()
    else:
        w, R = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5), oracle.domino_ratios("two", 1, Fraction(1, 2))
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=n), w, seed, tl.options(colour_order=1, **kw))
    o = oracle.DominoOracle(n, oracle.table_from_ratios(R, metro), metropolis=metro, seed=seed, random_colours=True)
    return s, o


def run_both(s, o, steps=(1, 4, 9)):
    assert (s.export() == o.export()).all()
    for k in steps:
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all(), "after %d sweeps" % o.t


DOMINO = [(7, "uniform", False, "auto"), (40, "two", False, "auto"), (40, "uniform", True, "step"),
          (130, "uniform", False, "tiled"), (300, "two", False, "auto"), (300, "uniform", False, "step"),
          (257, "two", True, "tiled")]


@pytest.mark.parametrize("n,kind,metro,kernel", DOMINO, ids=["-".join(map(str, c)) for c in DOMINO])
def test_domino_random_order(n, kind, metro, kernel):
    tl = need_gpu()
    say("random order domino n=%d %s metro=%s %s" % (n, kind, metro, kernel))
    s, o = domino_pair(tl, n, 17, kind, metro, **KERNELS[kernel])
    run_both(s, o)


LOZ = [((3, 4, 5), Fraction(1, 2), "auto"), ((20, 18, 16), Fraction(1999, 2000), "auto"),
       ((20, 18, 16), Fraction(1), "step"), ((40, 50, 45), Fraction(2, 3), "tiled")]


@pytest.mark.parametrize("abc,q,kernel", LOZ, ids=["%s-%s-%s" % c for c in LOZ])
def test_lozenge_random_order(abc, q, kernel):
    tl = need_gpu()
    say("random order lozenge %s q=%s %s" % (abc, q, kernel))
    w = tl.weights(tl.TL_W_VOLUME, q.numerator, q.denominator)
    s = tl.Sampler(tl.domain(tl.TL_LOZENGE, a=abc[0], b=abc[1], c=abc[2]), w, 5,
                   tl.options(colour_order=1, **KERNELS[kernel]))
    o = oracle.LozengeOracle(*abc, oracle.table_from_ratios(oracle.lozenge_ratios(q), False), seed=5,
                             random_colours=True)
    run_both(s, o)


SIXV = [(5, (1, 1, 1), "auto"), (40, (1, 1, 2), "auto"), (40, (1, 1, 1), "step"), (100, (1, 1, 2), "tiled"),
        (64, (4, 1, 4), "tiled")]


@pytest.mark.parametrize("N,w2,kernel", SIXV, ids=["%s-%s-%s" % c for c in SIXV])
def test_sixvertex_random_order(N, w2, kernel):
    tl = need_gpu()
    say("random order six-vertex N=%d %s %s" % (N, w2, kernel))
    w = tl.weights(tl.TL_W_SIXVERTEX, *[float(x) for x in w2])
    s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=N), w, 8, tl.options(colour_order=1, **KERNELS[kernel]))
    a = int(round(w2[0] ** 0.5))
    b = int(round(w2[1] ** 0.5))
    o = oracle.SixVertexOracle(N, oracle.table_from_ratios(oracle.sixv_ratios(a, b, w2[2]), False), seed=8,
                               random_colours=True)
    run_both(s, o)


def test_domain_random_order():
    tl = need_gpu()
    m = l_shape(40, 16, 20)
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, mask=m), tl.weights(tl.TL_W_UNIFORM), 3, tl.options(colour_order=1))
    o = oracle.DominoRegionOracle(m, thr, seed=3, random_colours=True)
    run_both(s, o)


def test_split_sweeps_and_large_order():
    tl = need_gpu()
    say("random order: split sweeps, order 2048 tiled vs one launch per step")
    a = tl.Sampler(tl.domain(tl.TL_DOMINO, n=2048), tl.weights(tl.TL_W_UNIFORM), 7, tl.options(colour_order=1))
    b = tl.Sampler(tl.domain(tl.TL_DOMINO, n=2048), tl.weights(tl.TL_W_UNIFORM), 7,
                   tl.options(colour_order=1, kernel=1))
    a.sweep(23)
    a.sweep(37)
    b.sweep(60)
    assert a.hash() == b.hash()
    mid = a.export()
    o = oracle.DominoOracle(2048, oracle.table_from_ratios(oracle.domino_ratios(), False), seed=7,
                            random_colours=True)
    o.load(mid)
    o.t = 60
    a.sweep(1)
    o.sweep(1)
    assert (a.export() == o.export()).all()
    # the fixed order gives another chain
    c = tl.Sampler(tl.domain(tl.TL_DOMINO, n=2048), tl.weights(tl.TL_W_UNIFORM), 7)
    c.sweep(60)
    assert c.hash() != b.hash()


CFTP = [("domino", 12), ("lozenge", (6, 5, 4)), ("sixv", 16)]


@pytest.mark.parametrize("kind,size", CFTP, ids=[c[0] for c in CFTP])
def test_cftp_random_order(kind, size):
    tl = need_gpu()
    say("random order cftp %s %s" % (kind, size))
    if kind == "domino":
        dom, w = tl.domain(tl.TL_DOMINO, n=size), tl.weights(tl.TL_W_UNIFORM)
        thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
        make = lambda sd: (lambda init: oracle.DominoOracle(size, thr, seed=sd, init=init, random_colours=True))
    elif kind == "lozenge":
        dom, w = tl.domain(tl.TL_LOZENGE, a=size[0], b=size[1], c=size[2]), tl.weights(tl.TL_W_VOLUME, 1.0, 2.0)
        thr = oracle.table_from_ratios(oracle.lozenge_ratios(Fraction(1, 2)), False)
        make = lambda sd: (lambda init: oracle.LozengeOracle(*size, thr, seed=sd, init=init, random_colours=True))
    else:
        dom, w = tl.domain(tl.TL_SIXVERTEX, n=size), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)
        thr = oracle.table_from_ratios(oracle.sixv_ratios(1, 1, 2), False)
        make = lambda sd: (lambda init: oracle.SixVertexOracle(size, thr, seed=sd, init=init, random_colours=True))
    for seed in (1, 2):
        s = tl.Sampler(dom, w, seed, tl.options(colour_order=1))
        info = s.cftp(24)
        R, sample = oracle.cftp(make(seed), max_log2=24)
        assert info["log2_sweeps"] == R
        assert (s.export() == sample).all()


def test_random_order_limits():
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Batch, Server
    w = tl.weights(tl.TL_W_UNIFORM)
    with pytest.raises(tl.TlError) as e:
        tl.Sampler(tl.domain(tl.TL_DOMINO, n=4), w, 1, tl.options(colour_order=2))
    assert e.value.status == tl.TL_EINVAL
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=4), w, 1, tl.options(colour_order=1))
    s.import_(s.export(), (1 << 31) - 1)
    s.sweep(1)                      # steps up to 2^32 - 1
    with pytest.raises(tl.TlError) as e:
        s.sweep(1)
    assert e.value.status == tl.TL_EINVAL
    with pytest.raises(tl.TlError) as e:
        s.cftp(31)
    assert e.value.status == tl.TL_EINVAL
    # batches and servers take the random order, with the same step limit
    with pytest.raises(tl.TlError) as e:
        Batch([tl.domain(tl.TL_DOMINO, n=8)], w, [1], tl.options(colour_order=2))
    assert e.value.status == tl.TL_EINVAL
    b = Batch([tl.domain(tl.TL_DOMINO, n=8)], w, [1], tl.options(colour_order=1))
    with pytest.raises(tl.TlError) as e:
        b.sweep((1 << 31) + 1)          # checked before any launch
    assert e.value.status == tl.TL_EINVAL
    b.destroy()
    with pytest.raises(tl.TlError) as e:
        Server(1 << 26, 4, tl.options(colour_order=2))
    assert e.value.status == tl.TL_EINVAL
    sv = Server(1 << 26, 4, tl.options(colour_order=1))
    with pytest.raises(tl.TlError) as e:
        sv.submit(tl.domain(tl.TL_DOMINO, n=8), w, 1, (1 << 31) + 1)
    assert e.value.status == tl.TL_EINVAL
    sv.destroy()
