"""GPU parity for the height-function models (lozenge tilings of hexagons,
six-vertex model with domain-wall boundary): the HIP path against the oracle,
bit for bit on the canonical height export and the integer observables."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def loz_sampler(tl, a, b, c, seed, q=None, metro=False, init=0, **kw):
    w = tl.weights(tl.TL_W_UNIFORM) if q is None else tl.weights(tl.TL_W_VOLUME, q.numerator, q.denominator)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return tl.Sampler(tl.domain(tl.TL_LOZENGE, a=a, b=b, c=c, init=init), w, seed, tl.options(**kw))


def loz_oracle(a, b, c, seed, q=None, metro=False, init="min", **kw):
    thr = oracle.table_from_ratios(oracle.lozenge_ratios(q if q is not None else 1), metro)
    return oracle.LozengeOracle(a, b, c, thr, metropolis=metro, seed=seed, init=init, **kw)


def sixv_sampler(tl, N, seed, w2=None, metro=False, init=0, **kw):
    w = tl.weights(tl.TL_W_UNIFORM) if w2 is None else tl.weights(tl.TL_W_SIXVERTEX, *w2)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=N, init=init), w, seed, tl.options(**kw))


def sixv_oracle(N, seed, w2=None, metro=False, init="min", **kw):
    a2, b2, c2 = w2 if w2 is not None else (1, 1, 1)
    # the oracle takes a, b and c^2 (the squares used here are of integers)
    ratios = oracle.sixv_ratios(int(round(a2 ** 0.5)), int(round(b2 ** 0.5)), c2)
    thr = oracle.table_from_ratios(ratios, metro)
    return oracle.SixVertexOracle(N, thr, metropolis=metro, seed=seed, init=init, **kw)


@pytest.mark.parametrize("abc", [(1, 1, 1), (2, 3, 4), (5, 5, 5), (7, 3, 11), (40, 37, 45), (130, 120, 140)])
@pytest.mark.parametrize("kind", ["uniform", "q", "qmetro"])
def test_lozenge_parity(abc, kind):
    tl = need_gpu()
    say("lozenge parity %s %s" % (abc, kind))
    q = None if kind == "uniform" else Fraction(1999, 2000) if kind == "q" else Fraction(1, 2)
    metro = kind == "qmetro"
    s = loz_sampler(tl, *abc, seed=11, q=q, metro=metro)
    o = loz_oracle(*abc, seed=11, q=q, metro=metro)
    assert (s.export() == o.export()).all()
    for k in (1, 3, 8):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all(), "%s %s after %d sweeps" % (abc, kind, o.t)


@pytest.mark.parametrize("abc,tile_rows,spl,kernel,groups", [((60, 70, 80), 16, 3, 2, 0), ((130, 120, 140), 24, 5, 2, 0),
                                                              ((200, 90, 300), 32, 40, 2, 0), ((33, 44, 55), 0, 0, 1, 0),
                                                              ((150, 140, 160), 5, 3, 2, 1), ((90, 100, 80), 7, 4, 2, 2)])
def test_lozenge_tiles_and_streaming(abc, tile_rows, spl, kernel, groups):
    tl = need_gpu()
    s = loz_sampler(tl, *abc, seed=5, q=Fraction(3, 4), kernel=kernel, tile_rows=tile_rows, sweeps_per_launch=spl,
                    tile_groups=groups)
    o = loz_oracle(*abc, seed=5, q=Fraction(3, 4))
    sweeps = max(11, 2 * spl + 1)   # two full launches and a partial one
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


def test_lozenge_init_max_observables_hash_import():
    tl = need_gpu()
    a, b, c = 23, 17, 29
    s = loz_sampler(tl, a, b, c, seed=3, q=Fraction(7, 8), init=tl.TL_INIT_MAX, obs_every=2, obs_bin=8)
    o = loz_oracle(a, b, c, seed=3, q=Fraction(7, 8), init="max", obs_every=2, bin_=8)
    assert (s.export() == o.export()).all()
    s.sweep(9)
    o.sweep(9)
    assert (s.export() == o.export()).all()
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 4
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_now"] == o.observe(1)[0]
    dens = oracle.bin_density(o.bin_sum, 4, o.in_domain_cells(), 8)
    assert np.allclose(obs["bin_density"], dens, rtol=1e-12, atol=0)
    assert s.hash() == oracle.canonical_hash(o.export())
    mid = s.export()
    s.sweep(5)
    r = loz_sampler(tl, a, b, c, seed=3, q=Fraction(7, 8))
    r.import_(mid, 9)
    r.sweep(5)
    assert (r.export() == s.export()).all()
    bad = mid.copy()
    bad[10, 10] += 3
    with pytest.raises(tl.TlError):
        r.import_(bad, 0)


def test_lozenge_hexagon_1024_one_sweep_sampled():
    # The lozenge workload at full size (a = b = c = 1024, q = 1999/2000, seed
    # 11, the full 2 x 10^4 sweeps from the empty box): the oracle, started
    # from the GPU's final state, takes the next sweep exactly as the GPU does.
    tl = need_gpu()
    say("lozenge 1024^3, 2e4 sweeps + one-sweep parity")
    q = Fraction(1999, 2000)
    s = loz_sampler(tl, 1024, 1024, 1024, seed=11, q=q)
    s.sweep(20000)
    mid = s.export()
    o = loz_oracle(1024, 1024, 1024, seed=11, q=q)
    o.load(mid)
    o.t = 20000
    s.sweep(1)
    o.sweep(1)
    assert (s.export() == o.export()).all()
    assert s.hash() == oracle.canonical_hash(o.export())


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 8, 9, 33, 64, 130, 257])
@pytest.mark.parametrize("kind", ["uniform", "sqrt2", "sqrt2metro", "a2"])
def test_sixvertex_parity(N, kind):
    tl = need_gpu()
    say("six-vertex parity N=%d %s" % (N, kind))
    w2 = {"uniform": None, "sqrt2": (1, 1, 2), "sqrt2metro": (1, 1, 2), "a2": (4, 1, 4)}[kind]
    metro = kind == "sqrt2metro"
    s = sixv_sampler(tl, N, seed=17, w2=w2, metro=metro)
    o = sixv_oracle(N, seed=17, w2=w2, metro=metro)
    assert (s.export() == o.export()).all()
    for k in (1, 2, 7):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all(), "N=%d %s after %d sweeps" % (N, kind, o.t)


# Odd tile heights put tiles at odd first rows, where a six-vertex tile's
# threads start on the other row parity; tile_groups splits rows into columns.
@pytest.mark.parametrize("N,tile_rows,spl,kernel,groups,order",
                         [(100, 16, 3, 2, 0, 0), (300, 20, 6, 2, 0, 0), (513, 32, 30, 2, 0, 0), (77, 0, 0, 1, 0, 0),
                          (211, 5, 3, 2, 0, 0), (150, 7, 4, 2, 1, 0), (64, 3, 2, 2, 0, 0), (301, 9, 5, 2, 2, 0),
                          (211, 5, 3, 2, 0, 1), (150, 7, 2, 2, 1, 1)])
def test_sixvertex_tiles_and_streaming(N, tile_rows, spl, kernel, groups, order):
    tl = need_gpu()
    say("six-vertex tiles N=%d rows=%d spl=%d kernel=%d groups=%d order=%d" % (N, tile_rows, spl, kernel, groups,
                                                                             order))
    s = sixv_sampler(tl, N, seed=8, w2=(1, 1, 2), kernel=kernel, tile_rows=tile_rows, sweeps_per_launch=spl,
                     tile_groups=groups, colour_order=order)
    o = sixv_oracle(N, seed=8, w2=(1, 1, 2), random_colours=order == 1)
    sweeps = max(13, 2 * spl + 1)   # two full launches and a partial one
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


@pytest.mark.parametrize("model,size,weights,order,sweeps",
                         [("loz", 150, None, 0, 50), ("loz", 260, Fraction(1999, 2000), 0, 50),
                          ("loz", 150, None, 1, 40), ("sixv", 700, None, 0, 50), ("sixv", 700, (1, 1, 2), 0, 50),
                          ("sixv", 513, (1, 1, 2), 1, 40)])
def test_default_tile_plan_parity(model, size, weights, order, sweeps):
    # the automatic tile plans of the benchmark workloads (one-bit decisions:
    # 8-row tiles, 16 sweeps per launch; weighted: 4-row tiles, 6 sweeps),
    # multi-tile, over several launches, against the oracle
    tl = need_gpu()
    say("%s default plan size=%d weights=%s order=%d, %d sweeps" % (model, size, weights, order, sweeps))
    if model == "loz":
        s = loz_sampler(tl, size, size, size, seed=47, q=weights, colour_order=order)
        o = loz_oracle(size, size, size, seed=47, q=weights, random_colours=order == 1)
    else:
        s = sixv_sampler(tl, size, seed=47, w2=weights, colour_order=order)
        o = sixv_oracle(size, seed=47, w2=weights, random_colours=order == 1)
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


def test_sixvertex_init_max_observables_hash_import():
    tl = need_gpu()
    N = 45
    s = sixv_sampler(tl, N, seed=2, w2=(1, 1, 2), init=tl.TL_INIT_MAX, obs_every=3, obs_bin=4)
    o = sixv_oracle(N, seed=2, w2=(1, 1, 2), init="max", obs_every=3, bin_=4)
    assert (s.export() == o.export()).all()
    s.sweep(10)
    o.sweep(10)
    assert (s.export() == o.export()).all()
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 3
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_now"] == o.observe(1)[0]
    assert s.hash() == oracle.canonical_hash(o.export())
    mid = s.export()
    s.sweep(4)
    r = sixv_sampler(tl, N, seed=2, w2=(1, 1, 2))
    r.import_(mid, 10)
    r.sweep(4)
    assert (r.export() == s.export()).all()
    bad = mid.copy()
    bad[5, 5] += 2
    with pytest.raises(tl.TlError):
        r.import_(bad, 0)


@pytest.mark.parametrize("w2,metro", [((1, 1, 2), False), ((1, 1, 2), True), ((1, 1, 1), False)])
def test_sixvertex_1024_one_sweep_sampled(w2, metro):
    # The largest served request at full size (N = 1024, 2000 sweeps from
    # h_min): the oracle, started from the GPU's final state, takes sweep 2000
    # exactly as the GPU does.
    tl = need_gpu()
    say("six-vertex N=1024 %s metro=%s, 2000 sweeps + one-sweep parity" % (w2, metro))
    s = sixv_sampler(tl, 1024, seed=3, w2=w2, metro=metro)
    s.sweep(2000)
    mid = s.export()
    o = sixv_oracle(1024, seed=3, w2=w2, metro=metro)
    o.load(mid)
    o.t = 2000
    s.sweep(1)
    o.sweep(1)
    assert (s.export() == o.export()).all()
    assert s.hash() == oracle.canonical_hash(o.export())


SIX = (1, 2, Fraction(3, 2), Fraction(1, 2), 1, 3)   # a1, a2, b1, b2, c1, c2


@pytest.mark.parametrize("N,metro,kw", [(9, False, {}), (9, True, {}), (64, False, {}), (130, True, {}),
                                        (300, False, {"tile_rows": 12, "sweeps_per_launch": 5}),
                                        (77, True, {"kernel": 1})])
def test_sixvertex_six_weights_parity(N, metro, kw):
    # six distinct vertex weights: thresholds by the whole mask of diagonals
    tl = need_gpu()
    say("six-vertex six weights N=%d metro=%s %s" % (N, metro, kw))
    w = tl.weights(tl.TL_W_SIXVERTEX6, *[float(x) for x in SIX])
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=N), w, 19, tl.options(**kw))
    thr = oracle.table_from_ratios(oracle.sixv_ratios6(*SIX), metro)
    o = oracle.SixVertexOracle(N, thr, metropolis=metro, seed=19)
    assert s.thresholds() == list(o.thr)
    for k in (1, 6):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all()


@pytest.mark.parametrize("B", [1, 3, 16, 64, 100])
def test_lozenge_volume_bins(B):
    tl = need_gpu()
    a, b, c = 37, 20, 45
    s = loz_sampler(tl, a, b, c, seed=23, q=Fraction(3, 2), obs_every=3, obs_bin=B)
    o = loz_oracle(a, b, c, seed=23, q=Fraction(3, 2), obs_every=3, bin_=B)
    s.sweep(10)
    o.sweep(10)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 3
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_now"] == o.observe(1)[0]


@pytest.mark.parametrize("abc,B", [((150, 40, 170), 1), ((150, 40, 170), 7), ((150, 40, 170), 64),
                                   ((300, 64, 80), 100), ((6200, 3, 4), 64)])
def test_lozenge_volume_bins_wide_rows(abc, B):
    # rows of several 96-vertex words (the observable kernel's chunks), and a
    # row of more than 64 of them (several passes of one wavefront)
    tl = need_gpu()
    say("lozenge volume bins %s B=%d" % (abc, B))
    s = loz_sampler(tl, *abc, seed=31, q=Fraction(3, 2), obs_every=4, obs_bin=B)
    o = loz_oracle(*abc, seed=31, q=Fraction(3, 2), obs_every=4, bin_=B)
    s.sweep(12)
    o.sweep(12)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 3
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_now"] == o.observe(1)[0]


@pytest.mark.parametrize("model", ["lozenge", "sixvertex"])
def test_height_exports_of_wide_rows(model):
    # rows of more than 64 chunks (96 lozenge vertices or 64 six-vertex faces
    # each): the export kernel's wavefront takes them in several passes
    tl = need_gpu()
    say("wide-row export %s" % model)
    if model == "lozenge":
        s = loz_sampler(tl, 6200, 3, 4, seed=37, q=Fraction(3, 2))
        o = loz_oracle(6200, 3, 4, seed=37, q=Fraction(3, 2))
        sweeps = 6
    else:
        s = sixv_sampler(tl, 4160, seed=37, w2=(1, 1, 2))
        o = sixv_oracle(4160, seed=37, w2=(1, 1, 2))
        sweeps = 2
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


@pytest.mark.parametrize("N,B", [(1, 1), (2, 1), (33, 5), (130, 32), (130, 64), (77, 200), (64, 3)])
def test_sixvertex_c_vertex_bins(N, B):
    tl = need_gpu()
    s = sixv_sampler(tl, N, seed=29, w2=(1, 1, 2), obs_every=2, obs_bin=B)
    o = sixv_oracle(N, seed=29, w2=(1, 1, 2), obs_every=2, bin_=B)
    s.sweep(7)
    o.sweep(7)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 3
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_now"] == o.observe(1)[0]
