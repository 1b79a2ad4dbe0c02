"""GPU parity for domino tilings of general domains given by masks (Section
1.1): the HIP path against the oracle's chain on the same embedding, bit for
bit on the canonical export, the observables and coupling from the past."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say
from test_oracle_region import l_shape, ones, random_domain

pytestmark = pytest.mark.gpu


def tileable_random(seed, w, h, fill):
    rng = np.random.default_rng(seed)
    while True:
        m = random_domain(rng, w, h, fill)
        try:
            oracle.extremal_heights(m, 0)
            return m
        except oracle.Untileable:
            continue


def mask_of(name):
    if name == "square8":
        return ones(8, 8)
    if name == "rect30x50":
        return ones(30, 50)
    if name == "l40":
        return l_shape(40, 16, 20)
    if name == "random40":
        return tileable_random(7, 40, 36, 0.7)
    if name == "aztec20":
        return oracle.DominoOracle(20, [0] * 4).in_domain_cells()
    if name == "square130":
        return ones(130, 130)
    if name == "ragged67x200":
        return ones(67, 200)
    if name == "strip2x300":
        return ones(2, 300)
    raise KeyError(name)


def weights_of(tl, kind, metro):
    if kind == "uniform":
        w, R = tl.weights(tl.TL_W_UNIFORM), oracle.domino_ratios()
    elif kind == "two":
        w, R = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5), oracle.domino_ratios("two", 1, Fraction(1, 2))
    else:
        w = tl.weights(tl.TL_W_VOLUME_BW, 5.0, 4.0, 2.0, 3.0)
        R = oracle.domino_ratios("volume", Fraction(5, 4), Fraction(2, 3))
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return w, oracle.table_from_ratios(R, metro)


def pair(tl, m, seed, kind="uniform", metro=False, init="min", obs_every=0, obs_bin=1, **kw):
    w, thr = weights_of(tl, kind, metro)
    dom = tl.domain(tl.TL_DOMINO, mask=m, init=tl.TL_INIT_MAX if init == "max" else tl.TL_INIT_MIN)
    s = tl.Sampler(dom, w, seed, tl.options(obs_every=obs_every, obs_bin=obs_bin, **kw))
    o = oracle.DominoRegionOracle(m, thr, metropolis=metro, seed=seed, init=init, obs_every=obs_every,
                                  bin_=obs_bin)
    assert s.thresholds() == list(o.thr)
    return s, o


CASES = [("square8", "uniform", False, "min", {}), ("square8", "uniform", False, "max", {}),
         ("rect30x50", "uniform", False, "min", {}), ("rect30x50", "two", True, "max", {}),
         ("l40", "uniform", False, "max", {}), ("l40", "volume", False, "min", {"kernel": 1}),
         ("random40", "uniform", False, "min", {}), ("random40", "two", False, "max", {"kernel": 1}),
         ("aztec20", "uniform", False, "max", {}), ("square130", "uniform", False, "min", {}),
         ("square130", "volume", True, "max", {"kernel": 2, "tile_rows": 8, "sweeps_per_launch": 3}),
         ("ragged67x200", "uniform", False, "min", {"kernel": 2, "tile_rows": 16, "sweeps_per_launch": 5}),
         ("strip2x300", "uniform", False, "min", {})]


@pytest.mark.parametrize("name,kind,metro,init,opts", CASES, ids=["-".join(map(str, c[:4])) for c in CASES])
def test_domain_parity(name, kind, metro, init, opts):
    tl = need_gpu()
    say("domain parity %s %s metro=%s init=%s %s" % (name, kind, metro, init, opts))
    m = mask_of(name)
    s, o = pair(tl, m, 41, kind, metro, init, **opts)
    assert (s.rows, s.row_bytes) == m.shape
    assert (s.export() == o.export()).all()
    for steps in (1, 4, 12):
        s.sweep(steps)
        o.sweep(steps)
        assert (s.export() == o.export()).all(), "after %d sweeps" % o.t
    assert s.hash() == oracle.canonical_hash(o.export())
    sites, colours = s.info()
    assert sites == len(o.sites()) and colours == 2


@pytest.mark.parametrize("name,B", [("l40", 1), ("l40", 7), ("rect30x50", 40), ("square130", 32),
                                    ("random40", 64)])
def test_domain_observables(name, B):
    tl = need_gpu()
    m = mask_of(name)
    s, o = pair(tl, m, 5, obs_every=3, obs_bin=B)
    s.sweep(20)
    o.sweep(20)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 6
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_sum"] == int(o.scalar_sum[0])
    v, now = o.observe(B)
    assert obs["scalar_now"] == v and (obs["bin_now"].reshape(-1) == now).all()
    dens = oracle.bin_density(o.bin_sum, int(o.samples[0]), m, B)
    assert np.allclose(obs["bin_density"], dens, rtol=1e-12, atol=0)


def test_domain_import_export_and_rejects():
    tl = need_gpu()
    m = l_shape(24, 10, 6)
    s, o = pair(tl, m, 9)
    o.sweep(30)
    mid = o.export()
    s.import_(mid, 30)
    s.sweep(7)
    o.sweep(7)
    assert (s.export() == o.export()).all()
    bad = mid.copy()
    bad[m.shape[0] - 1, m.shape[1] - 1] = 2          # a face outside the domain
    with pytest.raises(tl.TlError) as e:
        s.import_(bad, 0)
    assert e.value.status == tl.TL_EINVAL
    bad = mid.copy()
    ys, xs = np.nonzero(m)
    bad[ys[0], xs[0]] = 255                           # a face of the domain left uncovered
    with pytest.raises(tl.TlError) as e:
        s.import_(bad, 0)
    assert e.value.status == tl.TL_EINVAL
    # reset returns to the extremal start
    s.reset(9)
    assert (s.export() == oracle.DominoRegionOracle(m, [0] * 4).tmin).all()


def test_domain_create_errors():
    tl = need_gpu()
    w = tl.weights(tl.TL_W_UNIFORM)
    board = ones(8, 8)
    board[0, 0] = board[7, 7] = False
    with pytest.raises(tl.TlError) as e:
        tl.Sampler(tl.domain(tl.TL_DOMINO, mask=board), w, 1)
    assert e.value.status == tl.TL_EUNTILEABLE
    ring = ones(5, 5)
    ring[2, 2] = False
    with pytest.raises(tl.TlError) as e:
        tl.Sampler(tl.domain(tl.TL_DOMINO, mask=ring), w, 1)
    assert e.value.status == tl.TL_EINVAL
    with pytest.raises(ValueError):      # lozenge masks select triangles: (h, w, 2)
        tl.domain(tl.TL_LOZENGE, mask=ones(4, 4))


def test_batch_and_server_mask_refusals():
    """Batches hold domino chains only; a server refuses what a sampler refuses."""
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Batch, Server
    w = tl.weights(tl.TL_W_UNIFORM)
    with pytest.raises(tl.TlError) as e:
        Batch([tl.domain(tl.TL_SIXVERTEX, mask=ones(4, 4))], tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 1.0), [1])
    assert e.value.status == tl.TL_EINVAL
    board = ones(8, 8)
    board[0, 0] = board[7, 7] = False
    sv = Server(1 << 26, 4)
    try:
        with pytest.raises(tl.TlError) as e:
            sv.submit(tl.domain(tl.TL_DOMINO, mask=board), w, 1, 10)
        assert e.value.status == tl.TL_EUNTILEABLE
    finally:
        sv.destroy()


CFTP_CASES = [("square8", "uniform"), ("l12", "uniform"), ("rect10x14", "two"), ("random16", "volume")]


@pytest.mark.parametrize("name,kind", CFTP_CASES, ids=["%s-%s" % c for c in CFTP_CASES])
def test_domain_cftp_equals_oracle(name, kind):
    tl = need_gpu()
    say("domain cftp %s %s" % (name, kind))
    m = {"square8": ones(8, 8), "l12": l_shape(12, 6, 4), "rect10x14": ones(10, 14),
         "random16": tileable_random(3, 16, 16, 0.75)}[name]
    w, thr = weights_of(tl, kind, False)
    for seed in (3, 4):
        s = tl.Sampler(tl.domain(tl.TL_DOMINO, mask=m), w, seed)
        info = s.cftp(24)
        make = lambda init, sd=seed: oracle.DominoRegionOracle(m, thr, seed=sd, init=init)
        R, sample = oracle.cftp(make, max_log2=24)
        assert info["log2_sweeps"] == R
        assert (s.export() == sample).all()
        o = make("min")
        o.load(sample)
        o.t = 1 << R
        s.sweep(3)
        o.sweep(3)
        assert (s.export() == o.export()).all()


def test_large_square_one_sweep_sampled():
    # a 2000 x 2000 square: 300 sweeps on the GPU, then the oracle, started
    # from that state (validated on load), takes the next sweep as the GPU does
    tl = need_gpu()
    say("domain square 2000, 300 sweeps + one-sweep parity")
    m = ones(2000, 2000)
    w, thr = weights_of(tl, "uniform", False)
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, mask=m), w, 11)
    start = s.export()
    s.sweep(300)
    mid = s.export()
    o = oracle.DominoRegionOracle(m, thr, seed=11, init=None)
    o.load(start)       # raises unless the start is a tiling of the square
    o.load(mid)
    o.t = 300
    s.sweep(1)
    o.sweep(1)
    assert (s.export() == o.export()).all()
    # from an extreme of a square only a few blocks can rotate at first, so
    # the chain spreads from them: some faces have changed, not most
    assert (mid != start).any() and (s.export() != mid).any()
