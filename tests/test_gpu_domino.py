"""GPU parity for the domino sampler: the HIP path against the oracle, bit for
bit on the canonical export and the integer observables (Aztec diamonds)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say, vertical_brick_faces

pytestmark = pytest.mark.gpu


def thr_uniform(metro=False):
    return oracle.table_from_ratios(oracle.domino_ratios(), metro)


def thr_two(a, b, metro=False):
    return oracle.table_from_ratios(oracle.domino_ratios("two", a, b), metro)


def gpu_sampler(tl, n, seed, kind="uniform", a=1.0, b=1.0, metro=False, init=0, obs_every=0, obs_bin=1, **kw):
    w = tl.weights(tl.TL_W_UNIFORM) if kind == "uniform" else tl.weights(tl.TL_W_TWO_PERIODIC, a, b)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return tl.Sampler(tl.domain(tl.TL_DOMINO, n=n, init=init), w, seed,
                      tl.options(obs_every=obs_every, obs_bin=obs_bin, **kw))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 8, 31, 32, 33, 65, 130, 257])
def test_uniform_parity_small(n):
    tl = need_gpu()
    say("domino uniform parity n=%d" % n)
    s = gpu_sampler(tl, n, seed=1234 + n)
    o = oracle.DominoOracle(n, thr_uniform(), seed=1234 + n)
    assert (s.export() == o.export()).all()
    for steps in (1, 2, 9):
        s.sweep(steps)
        o.sweep(steps)
        assert (s.export() == o.export()).all(), "n=%d after %d sweeps" % (n, o.t)


@pytest.mark.parametrize("metro", [False, True])
@pytest.mark.parametrize("n", [5, 40, 133])
def test_two_periodic_parity(n, metro):
    tl = need_gpu()
    say("domino two-periodic parity n=%d metro=%s" % (n, metro))
    s = gpu_sampler(tl, n, seed=77, kind="two", a=1.0, b=0.5, metro=metro)
    o = oracle.DominoOracle(n, thr_two(1, oracle.Fraction(1, 2), metro), metropolis=metro, seed=77)
    assert s.thresholds() == list(o.thr)
    s.sweep(15)
    o.sweep(15)
    assert (s.export() == o.export()).all()


def test_uniform_metropolis_parity():
    tl = need_gpu()
    s = gpu_sampler(tl, 50, seed=5, metro=True)
    o = oracle.DominoOracle(50, thr_uniform(True), metropolis=True, seed=5)
    s.sweep(12)
    o.sweep(12)
    assert (s.export() == o.export()).all()


def test_config1_aztec64_1000_sweeps_with_face_density():
    # Aztec n=64, uniform, brick start, 1000 sweeps, seed 1, per-face
    # horizontal counts sampled after every sweep.
    tl = need_gpu()
    say("domino config n=64 1000 sweeps")
    s = gpu_sampler(tl, 64, seed=1, obs_every=1, obs_bin=1)
    o = oracle.DominoOracle(64, thr_uniform(), seed=1, obs_every=1, bin_=1)
    s.sweep(1000)
    o.sweep(1000)
    assert (s.export() == o.export()).all()
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 1000
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert obs["scalar_sum"] == int(o.scalar_sum[0])
    v, _ = o.observe(1)
    assert obs["scalar_now"] == v
    dens = oracle.bin_density(o.bin_sum, int(o.samples[0]), o.in_domain_cells(), 1)
    assert np.allclose(obs["bin_density"], dens, rtol=1e-12, atol=0)
    assert s.hash() == oracle.canonical_hash(o.export())


def test_binned_density_and_ragged_bins():
    tl = need_gpu()
    n, B = 45, 16   # 90 x 90 faces -> 6 x 6 bins, last ones ragged
    s = gpu_sampler(tl, n, seed=9, obs_every=3, obs_bin=B)
    o = oracle.DominoOracle(n, thr_uniform(), seed=9, obs_every=3, bin_=B)
    s.sweep(31)
    o.sweep(31)
    obs = s.observables()
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    dens = oracle.bin_density(o.bin_sum, int(o.samples[0]), o.in_domain_cells(), B)
    assert np.allclose(obs["bin_density"], dens, rtol=1e-6, atol=0)
    s2 = gpu_sampler(tl, n, seed=9, obs_every=3, obs_bin=5)
    o2 = oracle.DominoOracle(n, thr_uniform(), seed=9, obs_every=3, bin_=5)
    s2.sweep(7)
    o2.sweep(7)
    assert (s2.observables()["bin_sum"].reshape(-1) == o2.bin_sum).all()


@pytest.mark.parametrize("n,B", [(300, 32), (300, 64), (130, 48), (257, 100), (70, 200)])
def test_large_bins(n, B):
    # bins of 32 faces or more (runs of an owner word counted at once)
    tl = need_gpu()
    s = gpu_sampler(tl, n, seed=13, obs_every=2, obs_bin=B)
    o = oracle.DominoOracle(n, thr_uniform(), seed=13, obs_every=2, bin_=B)
    s.sweep(9)
    o.sweep(9)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 4
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()


def test_init_max_and_import_resume():
    tl = need_gpu()
    n = 37
    s = gpu_sampler(tl, n, seed=3, init=tl.TL_INIT_MAX)
    vb = vertical_brick_faces(n)
    assert (s.export() == vb).all()
    o = oracle.DominoOracle(n, thr_uniform(), seed=3)
    o.load(vb)
    s.sweep(11)
    o.sweep(11)
    assert (s.export() == o.export()).all()
    # resume: export at t=11, import into a fresh sampler, continue
    mid = s.export()
    s.sweep(6)
    r = gpu_sampler(tl, n, seed=3)
    r.import_(mid, 11)
    r.sweep(6)
    assert (r.export() == s.export()).all()
    # split sweeps
    a = gpu_sampler(tl, n, seed=3)
    a.sweep(4)
    a.sweep(13)
    b = gpu_sampler(tl, n, seed=3)
    b.sweep(17)
    assert (a.export() == b.export()).all()


def test_import_rejects_invalid():
    tl = need_gpu()
    s = gpu_sampler(tl, 6, seed=1)
    bad = s.export().copy()
    bad[5, 5] = 0 if bad[5, 5] != 0 else 1
    with pytest.raises(tl.TlError) as e:
        s.import_(bad, 0)
    assert e.value.status == tl.TL_EINVAL


def test_full_size_order_2048_one_sweep_sampled():
    # The large plain-path workload at its full size, in the launch
    # configuration bench.py times (order 2048, seed 7, the full 10^4 sweeps
    # with density samples every 100 sweeps): the final state is a valid tiling
    # (host-validated import), and the oracle, started from it, takes sweep
    # 10^4 exactly as the GPU does.
    tl = need_gpu()
    say("domino order 2048, 10^4 sweeps + one-sweep parity")
    n = 2048
    s = gpu_sampler(tl, n, seed=7, obs_every=100, obs_bin=64)
    brick = s.export()
    s.sweep(10000)
    mid = s.export()
    obs = s.observables()
    assert obs["samples"] == 100
    inside = (mid != 255)
    assert obs["scalar_now"] == int(((mid == 2) | (mid == 3)).sum())
    o = oracle.DominoOracle(n, thr_uniform(), seed=7)
    o.load(mid)   # raises unless mid is a domino tiling of the diamond
    o.t = 10000
    s.sweep(1)
    o.sweep(1)
    assert (s.export() == o.export()).all()
    assert s.hash() == oracle.canonical_hash(o.export())
    # the chain has moved away from the brick start, and is still moving: each
    # flip rewrites the partners of four cells
    assert (mid != brick)[inside].mean() > 0.01
    assert (s.export() != mid)[inside].mean() > 0.01


def test_maximum_order_valid_tiling():
    # the largest order the library accepts: a few sweeps, then the export must
    # pass the host's tiling validation on import
    tl = need_gpu()
    n = 16384
    say("domino order %d" % n)
    s = gpu_sampler(tl, n, seed=1)
    s.sweep(20)
    f = s.export()
    r = gpu_sampler(tl, n, seed=1, kernel=1)
    r.import_(f, 20)
    assert r.hash() == s.hash()
    with pytest.raises(tl.TlError):
        gpu_sampler(tl, n + 1, seed=1)


@pytest.mark.parametrize("n,tile_rows,spl", [(100, 8, 3), (257, 16, 5), (700, 32, 8), (700, 24, 130), (333, 40, 1)])
def test_tiled_kernel_parity(n, tile_rows, spl):
    # multi-tile launches with row and column halos, several sweeps per launch:
    # two full launches and a partial one (spl = 130 is cut to the 128 steps
    # one halo group covers, and reaches that limit)
    tl = need_gpu()
    sweeps = max(13, 2 * spl + 1)
    say("domino tiled parity n=%d tile_rows=%d sweeps_per_launch=%d, %d sweeps" % (n, tile_rows, spl, sweeps))
    s = gpu_sampler(tl, n, seed=21, kernel=2, tile_rows=tile_rows, sweeps_per_launch=spl)
    o = oracle.DominoOracle(n, thr_uniform(), seed=21)
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


@pytest.mark.parametrize("n,order,kind,sweeps", [(700, 0, "uniform", 60), (1100, 0, "uniform", 52),
                                                 (700, 1, "uniform", 40), (600, 0, "two", 53),
                                                 (600, 1, "two", 35)])
def test_default_tile_plan_parity(n, order, kind, sweeps):
    # the automatic tile plans the benchmark uses (32 rows x 4 groups x 25
    # sweeps; 64 rows x 2 groups x 16 sweeps under the random colour order),
    # over several full launches and a partial one, against the oracle
    tl = need_gpu()
    say("domino default plan n=%d order=%d %s, %d sweeps" % (n, order, kind, sweeps))
    s = gpu_sampler(tl, n, seed=41, kind=kind, a=1.0, b=0.5, colour_order=order)
    thr = thr_uniform() if kind == "uniform" else thr_two(1, Fraction(1, 2))
    o = oracle.DominoOracle(n, thr, seed=41, random_colours=order == 1)
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()


@pytest.mark.parametrize("groups", [1, 2])
def test_random_order_tallest_tiles(groups):
    # under the random colour order the tallest accepted tile leaves room for
    # two halo rows per sweep: the tile heights just below the row limit of a
    # work-group (1024 threads / (groups + 2 halo groups) rows) run and agree
    tl = need_gpu()
    n = 1500
    max_rows = 1024 // (groups + 2)
    o = oracle.DominoOracle(n, thr_uniform(), seed=43, random_colours=True)
    o.sweep(7)
    for rows in (max_rows - 4, max_rows - 3, max_rows - 2, max_rows):
        say("domino random order n=%d tile_rows=%d groups=%d" % (n, rows, groups))
        s = gpu_sampler(tl, n, seed=43, kernel=2, tile_rows=rows, tile_groups=groups, colour_order=1)
        s.sweep(7)
        assert (s.export() == o.export()).all(), rows
        s.destroy()


@pytest.mark.parametrize("n,rows,groups,spl,order,kind,metro,sweeps", [
    (1, 0, 0, 0, 0, "uniform", False, 5),          # a single row
    (2, 0, 0, 0, 0, "uniform", False, 9),
    (60, 0, 0, 0, 0, "uniform", False, 21),        # one tile, no halo
    (64, 0, 0, 0, 0, "two", False, 21),            # one tile of exactly 64 rows
    (100, 16, 0, 5, 0, "uniform", False, 13),      # one group per row, row halo only
    (257, 20, 1, 7, 0, "uniform", False, 22),      # three groups, one per tile: column halos
    (700, 32, 4, 16, 0, "uniform", False, 40),     # the default shape
    (700, 48, 4, 8, 0, "uniform", False, 19),
    (700, 24, 2, 8, 1, "uniform", False, 30),      # random colour order: two halo rows per sweep
    (600, 0, 0, 0, 0, "two", False, 40),           # bit-serial decisions
    (600, 0, 0, 0, 1, "two", False, 25),
    (333, 30, 3, 9, 0, "two", True, 31),           # lazy Metropolis
    (2048, 32, 14, 16, 0, "uniform", False, 17),   # 16 wavefronts per tile
])
def test_register_tile_parity(n, rows, groups, spl, order, kind, metro, sweeps):
    # register-resident tiles (kernel 3) against the oracle: several full
    # launches and a partial one, row and column halos, both colour orders,
    # one-bit and bit-serial decisions
    tl = need_gpu()
    say("domino register tiles n=%d rows=%d groups=%d spl=%d order=%d %s metro=%d, %d sweeps"
        % (n, rows, groups, spl, order, kind, metro, sweeps))
    s = gpu_sampler(tl, n, seed=51, kind=kind, a=1.0, b=0.5, metro=metro, kernel=3, tile_rows=rows,
                    tile_groups=groups, sweeps_per_launch=spl, colour_order=order)
    thr = thr_uniform(metro) if kind == "uniform" else thr_two(1, Fraction(1, 2), metro)
    o = oracle.DominoOracle(n, thr, metropolis=metro, seed=51, random_colours=order == 1)
    s.sweep(sweeps)
    o.sweep(sweeps)
    assert (s.export() == o.export()).all()
    s.destroy()


def test_register_tiles_equal_lds_tiles_order_2048():
    tl = need_gpu()
    say("domino order 2048 register tiles vs LDS tiles, 300 sweeps")
    a = gpu_sampler(tl, 2048, seed=7, kernel=2)
    b = gpu_sampler(tl, 2048, seed=7, kernel=3)
    a.sweep(300)
    b.sweep(300)
    assert a.hash() == b.hash()


@pytest.mark.parametrize("n", [9, 130, 700])
def test_streaming_kernel_parity(n):
    tl = need_gpu()
    s = gpu_sampler(tl, n, seed=4, kernel=1)
    o = oracle.DominoOracle(n, thr_uniform(), seed=4)
    s.sweep(10)
    o.sweep(10)
    assert (s.export() == o.export()).all()


@pytest.mark.parametrize("n,B,every", [(300, 1, 3), (300, 5, 20), (300, 16, 7), (257, 7, 40), (300, 64, 17)])
def test_observables_of_register_tile_launches(n, B, every):
    # samples taken between register-tile launches (bins in LDS when they
    # fit, global ones otherwise; runs of a word for bins of 32 faces or more,
    # single dominoes below): the same sums as the oracle and as the LDS tiles
    tl = need_gpu()
    say("register-tile observables n=%d B=%d every=%d" % (n, B, every))
    s = gpu_sampler(tl, n, seed=29, obs_every=every, obs_bin=B)
    l = gpu_sampler(tl, n, seed=29, obs_every=every, obs_bin=B, kernel=2)
    o = oracle.DominoOracle(n, thr_uniform(), seed=29, obs_every=every, bin_=B)
    for k in (every + 1, 2 * every):
        s.sweep(k)
        l.sweep(k)
        o.sweep(k)
    a, b = s.observables(), l.observables()
    assert a["samples"] == b["samples"] == int(o.samples[0]) == (3 * every + 1) // every
    assert (a["bin_sum"].reshape(-1) == o.bin_sum).all()
    assert (b["bin_sum"] == a["bin_sum"]).all()
    assert s.hash() == l.hash()


def test_streaming_equals_tiled_order_2048():
    tl = need_gpu()
    say("domino order 2048 streaming vs tiled")
    a = gpu_sampler(tl, 2048, seed=7, kernel=1)
    b = gpu_sampler(tl, 2048, seed=7, kernel=2)
    a.sweep(300)
    b.sweep(300)
    assert a.hash() == b.hash()
    assert (a.export() == b.export()).all()


def test_reset_and_timing():
    tl = need_gpu()
    s = gpu_sampler(tl, 300, seed=2, obs_every=5, obs_bin=64)
    s.set_timing(True)
    s.sweep(20)
    h1 = s.hash()
    o1 = s.observables()
    ms, launches, steps, bpc = s.kernel_time()
    assert launches > 0 and steps == 40 and ms > 0 and bpc == 300 * 300
    s.reset(2)
    s.sweep(20)
    assert s.hash() == h1
    o2 = s.observables()
    assert (o1["bin_sum"] == o2["bin_sum"]).all() and o2["samples"] == 4


@pytest.mark.parametrize("n,q,metro,kw", [(9, (Fraction(5, 4), Fraction(2, 3)), False, {}),
                                          (40, (Fraction(20), Fraction(1, 20)), False, {}),
                                          (150, (Fraction(5, 4), Fraction(2, 3)), True, {}),
                                          (300, (Fraction(20), Fraction(1, 20)), False,
                                           {"tile_rows": 16, "sweeps_per_launch": 7})])
def test_volume_weights_parity(n, q, metro, kw):
    # volume weights q on black and q' on white vertices (the paper's Aztec
    # example uses 20 and 1/20)
    tl = need_gpu()
    say("domino volume weights n=%d q=%s metro=%s" % (n, q, metro))
    w = tl.weights(tl.TL_W_VOLUME_BW, q[0].numerator, q[0].denominator, q[1].numerator, q[1].denominator)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=n), w, 31, tl.options(**kw))
    thr = oracle.table_from_ratios(oracle.domino_ratios("volume", *q), metro)
    o = oracle.DominoOracle(n, thr, metropolis=metro, seed=31)
    assert s.thresholds() == list(o.thr)
    s.sweep(17)
    o.sweep(17)
    assert (s.export() == o.export()).all()
