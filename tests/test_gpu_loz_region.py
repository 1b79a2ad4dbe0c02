"""GPU parity for lozenge tilings of domains given by triangle masks (Section
1.1 domains on the triangular lattice of Section 1.2: partial hexagons, the
paper's weird region): the HIP path against the oracle's chain, bit for bit,
and the hexagon's own mask against the hexagon sampler."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say
from test_oracle_loz_region import random_tri_domain

pytestmark = pytest.mark.gpu

KERNELS = {"auto": {}, "step": {"kernel": 1}, "tiled": {"kernel": 2, "tile_rows": 8, "sweeps_per_launch": 3}}


def weights(tl, q, metro=False):
    w = tl.weights(tl.TL_W_VOLUME, q.numerator, q.denominator)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return w, oracle.table_from_ratios(oracle.lozenge_ratios(q), metro)


def lozenge_triangles(H, x, y):
    """The two triangles of the lozenge that covers triangle (x, y, 0) in the
    tiling with heights H: its partner is across the edge where the heights
    along (1,0) then (0,1) step by (0, 0) (the diagonal), (-1, 0) (the bottom)
    or (0, -1) (the right side)."""
    d1, d2 = H[y, x + 1] - H[y, x], H[y + 1, x + 1] - H[y, x + 1]
    other = {(0, 0): (x, y, 1), (-1, 0): (x, y - 1, 1), (0, -1): (x + 1, y, 1)}[(int(d1), int(d2))]
    return (x, y, 0), other


def weird(n, seed=0):
    """A partial hexagon that is tileable by construction: the lozenges of a
    tiling of the n x n x n hexagon (after a few sweeps from the empty box)
    that lie outside two discs bitten from its boundary."""
    o = oracle.LozengeOracle(n, n, n, oracle.table_from_ratios(oracle.lozenge_ratios(1), False), seed=seed)
    o.sweep(5)
    H = o.export().astype(np.int64)
    m0 = oracle.hexagon_mask(n, n, n)
    h, w = m0.shape[:2]
    centres = [(w * 0.8, h * 0.9, n * 0.45), (w * 0.95, h * 0.45, n * 0.3)]
    m = np.zeros_like(m0)
    for y, x in zip(*np.nonzero(m0[:, :, 0])):
        a, b = lozenge_triangles(H, x, y)
        cx = (a[0] + b[0]) / 2.0 + 0.5
        cy = (a[1] + b[1]) / 2.0 + 0.5
        if all((cx - px) ** 2 + (cy - py) ** 2 > r * r for px, py, r in centres):
            m[a[1], a[0], a[2]] = m[b[1], b[0], b[2]] = True
    oracle.check_loz_region(m)
    return m


def tileable_random(seed):
    rng = np.random.default_rng(seed)
    while True:
        m = random_tri_domain(rng, 20, 16, 0.85)
        try:
            oracle.loz_extremal_heights(m)
            return m
        except oracle.Untileable:
            continue


@pytest.mark.parametrize("abc,q,kernel,order", [((20, 18, 16), Fraction(1999, 2000), "auto", 0),
                                                ((40, 50, 45), Fraction(2, 3), "tiled", 0),
                                                ((20, 18, 16), Fraction(1, 2), "step", 1),
                                                ((140, 130, 120), Fraction(1), "auto", 0)])
def test_hexagon_mask_equals_hexagon(abc, q, kernel, order):
    tl = need_gpu()
    say("lozenge hexagon mask %s q=%s %s order=%d" % (abc, q, kernel, order))
    w, _ = weights(tl, q)
    m = oracle.hexagon_mask(*abc)
    for init in (tl.TL_INIT_MIN, tl.TL_INIT_MAX):
        opt = tl.options(colour_order=order, obs_every=2, obs_bin=7, **KERNELS[kernel])
        a = tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=m, init=init), w, 5, opt)
        b = tl.Sampler(tl.domain(tl.TL_LOZENGE, a=abc[0], b=abc[1], c=abc[2], init=init), w, 5, opt)
        for k in (0, 3, 8):
            a.sweep(k)
            b.sweep(k)
            assert (a.export() == b.export()).all()
        oa, ob = a.observables(), b.observables()
        assert (oa["bin_sum"] == ob["bin_sum"]).all() and oa["scalar_now"] == ob["scalar_now"]
        assert np.allclose(oa["bin_density"], ob["bin_density"], rtol=1e-12, atol=0)


CASES = [("weird30", Fraction(1999, 2000), False, "min", "auto"), ("weird30", Fraction(1), True, "max", "step"),
         ("weird60", Fraction(2, 3), False, "max", "tiled"), ("random", Fraction(1, 2), False, "min", "auto"),
         ("weird150", Fraction(1), False, "min", "auto")]


def mask_of(name):
    return {"weird30": weird(30), "weird60": weird(60), "weird150": weird(150),
            "random": tileable_random(1)}[name]


@pytest.mark.parametrize("name,q,metro,init,kernel", CASES, ids=["-".join(map(str, c)) for c in CASES])
def test_domain_parity(name, q, metro, init, kernel):
    tl = need_gpu()
    say("lozenge domain parity %s q=%s metro=%s init=%s %s" % (name, q, metro, init, kernel))
    m = mask_of(name)
    w, thr = weights(tl, q, metro)
    dom = tl.domain(tl.TL_LOZENGE, mask=m, init=tl.TL_INIT_MAX if init == "max" else tl.TL_INIT_MIN)
    s = tl.Sampler(dom, w, 23, tl.options(**KERNELS[kernel]))
    o = oracle.LozengeRegionOracle(m, thr, metropolis=metro, seed=23, init=init)
    assert (s.rows, s.row_bytes // 4) == (m.shape[0] + 1, m.shape[1] + 1)
    assert (s.export() == o.export()).all()
    for k in (1, 4, 12):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all(), "after %d sweeps" % o.t
    assert s.hash() == oracle.canonical_hash(o.export())
    assert s.info() == (len(o.sites()), 3)


def test_domain_random_order():
    tl = need_gpu()
    m = weird(30)
    w, thr = weights(tl, Fraction(1, 2))
    s = tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=m), w, 4, tl.options(colour_order=1))
    o = oracle.LozengeRegionOracle(m, thr, seed=4, random_colours=True)
    for k in (2, 9):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all()


@pytest.mark.parametrize("name,B", [("weird30", 1), ("weird30", 7), ("weird60", 40), ("random", 3)])
def test_domain_observables(name, B):
    tl = need_gpu()
    m = mask_of(name)
    w, thr = weights(tl, Fraction(2, 3))
    s = tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=m), w, 6, tl.options(obs_every=3, obs_bin=B))
    o = oracle.LozengeRegionOracle(m, thr, seed=6, obs_every=3, bin_=B)
    s.sweep(20)
    o.sweep(20)
    obs = s.observables()
    assert obs["samples"] == int(o.samples[0]) == 6
    assert (obs["bin_sum"].reshape(-1) == o.bin_sum).all()
    v, now = o.observe(B)
    assert obs["scalar_now"] == v and (obs["bin_now"].reshape(-1) == now).all()
    dens = oracle.bin_density(o.bin_sum, int(o.samples[0]), o.in_domain_cells(), B)
    assert np.allclose(obs["bin_density"], dens, rtol=1e-12, atol=0)


def test_domain_import_export_and_rejects():
    tl = need_gpu()
    m = weird(24)
    w, thr = weights(tl, Fraction(1))
    s = tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=m), w, 8)
    o = oracle.LozengeRegionOracle(m, thr, seed=8)
    o.sweep(25)
    mid = o.export()
    s.import_(mid, 25)
    s.sweep(6)
    o.sweep(6)
    assert (s.export() == o.export()).all()
    pts, sites = oracle.loz_points(m)
    Y, X = np.argwhere(sites)[len(np.argwhere(sites)) // 2]
    bad = mid.copy()
    bad[Y, X] += 3                                   # steps out of {0, -1}
    with pytest.raises(tl.TlError) as e:
        s.import_(bad, 0)
    assert e.value.status == tl.TL_EINVAL
    bad = mid.copy()
    Yb, Xb = np.argwhere(pts & ~sites)[0]
    bad[Yb, Xb] += 1                                 # a boundary height
    with pytest.raises(tl.TlError) as e:
        s.import_(bad, 0)
    assert e.value.status == tl.TL_EINVAL


def test_domain_create_errors():
    tl = need_gpu()
    w = tl.weights(tl.TL_W_UNIFORM)
    one = np.zeros((2, 2, 2), dtype=bool)
    one[0, 0, 0] = True
    with pytest.raises(tl.TlError) as e:
        tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=one), w, 1)
    assert e.value.status == tl.TL_EUNTILEABLE
    ring = np.ones((5, 5, 2), dtype=bool)
    ring[2, 2, :] = False
    with pytest.raises(tl.TlError) as e:
        tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=ring), w, 1)
    assert e.value.status == tl.TL_EINVAL


@pytest.mark.parametrize("name,q", [("weird12", Fraction(1, 2)), ("weird18", Fraction(1)),
                                    ("random", Fraction(3, 2))])
def test_domain_cftp_equals_oracle(name, q):
    tl = need_gpu()
    say("lozenge domain cftp %s q=%s" % (name, q))
    m = {"weird12": weird(12), "weird18": weird(18), "random": tileable_random(1)}[name]
    w, thr = weights(tl, q)
    for seed in (3, 4):
        s = tl.Sampler(tl.domain(tl.TL_LOZENGE, mask=m), w, seed)
        info = s.cftp(24)
        make = lambda init, sd=seed: oracle.LozengeRegionOracle(m, thr, seed=sd, init=init)
        R, sample = oracle.cftp(make, max_log2=24)
        assert info["log2_sweeps"] == R
        assert (s.export() == sample).all()
