"""The library's host pre-pass for mask domains (Thurston's tileability test
and extremal tilings, Section 1.1) against the oracle's, bit for bit; no
device work is involved."""
import ctypes
import time

import numpy as np
import pytest

import oracle
import paper_1804_07250_amd as tl
from test_oracle_region import l_shape, ones, random_domain


def extremes(mask):
    return tl.domain_extremes(tl.domain(tl.TL_DOMINO, mask=mask))


def oracle_extremes(mask):
    o = oracle.DominoRegionOracle(mask, [0] * 4)
    return o.tmax, o.tmin


@pytest.mark.parametrize("seed", range(6))
def test_random_domains_match_the_oracle(seed):
    rng = np.random.default_rng(seed)
    tileable = 0
    for _ in range(60):
        w, h = int(rng.integers(1, 14)), int(rng.integers(1, 14))
        m = random_domain(rng, w, h, rng.uniform(0.4, 1.0))
        try:
            want = oracle_extremes(m)
        except oracle.Untileable:
            with pytest.raises(tl.TlError) as e:
                extremes(m)
            assert e.value.status == tl.TL_EUNTILEABLE
            continue
        got = extremes(m)
        assert (got[0] == want[0]).all() and (got[1] == want[1]).all()
        tileable += 1
    assert tileable > 5


@pytest.mark.parametrize("shape", ["square", "rect", "l", "aztec", "tall", "wide"])
def test_named_domains_match_the_oracle(shape):
    m = {"square": ones(40, 40), "rect": ones(17, 30), "l": l_shape(30, 12, 18),
         "aztec": oracle.DominoOracle(12, [0] * 4).in_domain_cells(), "tall": ones(60, 2),
         "wide": ones(1, 64)}[shape]
    got, want = extremes(m), oracle_extremes(m)
    assert (got[0] == want[0]).all() and (got[1] == want[1]).all()


def test_aztec_mask_gives_the_bricks():
    for n in (3, 4):
        d = oracle.DominoOracle(n, [0] * 4)
        horizontal = d.export()
        vertical = oracle.domino_vertical_brick(horizontal)
        tmax, tmin = extremes(d.in_domain_cells())
        assert ((tmax == vertical).all() and (tmin == horizontal).all()) == (n % 2 == 1)
        assert ((tmax == horizontal).all() and (tmin == vertical).all()) == (n % 2 == 0)


def test_rejected_domains():
    ring = ones(4, 4)
    ring[1:3, 1:3] = False
    pinch = np.array([[1, 1, 0], [1, 1, 0], [0, 0, 1]], dtype=bool)
    split = np.array([[1, 1, 0, 1, 1]], dtype=bool)
    for m in (ring, pinch, split, np.zeros((3, 3), dtype=bool)):
        with pytest.raises(tl.TlError) as e:
            extremes(m)
        assert e.value.status == tl.TL_EINVAL
    board = ones(8, 8)
    board[0, 0] = board[7, 7] = False
    for m in (board, ones(3, 5)):
        with pytest.raises(tl.TlError) as e:
            extremes(m)
        assert e.value.status == tl.TL_EUNTILEABLE
    # not a mask domain
    with pytest.raises(tl.TlError) as e:
        tl.domain_extremes(tl.domain(tl.TL_DOMINO, n=4))
    assert e.value.status == tl.TL_EINVAL


def test_box_limits():
    # w + h above 32768 is refused before the mask is read
    d = tl.domain(tl.TL_DOMINO, mask=ones(2, 2))
    d.w, d.h = 20000, 12769
    assert tl.lib().tl_domain_extremes(ctypes.byref(d), None, None, 0) == tl.TL_EINVAL
    d.w, d.h = 0, 2
    assert tl.lib().tl_domain_extremes(ctypes.byref(d), None, None, 0) == tl.TL_EINVAL
    d.w, d.h = 2, 2
    assert tl.lib().tl_domain_extremes(ctypes.byref(d), None, None, 0) == tl.TL_OK
    small = np.zeros(3, dtype=np.uint8)
    assert tl.lib().tl_domain_extremes(ctypes.byref(d), small.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                       None, 3) == tl.TL_EINVAL


def test_large_square_is_linear_time():
    m = ones(1024, 1024)
    t = time.time()
    tmax, tmin = extremes(m)
    assert time.time() - t < 20
    assert (tmax != 255).all() and (tmin != 255).all()
    # the extremes differ, and each is a tiling (partners point back)
    for f in (tmax, tmin):
        ys, xs = np.nonzero(f == 2)
        assert (f[ys, xs + 1] == 3).all()
        ys, xs = np.nonzero(f == 0)
        assert (f[ys + 1, xs] == 1).all()
    assert (tmax != tmin).any()


def sixv_extremes(mask):
    return tl.domain_extremes(tl.domain(tl.TL_SIXVERTEX, mask=mask))


@pytest.mark.parametrize("seed", range(4))
def test_sixvertex_domains_match_the_oracle(seed):
    rng = np.random.default_rng(100 + seed)
    ok = 0
    for _ in range(60):
        w, h = int(rng.integers(1, 12)), int(rng.integers(1, 12))
        m = random_domain(rng, w, h, rng.uniform(0.6, 1.0))
        try:
            want = oracle.sixv_extremal_heights(m)
        except oracle.Untileable:
            with pytest.raises(tl.TlError) as e:
                sixv_extremes(m)
            assert e.value.status == tl.TL_EUNTILEABLE
            continue
        got = sixv_extremes(m)
        assert (got[0] == want[0]).all() and (got[1] == want[1]).all()
        ok += 1
    assert ok > 2   # most random domains admit no domain-wall type configuration


@pytest.mark.parametrize("shape", ["square", "l", "l2", "big_l"])
def test_sixvertex_named_domains_match_the_oracle(shape):
    m = {"square": ones(20, 20), "l": l_shape(12, 5, 6), "l2": l_shape(16, 8, 8), "big_l": l_shape(200, 80, 90)}[shape]
    got, want = sixv_extremes(m), oracle.sixv_extremal_heights(m)
    assert (got[0] == want[0]).all() and (got[1] == want[1]).all()
    if shape == "square":
        I, J = np.meshgrid(np.arange(21), np.arange(21))
        assert (got[1] == np.abs(I - J)).all() and (got[0] == 20 - np.abs(I + J - 20)).all()


@pytest.mark.parametrize("seed", range(3))
def test_lozenge_domains_match_the_oracle(seed):
    from test_oracle_loz_region import random_tri_domain
    rng = np.random.default_rng(200 + seed)
    ok = 0
    for _ in range(40):
        m = random_tri_domain(rng, int(rng.integers(2, 8)), int(rng.integers(2, 7)), rng.uniform(0.6, 1.0))
        try:
            want = oracle.loz_extremal_heights(m)
        except oracle.Untileable:
            with pytest.raises(tl.TlError) as e:
                tl.domain_extremes(tl.domain(tl.TL_LOZENGE, mask=m))
            assert e.value.status == tl.TL_EUNTILEABLE
            continue
        got = tl.domain_extremes(tl.domain(tl.TL_LOZENGE, mask=m))
        assert (got[0] == want[0]).all() and (got[1] == want[1]).all()
        ok += 1
    assert ok > 2


@pytest.mark.parametrize("abc", [(1, 1, 1), (7, 5, 6), (40, 31, 25)])
def test_lozenge_hexagon_masks_give_the_boxes(abc):
    got = tl.domain_extremes(tl.domain(tl.TL_LOZENGE, mask=oracle.hexagon_mask(*abc)))
    assert (got[1] == oracle.LozengeOracle(*abc, [0, 0]).export()).all()
    assert (got[0] == oracle.LozengeOracle(*abc, [0, 0], init="max").export()).all()


def test_lozenge_mask_errors():
    ring = np.ones((4, 4, 2), dtype=bool)
    ring[1:3, 1:3, :] = False
    with pytest.raises(tl.TlError) as e:
        tl.domain_extremes(tl.domain(tl.TL_LOZENGE, mask=ring))
    assert e.value.status == tl.TL_EINVAL
    one = np.zeros((1, 1, 2), dtype=bool)
    one[0, 0, 0] = True
    with pytest.raises(tl.TlError) as e:
        tl.domain_extremes(tl.domain(tl.TL_LOZENGE, mask=one))
    assert e.value.status == tl.TL_EUNTILEABLE
    with pytest.raises(ValueError):
        tl.domain(tl.TL_LOZENGE, mask=np.ones((3, 3), dtype=bool))


@pytest.mark.parametrize("hw", [(4, 6), (10, 17), (3, 3), (40, 90)])
def test_sixvertex_free_north_matches_the_oracle(hw):
    m = ones(*hw)
    want = oracle.sixv_extremal_heights(m, free_north=True)
    got = tl.domain_extremes(tl.domain(tl.TL_SIXVERTEX, mask=m, free_north=True))
    assert (got[0] == want[0]).all() and (got[1] == want[1]).all()


def test_free_north_thresholds_match_the_oracle():
    from fractions import Fraction
    m = ones(5, 7)
    for wts in ((1, 1, 0.25, 0.75, 0.25, 0.75), (2, 1, 0.5, 1.5, 0.5, 3)):
        for rule in (tl.TL_HEATBATH, tl.TL_METROPOLIS):
            w = tl.weights(tl.TL_W_SIXVERTEX6, *wts, rule=rule)
            metro = rule == tl.TL_METROPOLIS
            want = list(oracle.table_from_ratios(oracle.sixv_ratios6(*map(Fraction, wts)), metro)) + \
                list(oracle.table_from_ratios(oracle.sixv_free_ratios6(*map(Fraction, wts)), metro))
            assert tl.thresholds(tl.domain(tl.TL_SIXVERTEX, mask=m, free_north=True), w) == want
    # three-weight kinds carry only squares: refused with free edges
    with pytest.raises(tl.TlError) as e:
        tl.thresholds(tl.domain(tl.TL_SIXVERTEX, mask=m, free_north=True), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0))
    assert e.value.status == tl.TL_EINVAL


def test_free_north_refusals():
    with pytest.raises(tl.TlError) as e:      # free edges split the fixed boundary of an L-shape
        tl.domain_extremes(tl.domain(tl.TL_SIXVERTEX, mask=l_shape(6, 3, 3), free_north=True))
    assert e.value.status == tl.TL_EINVAL


# every free side: extremes and tables equal the oracle's (wide boxes for a
# free north or south side, tall ones for east or west; a box of the other
# kind has no configuration), and invalid flag sets are refused
SIDE_HW = {"north": [(4, 6), (10, 17)], "south": [(4, 6), (10, 17), (3, 3)], "east": [(6, 4), (17, 10), (3, 3)],
           "west": [(6, 4), (17, 10), (40, 25)]}


@pytest.mark.parametrize("side,hw", [(s_, hw) for s_, l in SIDE_HW.items() for hw in l])
def test_sixvertex_free_side_matches_the_oracle(side, hw):
    m = ones(*hw)
    want = oracle.sixv_extremal_heights(m, free_side=side)
    got = tl.domain_extremes(tl.domain(tl.TL_SIXVERTEX, mask=m, free_side=side))
    assert (got[0] == want[0]).all() and (got[1] == want[1]).all()


@pytest.mark.parametrize("side", ["north", "south", "east", "west"])
def test_free_side_thresholds_match_the_oracle(side):
    from fractions import Fraction
    m = ones(*SIDE_HW[side][0])
    for wts in ((1, 1, 0.25, 0.75, 0.25, 0.75), (2, 1, 0.5, 1.5, 0.5, 3)):
        for rule in (tl.TL_HEATBATH, tl.TL_METROPOLIS):
            w = tl.weights(tl.TL_W_SIXVERTEX6, *wts, rule=rule)
            metro = rule == tl.TL_METROPOLIS
            want = list(oracle.table_from_ratios(oracle.sixv_ratios6(*map(Fraction, wts)), metro)) + \
                list(oracle.table_from_ratios(oracle.sixv_free_ratios6(*map(Fraction, wts), side=side), metro))
            assert tl.thresholds(tl.domain(tl.TL_SIXVERTEX, mask=m, free_side=side), w) == want


def test_free_side_refusals():
    m = ones(6, 4)
    bad = tl.domain(tl.TL_SIXVERTEX, mask=m)
    bad.flags = tl.TL_FREE_EAST | tl.TL_FREE_WEST   # one side per domain
    with pytest.raises(tl.TlError) as e:
        tl.domain_extremes(bad)
    assert e.value.status == tl.TL_EINVAL
    with pytest.raises(tl.TlError) as e:      # a wide box has no configuration with a free east side
        tl.domain_extremes(tl.domain(tl.TL_SIXVERTEX, mask=ones(4, 6), free_side="east"))
    assert e.value.status == tl.TL_EUNTILEABLE
    dom = tl.domain(tl.TL_DOMINO, mask=ones(4, 4))
    dom.flags = tl.TL_FREE_SOUTH                # dominoes have no free sides
    with pytest.raises(tl.TlError) as e:
        tl.thresholds(dom, tl.weights(tl.TL_W_UNIFORM))
    assert e.value.status == tl.TL_EINVAL
