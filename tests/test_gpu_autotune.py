"""Tile shapes picked by measurement (tl_sampler_autotune): the chain of an
autotuned sampler equals the oracle's and an untuned sampler's bit for bit,
the probe leaves the sampler's state and sweep counter alone, and the shape
cache is written once and then read back without probing."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def cases(tl):
    return {
        "aztec300": (tl.domain(tl.TL_DOMINO, n=300), tl.weights(tl.TL_W_UNIFORM)),
        "aztec200two": (tl.domain(tl.TL_DOMINO, n=200), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)),
        "hexagon80": (tl.domain(tl.TL_LOZENGE, a=80, b=70, c=90), tl.weights(tl.TL_W_VOLUME, 3.0, 4.0)),
        "sixv257": (tl.domain(tl.TL_SIXVERTEX, n=257), tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)),
    }


@pytest.mark.parametrize("name", ["aztec300", "aztec200two", "hexagon80", "sixv257"])
def test_autotuned_chain_is_unchanged(name):
    tl = need_gpu()
    say("autotune %s" % name)
    dom, w = cases(tl)[name]
    a = tl.Sampler(dom, w, 13)
    b = tl.Sampler(dom, w, 13)
    a.sweep(5)
    b.sweep(5)
    before = b.export()
    info = b.autotune(12)
    assert info["from_cache"] == 0 and info["candidates"] > 1 and info["ms_per_sweep"] > 0
    assert (b.export() == before).all()          # the probe ran on a copy
    for k in (7, 30):
        a.sweep(k)
        b.sweep(k)
        assert (a.export() == b.export()).all()
    assert a.hash() == b.hash()


def test_autotuned_equals_oracle():
    tl = need_gpu()
    n = 60
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=n), tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5), 4)
    s.autotune(6)
    o = oracle.DominoOracle(n, oracle.table_from_ratios(oracle.domino_ratios("two", 1, Fraction(1, 2)), False),
                            seed=4)
    for k in (3, 20):
        s.sweep(k)
        o.sweep(k)
        assert (s.export() == o.export()).all()


def test_cache_is_written_and_reused(tmp_path):
    tl = need_gpu()
    path = str(tmp_path / "tiles.txt")
    dom = tl.domain(tl.TL_LOZENGE, a=60, b=60, c=60)
    w = tl.weights(tl.TL_W_VOLUME, 1.0, 2.0)
    first = tl.Sampler(dom, w, 1, tl.options(tune_cache=path)).autotune(8)
    assert first["from_cache"] == 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:] == [str(first["tile_rows"]), str(first["tile_groups"]),
                                                          str(first["sweeps_per_launch"]), str(first["kernel"])]
    s = tl.Sampler(dom, w, 2, tl.options(tune_cache=path))
    again = s.autotune(8)
    assert again["from_cache"] == 1 and again["candidates"] == 0
    assert [again[k] for k in ("tile_rows", "tile_groups", "sweeps_per_launch", "kernel")] == \
        [first[k] for k in ("tile_rows", "tile_groups", "sweeps_per_launch", "kernel")]
    assert len(open(path).read().splitlines()) == 1
    # another table kind is another entry
    u = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), 3, tl.options(tune_cache=path)).autotune(8)
    assert u["from_cache"] == 0 and len(open(path).read().splitlines()) == 2
    ref = tl.Sampler(dom, w, 2)
    s.sweep(25)
    ref.sweep(25)
    assert (s.export() == ref.export()).all()


def test_autotune_refuses_the_streaming_kernel():
    tl = need_gpu()
    s = tl.Sampler(tl.domain(tl.TL_DOMINO, n=16), tl.weights(tl.TL_W_UNIFORM), 1, tl.options(kernel=1))
    with pytest.raises(tl.TlError) as e:
        s.autotune()
    assert e.value.status == tl.TL_EINVAL


def test_domino_autotune_register_tiles_cache(tmp_path):
    # a domino large enough for register tiles: the chosen kernel goes to the
    # cache with the shape, comes back from it, and the chain is unchanged
    tl = need_gpu()
    path = str(tmp_path / "tiles.txt")
    dom = tl.domain(tl.TL_DOMINO, n=700)
    first = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), 1, tl.options(tune_cache=path)).autotune(20)
    assert first["from_cache"] == 0 and first["kernel"] in (2, 3) and first["candidates"] > 1
    s = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), 5, tl.options(tune_cache=path))
    again = s.autotune(20)
    assert again["from_cache"] == 1 and again["kernel"] == first["kernel"]
    ref = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), 5, tl.options(kernel=1))
    s.sweep(37)
    ref.sweep(37)
    assert s.hash() == ref.hash()
