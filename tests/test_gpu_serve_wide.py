"""Served jobs beyond the fixed shapes and the fixed colour order: domains
given by masks of every model (Section 1.1 domains; Section 1.2 models;
free north edges) and the paper's random colour choice per step (Section
2.2), mixed with fixed shapes in one server: every result equals the same job
on a lone sampler, and for some jobs the oracle's chain."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say
from test_gpu_loz_region import weird
from test_gpu_region import mask_of as domino_mask
from test_gpu_sixv_region import STOCH, mask_of as sixv_mask
from test_oracle_region import ones

pytestmark = pytest.mark.gpu


def jobs_of(tl):
    """(name, domain, weights) of the mix."""
    def w(kind, *v, metro=False):
        x = tl.weights(kind, *v)
        x.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
        return x
    return [
        ("domino l40", tl.domain(tl.TL_DOMINO, mask=domino_mask("l40")), w(tl.TL_W_UNIFORM)),
        ("domino random40 max", tl.domain(tl.TL_DOMINO, mask=domino_mask("random40"), init=tl.TL_INIT_MAX),
         w(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)),
        ("domino square130", tl.domain(tl.TL_DOMINO, mask=domino_mask("square130")), w(tl.TL_W_UNIFORM)),
        ("six-vertex l40", tl.domain(tl.TL_SIXVERTEX, mask=sixv_mask("l40")), w(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)),
        ("six-vertex random30 metro", tl.domain(tl.TL_SIXVERTEX, mask=sixv_mask("random30")),
         w(tl.TL_W_SIXVERTEX, 1.0, 1.0, 1.0, metro=True)),
        ("six-vertex l130", tl.domain(tl.TL_SIXVERTEX, mask=sixv_mask("l130"), init=tl.TL_INIT_MAX),
         w(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)),
        ("six-vertex free north", tl.domain(tl.TL_SIXVERTEX, mask=ones(30, 50), free_north=True),
         w(tl.TL_W_SIXVERTEX6, *STOCH)),
        ("lozenge weird", tl.domain(tl.TL_LOZENGE, mask=weird(12)), w(tl.TL_W_VOLUME, 9.0, 10.0)),
        ("Aztec 70", tl.domain(tl.TL_DOMINO, n=70), w(tl.TL_W_UNIFORM)),
        ("six-vertex N=40", tl.domain(tl.TL_SIXVERTEX, n=40), w(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0, metro=True)),
        ("hexagon 12", tl.domain(tl.TL_LOZENGE, a=12, b=12, c=12), w(tl.TL_W_VOLUME, 9.0, 10.0)),
    ]


@pytest.mark.parametrize("order", [0, 1])
def test_served_masks_equal_lone_samplers(order):
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    mix = jobs_of(tl)
    say("served mix of %d jobs (masks and fixed shapes), colour order %d" % (len(mix), order))
    sv = Server(64 << 20, 6, tl.options(sweeps_per_launch=5, colour_order=order))
    sweeps = 23
    tickets = [sv.submit(dom, w, 40 + i, sweeps) for i, (_, dom, w) in enumerate(mix)]
    res = [sv.wait(t, 120.0) for t in tickets]
    st = sv.stats()
    sv.destroy()
    assert st["peak_active"] <= 6
    for i, ((name, dom, w), r) in enumerate(zip(mix, res)):
        assert r["status"] == tl.TL_OK and r["sweeps"] == sweeps, name
        s = tl.Sampler(dom, w, 40 + i, tl.options(colour_order=order))
        s.sweep(sweeps)
        assert r["hash"] == s.hash(), name
        assert r["scalar_now"] == s.observables()["scalar_now"], name
        s.destroy()


def test_served_mask_jobs_against_oracle():
    # two masked jobs, random colour order, against the oracle's chains
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    sv = Server(64 << 20, 4, tl.options(sweeps_per_launch=4, colour_order=1))
    m_dom, m_six = domino_mask("random40"), sixv_mask("l40")
    wd = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)
    ws = tl.weights(tl.TL_W_SIXVERTEX, 1.0, 1.0, 2.0)
    ta = sv.submit(tl.domain(tl.TL_DOMINO, mask=m_dom), wd, 5, 19)
    tb = sv.submit(tl.domain(tl.TL_SIXVERTEX, mask=m_six), ws, 6, 19)
    ra, rb = sv.wait(ta, 60.0), sv.wait(tb, 60.0)
    sv.destroy()
    od = oracle.DominoRegionOracle(m_dom, oracle.table_from_ratios(oracle.domino_ratios("two", 1, Fraction(1, 2)),
                                                                   False), seed=5, random_colours=True)
    od.sweep(19)
    assert ra["hash"] == oracle.canonical_hash(od.export())
    os_ = oracle.SixVertexRegionOracle(m_six, oracle.table_from_ratios(oracle.sixv_ratios(1, 1, 2), False), seed=6,
                                       random_colours=True)
    os_.sweep(19)
    assert rb["hash"] == oracle.canonical_hash(os_.export())
