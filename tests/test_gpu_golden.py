"""Full-length parity of the benchmark workloads against stored oracle results.

``tests/golden/*.json`` are written by ``python -m oracle.goldens`` (the serial
oracle alone).  Each GPU test here runs the workload in the configuration the
benchmark times (the same sampler options, tile plans, batch and server
settings) over its whole chain and compares what the paper's RandomWalk
returns (Section 2.2: the tiling after the given number of steps) bit for bit:
the canonical hash, the integer observable counters, and the fp64 densities
to a relative 1e-6.
"""
import json
import os
import sys
from argparse import Namespace

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle result %s" % name)
    return json.load(open(path))


def bench_sampler(tl, workload):
    """The benchmark's sampler for a plain workload, with its default options."""
    import bench
    args = Namespace(kernel=0, sweeps_per_launch=0, tile_rows=0, tile_groups=0)
    return bench.make_sampler(tl, bench.WORKLOADS[workload], args), bench.WORKLOADS[workload]


def check_plain(tl, name, in_domain, variant=None):
    """variant: the stored result of a variant of the workload (aztec2048r:
    the random colour order; square2048: the square domain given as a mask),
    run with the sampler of the benchmark's variants leg."""
    g = golden(variant or name)
    s, wl = bench_sampler(tl, name)
    if variant:
        s.destroy()
        if variant == "square2048":
            dom = tl.domain(tl.TL_DOMINO, mask=np.ones((g["side"], g["side"]), dtype=np.uint8))
            order = 0
        else:
            dom = tl.domain(tl.TL_DOMINO, n=wl["n"])
            order = 1
        s = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), wl["seed"],
                       tl.options(obs_every=wl["obs_every"], obs_bin=wl["obs_bin"], colour_order=order))
    assert (wl["seed"], wl["sweeps"], wl["obs_every"], wl["obs_bin"]) == (g["seed"], g["sweeps"], g["obs_every"],
                                                                          g["bin"])
    assert s.thresholds() == g["thresholds"]
    # the benchmark's step: reset on the device, all sweeps in one call
    say("%s: %d sweeps in one call" % (name, g["sweeps"]))
    s.reset(wl["seed"])
    s.sweep(wl["sweeps"])
    obs = s.observables()
    assert s.hash() == g["hash"], "%s: final tiling differs from the oracle" % name
    assert obs["samples"] == g["samples"]
    assert obs["scalar_sum"] == g["scalar_sum"]
    assert (obs["bin_sum"].reshape(-1) == np.asarray(g["bin_sum"], dtype=np.uint64)).all()
    dens = oracle.bin_density(np.asarray(g["bin_sum"], dtype=np.uint64), g["samples"], in_domain, g["bin"])
    got = obs["bin_density"]
    assert got.shape == dens.shape
    assert np.allclose(got, dens, rtol=1e-6, atol=0.0)
    # the same chain in pieces, through the oracle's intermediate states
    s.reset(wl["seed"])
    t = 0
    for m in g["marks"]:
        s.sweep(m["t"] - t)
        t = m["t"]
        assert s.hash() == m["hash"], "%s: differs from the oracle after %d sweeps" % (name, t)
    assert s.observables()["bin_sum"].reshape(-1).tolist() == g["bin_sum"]
    s.destroy()


def test_aztec2048_full_chain():
    """Order-2048 Aztec diamond, uniform, brick start, seed 7, 10^4 sweeps,
    64 x 64-face density bins every 100 sweeps."""
    tl = need_gpu()
    n = 2048
    Y, X = np.mgrid[0:2 * n, 0:2 * n]
    inside = np.abs(2 * X - 2 * n + 1) + np.abs(2 * Y - 2 * n + 1) <= 2 * n
    check_plain(tl, "aztec2048", inside)


def test_aztec2048_random_order_full_chain():
    """The same job under the random colour choice per step (the benchmark's
    random-order variant: register tiles of 8 sweeps per launch)."""
    tl = need_gpu()
    n = 2048
    Y, X = np.mgrid[0:2 * n, 0:2 * n]
    inside = np.abs(2 * X - 2 * n + 1) + np.abs(2 * Y - 2 * n + 1) <= 2 * n
    check_plain(tl, "aztec2048", inside, variant="aztec2048r")


def test_square2048_domain_full_chain():
    """The same job on the 2048 x 2048 square given as a mask, from T_min (the
    benchmark's square-domain variant)."""
    tl = need_gpu()
    check_plain(tl, "aztec2048", np.ones((2048, 2048), dtype=bool), variant="square2048")


def test_hexagon1024_full_chain():
    """1024^3 hexagon, q = 1999/2000, empty-box start, seed 11, 2 x 10^4
    sweeps, volume bins of 64 x 64 vertices every 200 sweeps."""
    tl = need_gpu()
    a = b = c = 1024
    Y, X = np.mgrid[0:b + c + 1, 0:a + c + 1]
    x, y = X - c, Y - c
    inside = (x >= -c) & (x <= a) & (y >= -c) & (y <= b) & (x - y >= -b) & (x - y <= a)
    check_plain(tl, "hexagon1024", inside)


@pytest.mark.parametrize("name", ["sixv1024", "sixv1024u"])
def test_sixv1024_full_chain(name):
    """Six-vertex domain-wall square N = 1024, heat-bath (1,1,sqrt 2) (bit-serial
    decisions) and (1,1,1) (one-bit decisions), 2000 sweeps, c-vertex bins."""
    tl = need_gpu()
    check_plain(tl, name, np.ones((1024, 1024), dtype=bool))


def test_batch4096_full_call():
    """The benchmark's 4096-chain batch (two-periodic a = 1, b = 1/2) in one
    5000-sweep call after the benchmark's autotuning: the stored chains (every
    64th and the smallest and largest orders) equal the oracle's."""
    tl = need_gpu()
    from paper_1804_07250_amd import workloads
    from paper_1804_07250_amd.serving import Batch
    g = golden("batch4096")
    orders = workloads.batch_orders(g["chains_total"])
    say("batch of %d chains, %d sweeps" % (len(orders), g["sweeps"]))
    b = Batch([tl.domain(tl.TL_DOMINO, n=n) for n in orders], tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5),
              list(range(len(orders))))
    b.autotune(4)
    b.sweep(g["sweeps"])
    b.sync()
    bad = [c["chain"] for c in g["chains"] if orders[c["chain"]] != c["order"] or b.hash(c["chain"]) != c["hash"]]
    b.destroy()
    assert not bad, "chains differing from the oracle: %s" % bad


def test_cftp_exact_samples_of_the_benchmark():
    """The benchmark's exact samples by coupling from the past (uniform
    weights, seeds 0 and 1, at most 2^30 sweeps): the six-vertex N = 128
    square and the Aztec diamond of order 64 coalesce at the oracle's R and
    give its sample."""
    tl = need_gpu()
    g = golden("cftp")
    for c in g["cases"]:
        say("cftp %s n=%d seed %d" % (c["model"], c["n"], c["seed"]))
        model = tl.TL_SIXVERTEX if c["model"] == "sixvertex" else tl.TL_DOMINO
        s = tl.Sampler(tl.domain(model, n=c["n"]), tl.weights(tl.TL_W_UNIFORM), c["seed"])
        info = s.cftp(30)
        digest = s.hash()
        s.destroy()
        assert info["log2_sweeps"] == c["log2_sweeps"] and digest == c["hash"], c


def test_served_requests_in_a_budget_bound_mix():
    """The stored requests of the served stream (ten of each size and weight
    set), submitted together to a server whose memory budget, not its slots,
    limits how many run at once: every result equals the oracle's."""
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    g = golden("served")
    reqs = g["requests"]
    budget = 12 << 20
    sv = Server(budget, 64, tl.options(sweeps_per_launch=8))
    say("served: %d requests, budget %d MiB" % (len(reqs), budget >> 20))
    tickets = []
    for r in reqs:
        w = tl.weights(tl.TL_W_SIXVERTEX, *r["w2"])
        w.rule = tl.TL_METROPOLIS
        tickets.append(sv.submit(tl.domain(tl.TL_SIXVERTEX, n=r["N"]), w, r["seed"], g["sweeps"]))
    res = [sv.wait(t, 300.0) for t in tickets]
    st = sv.stats()
    sv.destroy()
    assert st["peak_bytes"] <= budget and st["peak_active"] < 64
    for r, x in zip(reqs, res):
        assert x["status"] == tl.TL_OK and x["sweeps"] == g["sweeps"]
        assert x["hash"] == r["hash"], "request %d (N=%d) differs from the oracle" % (r["request"], r["N"])
        assert x["scalar_now"] == r["scalar_now"]
