"""GPU tests of the batched form (many Aztec chains in one persistent,
graph-replayed launch) and the served form (continuous-batching request loop):
every chain / job must equal the same chain run alone, and the oracle."""
import time
from fractions import Fraction

import numpy as np
import pytest

import oracle
from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def two_periodic(tl, metro=False):
    w = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return w


ORDERS = [1, 2, 3, 5, 16, 31, 32, 33, 64, 100, 127, 128, 129, 200, 257, 300, 384, 511, 512, 17, 45, 90]


@pytest.mark.parametrize("metro", [False, True])
def test_batch_equals_single_chains_and_oracle(metro):
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Batch
    say("batch parity metro=%s" % metro)
    doms = [tl.domain(tl.TL_DOMINO, n=n) for n in ORDERS]
    seeds = [1000 + i for i in range(len(ORDERS))]
    b = Batch(doms, two_periodic(tl, metro), seeds)
    b.sweep(7)
    b.sweep(5)   # a second graph (different sweep count)
    b.sync()
    for i, n in enumerate(ORDERS):
        s = tl.Sampler(doms[i], two_periodic(tl, metro), seeds[i])
        s.sweep(12)
        assert (b.export(i) == s.export()).all(), "chain %d (order %d)" % (i, n)
        if n <= 64:
            o = oracle.DominoOracle(n, oracle.table_from_ratios(oracle.domino_ratios("two", 1, Fraction(1, 2)),
                                                                metro), metropolis=metro, seed=seeds[i])
            o.sweep(12)
            assert (b.export(i) == o.export()).all()
            assert b.hash(i) == oracle.canonical_hash(o.export())


def test_batch_graph_replays_and_autotune():
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Batch
    doms = [tl.domain(tl.TL_DOMINO, n=n) for n in (300, 17, 512, 64)]
    seeds = [5, 6, 7, 8]
    b = Batch(doms, tl.weights(tl.TL_W_UNIFORM), seeds)
    th, ms = b.autotune(2)
    assert th in (256, 512, 1024) and ms > 0
    for _ in range(4):          # same sweep count: replays of one captured graph
        b.sweep(3)
    b.sync()
    for i, d in enumerate(doms):
        s = tl.Sampler(d, tl.weights(tl.TL_W_UNIFORM), seeds[i])
        s.sweep(12)
        assert (b.export(i) == s.export()).all()
    b.reset()
    b.sweep(12)
    b.sync()
    s = tl.Sampler(doms[2], tl.weights(tl.TL_W_UNIFORM), seeds[2])
    s.sweep(12)
    assert b.hash(2) == s.hash()


def test_batch_rejects_bad_orders():
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Batch
    with pytest.raises(tl.TlError):
        Batch([tl.domain(tl.TL_DOMINO, n=600)], tl.weights(tl.TL_W_UNIFORM), [1])
    with pytest.raises(tl.TlError):
        Batch([tl.domain(tl.TL_SIXVERTEX, n=6)], tl.weights(tl.TL_W_UNIFORM), [1])


def sixv_w(tl, w2, metro=False):
    w = tl.weights(tl.TL_W_SIXVERTEX, *w2)
    w.rule = tl.TL_METROPOLIS if metro else tl.TL_HEATBATH
    return w


def test_server_mix_equals_alone_and_oracle():
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    say("server mix")
    jobs = []
    for i, N in enumerate([8, 16, 33, 64, 100, 16, 257, 8]):
        w2 = (1.0, 1.0, 2.0) if i % 2 == 0 else (1.0, 1.0, 1.0)
        jobs.append((tl.domain(tl.TL_SIXVERTEX, n=N), sixv_w(tl, w2, metro=(i % 3 == 2)), 40 + i, 30 + 7 * i))
    jobs.append((tl.domain(tl.TL_DOMINO, n=40), tl.weights(tl.TL_W_UNIFORM), 99, 25))
    jobs.append((tl.domain(tl.TL_LOZENGE, a=9, b=10, c=11), tl.weights(tl.TL_W_VOLUME, 3, 4), 98, 21))
    budget = 3 * 1024 * 1024
    sv = Server(budget, max_slots=4, opt=tl.options(sweeps_per_launch=8))
    tickets = [sv.submit(d, w, seed, n) for d, w, seed, n in jobs]
    res = [sv.wait(t, 120.0) for t in tickets]
    st = sv.stats()
    sv.destroy()
    assert st["completed"] == len(jobs) and st["peak_bytes"] <= budget and st["peak_active"] <= 4
    for (d, w, seed, n), r in zip(jobs, res):
        assert r["status"] == tl.TL_OK and r["sweeps"] == n
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
        s = tl.Sampler(d, w, seed)
        s.sweep(n)
        assert r["hash"] == s.hash(), "job seed %d differs from the same job alone" % seed
        assert r["scalar_now"] == s.observables()["scalar_now"]
    # small six-vertex jobs against the oracle
    for (d, w, seed, n), r in zip(jobs, res):
        if d.model == tl.TL_SIXVERTEX and d.n <= 33:
            c2 = int(w.w[2])
            o = oracle.SixVertexOracle(d.n, oracle.table_from_ratios(oracle.sixv_ratios(1, 1, c2),
                                                                     w.rule == tl.TL_METROPOLIS),
                                       metropolis=w.rule == tl.TL_METROPOLIS, seed=seed)
            o.sweep(n)
            assert r["hash"] == oracle.canonical_hash(o.export())


def test_server_budget_and_alone():
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    sv = Server(64 * 1024, max_slots=2)
    with pytest.raises(tl.TlError) as e:
        sv.submit(tl.domain(tl.TL_SIXVERTEX, n=1024), tl.weights(tl.TL_W_UNIFORM), 1, 10)
    assert e.value.status == tl.TL_EBUDGET
    t = sv.submit(tl.domain(tl.TL_SIXVERTEX, n=20), sixv_w(tl, (1.0, 1.0, 2.0)), 7, 50)
    r = sv.wait(t, 60.0)
    sv.destroy()
    sv2 = Server(64 * 1024 * 1024, max_slots=8)
    tickets = [sv2.submit(tl.domain(tl.TL_SIXVERTEX, n=n), sixv_w(tl, (1.0, 1.0, 2.0)), 100 + n, 50)
               for n in (64, 128, 20, 256)]
    r_mix = [sv2.wait(x, 60.0) for x in tickets]
    sv2.destroy()
    assert r_mix[2]["hash"] != r["hash"]   # different seed
    s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=20), sixv_w(tl, (1.0, 1.0, 2.0)), 7)
    s.sweep(50)
    assert r["hash"] == s.hash()


@pytest.mark.parametrize("quantum", [3, 8])
def test_server_multi_tile_jobs_equal_alone(quantum):
    # jobs large enough to be cut into row tiles with halos (six-vertex N=600,
    # Aztec order 300, a 200^3 hexagon), small single-tile ones, a job of zero
    # sweeps and sweep counts that are not multiples of the tick's share, more
    # jobs than slots: each result equals the same job run alone
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    say("server multi-tile jobs quantum=%d" % quantum)
    metro = sixv_w(tl, (1.0, 1.0, 2.0), metro=True)
    jobs = [(tl.domain(tl.TL_SIXVERTEX, n=600), sixv_w(tl, (1.0, 1.0, 2.0)), 5, 37),
            (tl.domain(tl.TL_DOMINO, n=300), tl.weights(tl.TL_W_UNIFORM), 6, 41),
            (tl.domain(tl.TL_LOZENGE, a=200, b=200, c=200), tl.weights(tl.TL_W_VOLUME, 1999, 2000), 7, 23),
            (tl.domain(tl.TL_SIXVERTEX, n=600), sixv_w(tl, (1.0, 1.0, 1.0)), 8, 50),
            (tl.domain(tl.TL_SIXVERTEX, n=48), metro, 9, 29),
            (tl.domain(tl.TL_DOMINO, n=150), two_periodic(tl), 10, 19),
            (tl.domain(tl.TL_SIXVERTEX, n=64), sixv_w(tl, (1.0, 1.0, 2.0)), 11, 0),
            (tl.domain(tl.TL_LOZENGE, a=30, b=20, c=10), tl.weights(tl.TL_W_UNIFORM), 12, 33),
            (tl.domain(tl.TL_SIXVERTEX, n=90), tl.weights(tl.TL_W_SIXVERTEX6, 1.0, 2.0, 1.5, 0.5, 1.0, 3.0), 13, 26),
            (tl.domain(tl.TL_DOMINO, n=64), tl.weights(tl.TL_W_VOLUME_BW, 20.0, 1.0, 1.0, 20.0), 14, 15)]
    sv = Server(256 * 1024 * 1024, max_slots=3, opt=tl.options(sweeps_per_launch=quantum))
    tickets = [sv.submit(d, w, seed, n) for d, w, seed, n in jobs]
    res = [sv.wait(t, 120.0) for t in tickets]
    st = sv.stats()
    sv.destroy()
    assert st["completed"] == len(jobs) and st["peak_active"] <= 3 and st["bytes_in_use"] == 0
    for (d, w, seed, n), r in zip(jobs, res):
        assert r["status"] == tl.TL_OK and r["sweeps"] == n
        s = tl.Sampler(d, w, seed)
        s.sweep(n)
        assert r["hash"] == s.hash(), "job seed %d differs from the same job alone" % seed
        assert r["scalar_now"] == s.observables()["scalar_now"]


def test_server_admission_waits_for_memory():
    # the memory budget, not the slots, bounds the jobs on the device: a budget
    # of 2.5 times the largest job holds two of them, so of six jobs submitted
    # together some wait in the queue until another job's memory returns; each
    # result still equals the same job alone and the oracle
    tl = need_gpu()
    from paper_1804_07250_amd.serving import Server
    say("server admission by memory budget")
    jobs = [(256, (1.0, 1.0, 2.0), False, 300 + i, 120 + 10 * i) for i in range(4)]
    jobs += [(200, (1.0, 1.0, 1.0), True, 310, 90), (256, (1.0, 1.0, 1.0), False, 311, 150)]
    probe = Server(256 << 20, 1)
    t = probe.submit(tl.domain(tl.TL_SIXVERTEX, n=256), sixv_w(tl, (1.0, 1.0, 2.0)), 1, 1)
    probe.wait(t, 60.0)
    largest = probe.stats()["peak_bytes"]       # device bytes of one N = 256 job
    probe.destroy()
    budget = int(2.5 * largest)
    sv = Server(budget, max_slots=16, opt=tl.options(sweeps_per_launch=4))
    tickets = [sv.submit(tl.domain(tl.TL_SIXVERTEX, n=N), sixv_w(tl, w2, metro), seed, n)
               for N, w2, metro, seed, n in jobs]
    res = [sv.wait(x, 120.0) for x in tickets]
    st = sv.stats()
    sv.destroy()
    assert st["completed"] == len(jobs) and st["bytes_in_use"] == 0
    assert st["peak_bytes"] <= budget
    assert 2 <= st["peak_active"] < len(jobs)
    # some job started only after another one had finished (it waited for memory)
    assert any(b["t_start"] >= a["t_done"] for a in res for b in res if a is not b)
    for (N, w2, metro, seed, n), r in zip(jobs, res):
        assert r["status"] == tl.TL_OK and r["sweeps"] == n
        s = tl.Sampler(tl.domain(tl.TL_SIXVERTEX, n=N), sixv_w(tl, w2, metro), seed)
        s.sweep(n)
        assert r["hash"] == s.hash(), "job seed %d differs from the same job alone" % seed
        o = oracle.SixVertexOracle(N, oracle.table_from_ratios(oracle.sixv_ratios(1, 1, int(w2[2])), metro),
                                   metropolis=metro, seed=seed)
        o.sweep(n)
        assert r["hash"] == oracle.canonical_hash(o.export())
        assert r["scalar_now"] == o.observe()[0]
