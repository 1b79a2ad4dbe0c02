"""Benchmark of the parallel Glauber sweep on one MI355X.

Default workload: domino tilings of the order-2048 Aztec diamond, uniform
weights, all-horizontal brick start, 10^4 sweeps, Philox seed 7, state
bit-packed at 2 bits per face, observables = 64 x 64-binned horizontal-domino
density (bins of 64 x 64 faces, sampled every 100 sweeps, fp64 densities),
output = canonical row hash of the final tiling.

One step = reset the chain on the device + 10^4 sweeps + observables + hash
(every row of the hot path).  value = site-updates per second over the timed
steps; a site-update is one attempted update of one site in one colour step.

Prints one JSON line with the roofline of the dominant kernel (the sweep
kernel, timed per launch by its own dispatch events), the other forms and
models of the path measured on the same GPU (the lozenge hexagon and the
weighted six-vertex square, the batched and served forms, coupling from the
past, the random colour order and a mask domain), each result compared with
the oracle's stored result where one exists (tests/golden), and the serial
CPU oracle's rate on a bounded, representative sample of the same workload,
single-core and over several processes.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS: 256 bytes per clock per CU for conflict-free 128-bit reads (gfx950),
# 256 CUs, 2.4 GHz
LDS_PEAK_GBS = 256 * 256 * 2.4
# VALU: 4 SIMDs of 16 lanes per CU (one wave64 instruction per SIMD every
# 4 clocks, 64 lane-operations per clock per CU) x 256 CUs x 2.4 GHz
VALU_PEAK_TOPS = 64 * 256 * 2.4e9 / 1e12

WORKLOADS = {
    "aztec2048": dict(model="domino", n=2048, sweeps=10000, seed=7, obs_every=100, obs_bin=64),
    "aztec64": dict(model="domino", n=64, sweeps=1000, seed=1, obs_every=1, obs_bin=1),
    "hexagon1024": dict(model="lozenge", a=1024, b=1024, c=1024, q=(1999, 2000), sweeps=20000, seed=11,
                        obs_every=200, obs_bin=64),
    "sixv1024": dict(model="sixvertex", n=1024, w2=(1.0, 1.0, 2.0), sweeps=2000, seed=0, obs_every=100, obs_bin=64),
    "sixv1024u": dict(model="sixvertex", n=1024, w2=(1.0, 1.0, 1.0), sweeps=2000, seed=1, obs_every=100, obs_bin=64),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="aztec2048", choices=sorted(WORKLOADS))
    p.add_argument("--kernel", type=int, default=0, help="0 auto, 1 one launch per colour step, 2 tiled")
    p.add_argument("--sweeps-per-launch", type=int, default=0)
    p.add_argument("--tile-rows", type=int, default=0)
    p.add_argument("--tile-groups", type=int, default=0)
    p.add_argument("--no-timing", action="store_true", help="no per-launch dispatch events")
    p.add_argument("--timing-period", type=int, default=8,
                   help="time every k-th sweep launch with its own dispatch events")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--cpu-procs", type=int, default=16, help="processes of the multi-process oracle figure (at most)")
    p.add_argument("--sweeps-only", action="store_true",
                   help="time only the sweeps (for profiler runs); no JSON contract line")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="run a plain device copy of this many MiB (profiler calibration) and exit")
    p.add_argument("--no-models", action="store_true",
                   help="skip the lozenge and weighted six-vertex legs of the default workload")
    p.add_argument("--model-steps", type=int, default=3, help="timed jobs of each model leg")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-served", action="store_true")
    p.add_argument("--batched-chains", type=int, default=4096)
    p.add_argument("--batched-sweeps", type=int, default=5000)
    p.add_argument("--served-requests", type=int, default=2000)
    p.add_argument("--served-rate", type=float, default=200.0)
    p.add_argument("--served-sweeps", type=int, default=2000)
    p.add_argument("--served-budget-mib", type=int, default=1024)
    p.add_argument("--served-tight-mib", type=int, default=16,
                   help="budget of the second served run, one the offered load fills (0: no second run)")
    p.add_argument("--served-slots", type=int, default=64)
    p.add_argument("--served-quantum", type=int, default=8, help="sweeps per tick of a weighted request")
    p.add_argument("--no-cftp", action="store_true")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the random-colour-order and general-domain legs of the plain workload")
    p.add_argument("--domain-side", type=int, default=2048, help="side of the square domain leg")
    p.add_argument("--cftp-n", type=int, default=128, help="six-vertex DWBC size for coupling from the past")
    p.add_argument("--cftp-aztec", type=int, default=64, help="Aztec order for coupling from the past")
    p.add_argument("--cftp-samples", type=int, default=2)
    return p.parse_args()


def golden(name):
    """The oracle's stored result of a workload (tests/golden/<name>.json,
    written by the oracle alone), or None."""
    path = os.path.join(ROOT, "tests", "golden", name + ".json")
    return json.load(open(path)) if os.path.exists(path) else None


def alu_roofline(rec, avg_launch_s):
    """Lane throughput of the VALU from rocprofv3 SQ counters: lane-operations
    per launch (SQ_THREAD_CYCLES_VALU) over the live launch time, against
    64 lanes x 256 CUs x 2.4 GHz.  The same as busy share x lane use."""
    if not rec or "valu_counters_raw" not in rec or avg_launch_s <= 0:
        return None
    ops = rec["valu_counters_raw"]["SQ_THREAD_CYCLES_VALU"]
    achieved = ops / avg_launch_s / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "T int32 lane-ops/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
            "lane_ops_per_launch": ops}


def hbm_figure(alg_bytes, rec, avg_launch_s):
    """Algorithmic bytes per launch over the launch time (the streaming
    formulation of a colour step), and the HBM bytes the counters measured."""
    achieved = alg_bytes / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    # a rate above the peak means the state did not stream through HBM: the
    # figure is then no roofline, and no fraction of it is given
    frac = achieved / HBM_PEAK_GBS
    out = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(frac, 4) if frac <= 1.0 else None, "algorithmic_bytes_per_launch": alg_bytes,
           "traffic": rec["bytes_per_launch"] if rec else None}
    if rec and avg_launch_s > 0:
        out["traffic_GBps"] = round(rec["bytes_per_launch"] / avg_launch_s / 1e9, 1)
    return out


def run_batched(tl, args):
    """Batched form: Aztec chains of orders uniform in [16, 512], two-periodic
    weights a = 1, b = 1/2, seeds 0..count-1, args.batched_sweeps sweeps in one
    graph-replayed persistent launch; work-group size from the autotuner.  The
    chains the oracle has stored results for are compared with them."""
    from paper_1804_07250_amd import workloads
    from paper_1804_07250_amd.serving import Batch
    orders = workloads.batch_orders(args.batched_chains)
    doms = [tl.domain(tl.TL_DOMINO, n=n) for n in orders]
    w = tl.weights(tl.TL_W_TWO_PERIODIC, 1.0, 0.5)
    b = Batch(doms, w, list(range(len(orders))))
    threads, probe_ms = b.autotune(4)
    info = b.info()
    b.sweep(args.batched_sweeps)   # warm-up (captures the graph)
    b.sync()
    b.reset()
    b.sync()
    b.set_timing(True)
    t0 = time.perf_counter()
    b.sweep(args.batched_sweeps)
    b.sync()
    el = time.perf_counter() - t0
    kms, launches, steps = b.kernel_time()
    # rocprofv3 counters of the same workload's full launches, if recorded for the current sources
    full = (len(orders), args.batched_sweeps) == (4096, 5000)
    rec = traffic_record("domino_batch_batched4096") if full else None
    avg_s = kms * 1e-3 / max(1, launches)
    updates = info["sites"] * args.batched_sweeps
    g = golden("batch4096") if full else None
    match = None
    if g:
        ok = sum(1 for c in g["chains"] if b.hash(c["chain"]) == c["hash"])
        match = "%d/%d" % (ok, len(g["chains"]))
    h0 = b.hash(0)
    b.destroy()
    # the streaming formulation's bytes (every chain's packed state read and
    # written per colour step); the chains stay in LDS for the whole call, so
    # this is no bound: the VALU lane throughput is
    alg = 2.0 * info["state_bytes"] * 2 * args.batched_sweeps
    roof = alu_roofline(rec, avg_s) or {"bound": "alu", "achieved": None, "peak": round(VALU_PEAK_TOPS, 2),
                                        "unit": "T int32 lane-ops/s", "frac": None}
    roof.update({"traffic": rec["bytes_per_launch"] if rec else None, "launches": launches,
                 "hbm": hbm_figure(alg, rec, avg_s), "lds": lds_roofline(rec, avg_s), "valu": valu_summary(rec, avg_s)})
    roof["hbm"]["note"] = "streaming-formulation bytes; the chains stay in LDS, so the HBM figure is not a bound"
    return {"value": updates / el, "unit": "site-updates/s", "ms_per_step": el * 1e3,
            "chains": len(orders), "sweeps": args.batched_sweeps, "sites": info["sites"],
            "state_bytes": info["state_bytes"], "threads": threads, "workgroups": info["workgroups"],
            "autotune_probe_ms": round(probe_ms, 3), "launch_ms": round(kms, 3),
            "roofline": roof, "chain0_hash": h0, "oracle_match": match,
            "workload": "batched: %d domino chains, Aztec orders uniform in [16,512] (PCG64 seed 0x5EED), "
                        "two-periodic a=1 b=1/2, %d sweeps, seeds 0..%d, one graph-replayed persistent launch"
                        % (len(orders), args.batched_sweeps, len(orders) - 1)}


def run_served(tl, args, budget_mib):
    """Served form: six-vertex domain-wall requests, N uniform over
    {64,...,1024}, weights (1,1,sqrt 2) / (1,1,1) alternating as lazy Metropolis
    thresholds, 2000 sweeps, Poisson arrivals; admitted by a device-memory
    budget.  Requests the oracle has stored results for are compared with them."""
    from paper_1804_07250_amd import workloads
    from paper_1804_07250_amd.serving import Server
    reqs = workloads.serve_requests(args.served_requests, args.served_rate)
    sv = Server(budget_mib << 20, args.served_slots, tl.options(sweeps_per_launch=args.served_quantum))
    start = time.perf_counter()
    tickets = []
    for r in reqs:
        delay = r["arrival"] - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        dom = tl.domain(tl.TL_SIXVERTEX, n=r["N"])
        w = tl.weights(tl.TL_W_SIXVERTEX, *r["w2"])
        w.rule = tl.TL_METROPOLIS if r["metropolis"] else tl.TL_HEATBATH
        tickets.append((sv.submit(dom, w, r["seed"], args.served_sweeps), r))
    res = [(sv.wait(t, 600.0), r) for t, r in tickets]
    end = time.perf_counter()
    st = sv.stats()
    sv.destroy()
    lat = np.array([x["t_done"] - x["t_submit"] for x, _ in res]) * 1e3
    wait = np.array([x["t_start"] - x["t_submit"] for x, _ in res]) * 1e3
    ok = all(x["status"] == tl.TL_OK for x, _ in res)
    updates = sum((r["N"] - 1) ** 2 * args.served_sweeps for _, r in res)
    g = golden("served") if args.served_sweeps == 2000 else None
    match = None
    if g:
        by_seed = {x["seed"]: x for x in g["requests"]}
        hits = [(x, by_seed[r["seed"]]) for x, r in res if r["seed"] in by_seed]
        good = sum(1 for x, e in hits if x["hash"] == e["hash"] and x["scalar_now"] == e["scalar_now"])
        match = "%d/%d" % (good, len(hits))
    return {"value": updates / (end - start), "unit": "site-updates/s", "requests": len(res), "all_ok": ok,
            "oracle_match": match,
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3), "queue_wait_p99_ms": round(float(np.percentile(wait, 99)), 3),
            "span_s": round(end - start, 3), "budget_bytes": budget_mib << 20,
            "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"],
            "workload": "served: six-vertex DWBC, N uniform over {64,128,256,512,1024}, weights (1,1,sqrt2) and "
                        "(1,1,1) alternating (lazy Metropolis), %d sweeps per request, Poisson %.0f/s, %d requests, budget %d MiB, "
                        "%d slots, ticks of %d sweeps (x2 for one-bit jobs)"
                        % (args.served_sweeps, args.served_rate, len(res), budget_mib, args.served_slots,
                           args.served_quantum)}


def run_cftp(tl, args):
    """Exact samples by coupling from the past: the six-vertex DWBC square with
    (a,b,c) = (1,1,1) and the uniform Aztec diamond, seeds 0..k-1."""
    out = {}
    cases = [("sixv", tl.domain(tl.TL_SIXVERTEX, n=args.cftp_n), tl.weights(tl.TL_W_UNIFORM),
              (args.cftp_n - 1) ** 2),
             ("aztec", tl.domain(tl.TL_DOMINO, n=args.cftp_aztec), tl.weights(tl.TL_W_UNIFORM),
              2 * args.cftp_aztec ** 2 - 2 * args.cftp_aztec + 1)]
    # the oracle's stored samples of these cases (R and canonical hash)
    g = golden("cftp")
    stored = {(c["model"], c["n"], c["seed"]): c for c in g["cases"]} if g else {}
    checked = matched = 0
    for name, dom, w, sites in cases:
        secs, logs, total = [], [], 0
        model = "sixvertex" if name == "sixv" else "domino"
        for seed in range(args.cftp_samples):
            s = tl.Sampler(dom, w, seed)
            s.sync()
            t0 = time.perf_counter()
            info = s.cftp(30)
            secs.append(time.perf_counter() - t0)
            logs.append(info["log2_sweeps"])
            total += info["total_sweeps"]
            c = stored.get((model, dom.n, seed))
            if c:
                checked += 1
                matched += int(info["log2_sweeps"] == c["log2_sweeps"] and s.hash() == c["hash"])
            s.destroy()
        out[name] = {"seconds_per_sample": round(sum(secs) / len(secs), 4), "log2_sweeps": logs,
                     "site_updates_per_s": sites * total / sum(secs)}
    out["oracle_match"] = "%d/%d" % (matched, checked) if checked else None
    out["workload"] = ("coupling from the past: six-vertex DWBC %dx%d with (a,b,c) = (1,1,1) and the uniform "
                       "Aztec diamond of order %d, seeds 0..%d, doubling from 2 sweeps"
                       % (args.cftp_n, args.cftp_n, args.cftp_aztec, args.cftp_samples - 1))
    return out


def run_variants(tl, wl, args):
    """The plain domino workload under the random colour order, and the same
    sweeps on a square domain given by a mask (start T_min), each timed over
    args.steps jobs after one warm-up job."""
    out = {}
    side = args.domain_side
    legs = [("random_order", tl.domain(tl.TL_DOMINO, n=wl["n"]), 1, 2 * wl["n"] ** 2 - 2 * wl["n"] + 1),
            ("square_domain", tl.domain(tl.TL_DOMINO, mask=np.ones((side, side), dtype=np.uint8)), 0, None)]
    for name, dom, order, sites in legs:
        t_make = time.perf_counter()
        s = tl.Sampler(dom, tl.weights(tl.TL_W_UNIFORM), wl["seed"],
                       tl.options(obs_every=wl["obs_every"], obs_bin=wl["obs_bin"], colour_order=order))
        t_make = time.perf_counter() - t_make
        sites = s.info()[0]

        def job():
            s.reset(wl["seed"])
            s.sweep(wl["sweeps"])
            s.observables()
            return s.hash()

        job()
        s.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            digest = job()
        s.sync()
        el = time.perf_counter() - t0
        s.destroy()
        out[name] = {"value": sites * wl["sweeps"] * args.steps / el, "unit": "site-updates/s",
                     "ms_per_step": el / args.steps * 1e3, "sites": sites, "hash": digest,
                     "create_s": round(t_make, 3)}
        # the oracle's stored final tilings of the two variants
        if name == "random_order":
            g = golden("aztec2048r")
            same = g and (g["n"], g["seed"], g["sweeps"]) == (wl["n"], wl["seed"], wl["sweeps"])
        else:
            g = golden("square2048")
            same = g and (g["side"], g["seed"], g["sweeps"]) == (side, wl["seed"], wl["sweeps"])
        if same:
            out[name]["oracle_match"] = digest == g["hash"]
    out["workload"] = ("the plain domino job (%d sweeps, density bins, row hash) with a random colour per step on "
                       "the order-%d Aztec diamond, and with the fixed order on the %dx%d square domain (mask, "
                       "T_min start; create_s includes the host tileability pre-pass)"
                       % (wl["sweeps"], wl["n"], side, side))
    return out


def make_sampler(tl, wl, args):
    opt = tl.options(obs_every=wl["obs_every"], obs_bin=wl["obs_bin"], kernel=args.kernel,
                     sweeps_per_launch=args.sweeps_per_launch, tile_rows=args.tile_rows,
                     tile_groups=args.tile_groups)
    if wl["model"] == "domino":
        dom = tl.domain(tl.TL_DOMINO, n=wl["n"])
        w = tl.weights(tl.TL_W_UNIFORM)
    elif wl["model"] == "lozenge":
        dom = tl.domain(tl.TL_LOZENGE, a=wl["a"], b=wl["b"], c=wl["c"])
        w = tl.weights(tl.TL_W_VOLUME, *wl["q"])
    else:
        dom = tl.domain(tl.TL_SIXVERTEX, n=wl["n"])
        w = tl.weights(tl.TL_W_SIXVERTEX, *wl["w2"])
    return tl.Sampler(dom, w, wl["seed"], opt)


def describe(wl):
    if wl["model"] == "domino":
        return ("plain: domino tilings of the order-%d Aztec diamond, uniform, brick start, %d sweeps, seed %d, "
                "2 bits/face, %dx%d-face density bins every %d sweeps, row hash"
                % (wl["n"], wl["sweeps"], wl["seed"], wl["obs_bin"], wl["obs_bin"], wl["obs_every"]))
    if wl["model"] == "lozenge":
        return ("plain: lozenge tilings of the %dx%dx%d hexagon, q = %d/%d, empty-box start, %d sweeps, seed %d, "
                "1 bit/vertex, volume bins %dx%d every %d sweeps, row hash"
                % (wl["a"], wl["b"], wl["c"], wl["q"][0], wl["q"][1], wl["sweeps"], wl["seed"], wl["obs_bin"],
                   wl["obs_bin"], wl["obs_every"]))
    return ("plain: six-vertex model, domain-wall %dx%d, (a^2,b^2,c^2) = %s, h_min start, %d sweeps, seed %d, "
            "1 bit/face, c-vertex bins %dx%d every %d sweeps, row hash"
            % (wl["n"], wl["n"], wl["w2"], wl["sweeps"], wl["seed"], wl["obs_bin"], wl["obs_bin"], wl["obs_every"]))


def traffic_record(name):
    """HBM bytes per launch measured with rocprofv3 counters, if recorded for the
    current kernel source (profiles/<name>_traffic.json carries its hash)."""
    path = os.path.join(ROOT, "profiles", name + "_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for name in rec.get("sources", []):
        src = os.path.join(ROOT, "paper_1804_07250_amd", "csrc", name)
        if not os.path.exists(src):
            return None
        h.update(open(src, "rb").read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return rec


def lds_roofline(rec, avg_launch_s):
    """LDS bytes per launch (rocprofv3 SQ_INSTS_LDS_{LOAD,STORE,ATOMIC}_BANDWIDTH,
    64-byte units) over the live average launch time, against the LDS peak;
    the fraction of CU-cycles the LDS was busy, and of those the share stalled
    by bank conflicts (SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT)."""
    if not rec or "lds_bytes_per_launch" not in rec or avg_launch_s <= 0:
        return None
    achieved = rec["lds_bytes_per_launch"] / avg_launch_s / 1e9
    busy = rec["lds_active_cycles_per_launch"] / (256 * 2.4e9 * avg_launch_s)
    return {"achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s",
            "frac": round(achieved / LDS_PEAK_GBS, 4), "bytes_per_launch": rec["lds_bytes_per_launch"],
            "busy_frac": round(busy, 4),
            "bank_conflict_frac": round(rec["lds_bank_conflict_cycles_per_launch"] /
                                        max(1.0, rec["lds_active_cycles_per_launch"]), 4)}


def valu_summary(rec, avg_launch_s):
    """VALU use of a launch from rocprofv3 SQ counters: the share of SIMD cycles
    issuing VALU work (SQ_ACTIVE_INST_VALU over 256 CUs x 2.4 GHz x the live
    launch time) and the share of lanes active in it (SQ_THREAD_CYCLES_VALU /
    (SQ_ACTIVE_INST_VALU x 64))."""
    if not rec or "valu_active_per_launch" not in rec or avg_launch_s <= 0:
        return None
    return {"busy_frac": round(rec["valu_active_per_launch"] / (256 * 2.4e9 * avg_launch_s), 4),
            "lane_util": rec["valu_lane_util"]}


def plain_leg(tl, name, args, steps, warmup):
    """One plain workload timed over `steps` jobs (reset + sweeps + observables
    + hash) after `warmup` jobs.  Returns (figures, sampler figures)."""
    wl = WORKLOADS[name]
    s = make_sampler(tl, wl, args)
    sites, colours = s.info()

    def step():
        s.reset(wl["seed"])
        s.sweep(wl["sweeps"])
        if args.sweeps_only:
            s.sync()
            return None, None
        obs = s.observables()
        return obs, s.hash()

    import torch
    for _ in range(warmup):
        step()
    s.sync()
    s.kernel_time()          # discard warm-up launches
    s.set_timing(0 if args.no_timing else args.timing_period)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs, digest = None, None
    for i in range(steps):
        obs, digest = step()
        print("%s step %d done" % (name, i), file=sys.stderr, flush=True)
    s.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kms, launches, csteps, bpc = s.kernel_time()
    s.destroy()
    avg_s = kms * 1e-3 / max(1, launches)
    bytes_per_launch = bpc * csteps / max(1, launches)
    kname = ("domino" if wl["model"] == "domino" else "height") + ("_tiled" if args.kernel != 1 else "_streaming")
    rec = traffic_record("%s_%s" % (kname, name))
    g = golden(name)
    match = None
    if g and digest is not None:
        match = bool(digest == g["hash"] and obs["samples"] == g["samples"] and obs["scalar_sum"] == g["scalar_sum"]
                     and obs["bin_sum"].reshape(-1).tolist() == g["bin_sum"])
    return {"value": sites * wl["sweeps"] * steps / el, "ms_per_step": el / steps * 1e3, "sites": sites,
            "colours": colours, "hash": digest, "oracle_match": match, "kernel": kname,
            "kernel_ms": kms, "launches": launches, "avg_launch_s": avg_s,
            "bytes_per_launch": bytes_per_launch, "rec": rec, "workload": describe(wl), "el": el}


def run_models(tl, args):
    """The lozenge hexagon (q = 1999/2000, 2 x 10^4 sweeps) and the weighted
    six-vertex square (N = 1024, (1,1,sqrt 2), 2000 sweeps), each with the
    roofline that binds it (the VALU lane throughput of the bit-serial
    decisions) and its streaming-formulation HBM figure."""
    out = {}
    for name in ("hexagon1024", "sixv1024"):
        r = plain_leg(tl, name, args, args.model_steps, 1)
        roof = alu_roofline(r["rec"], r["avg_launch_s"]) or {"bound": "alu", "achieved": None,
                                                             "peak": round(VALU_PEAK_TOPS, 2),
                                                             "unit": "T int32 lane-ops/s", "frac": None}
        roof.update({"kernel": r["kernel"], "avg_launch_us": round(r["avg_launch_s"] * 1e6, 3),
                     "launches": r["launches"], "traffic": r["rec"]["bytes_per_launch"] if r["rec"] else None,
                     "hbm": hbm_figure(r["bytes_per_launch"], r["rec"], r["avg_launch_s"]),
                     "lds": lds_roofline(r["rec"], r["avg_launch_s"]),
                     "valu": valu_summary(r["rec"], r["avg_launch_s"])})
        out[name] = {"value": r["value"], "unit": "site-updates/s", "ms_per_step": r["ms_per_step"],
                     "sites": r["sites"], "hash": r["hash"], "oracle_match": r["oracle_match"],
                     "roofline": roof, "workload": r["workload"]}
    return out


# --------------------------------------------------------------------- CPU oracle

def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu": model, "nproc": avail, "cpu_count": os.cpu_count()}


def cpu_baseline(budget_s):
    """The serial oracle (one core) on the headline workload, resumed from its
    own stored states at sweeps 2500, 5000 and 7500 of the chain (oracle
    checkpoints, tests/golden/ckpt) and timed for about budget_s / 3 seconds
    from each: a sample spread over the chain, not its frozen first sweeps."""
    import oracle
    g = golden("aztec2048")
    wl = WORKLOADS["aztec2048"]
    n = wl["n"]
    sites = 2 * n * n - 2 * n + 1
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    ckpts = [m for m in (g or {}).get("marks", []) if m.get("checkpoint")]
    done, spent, parts = 0, 0.0, []
    for m in ckpts:
        path = os.path.join(ROOT, "tests", "golden", "ckpt", m["checkpoint"])
        if not os.path.exists(path):
            continue
        o = oracle.DominoOracle(n, thr, seed=wl["seed"])
        with np.load(path, allow_pickle=False) as z:
            o.load(z["export"])
        o.t = m["t"]
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < budget_s / len(ckpts) and o.t < wl["sweeps"]:
            o.sweep(4)
            k += 4
        el = time.perf_counter() - t0
        done += k
        spent += el
        parts.append("%d sweeps from sweep %d" % (k, m["t"]))
    out = {"unit": "site-updates/s", "cores": 1, "kind": "oracle", "host": host_cpu()}
    if done:
        out["value"] = sites * done / spent
        out["sample"] = ("serial C oracle on the order-2048 Aztec chain (seed 7), resumed from its own states: %s; "
                         "%.1f s" % (", ".join(parts), spent))
    else:   # no stored states: the chain's first sweeps (frozen, faster than the average)
        o = oracle.DominoOracle(n, thr, seed=wl["seed"])
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            o.sweep(8)
            done += 8
        spent = time.perf_counter() - t0
        out["value"] = sites * done / spent
        out["sample"] = "serial C oracle, first %d sweeps of the order-2048 Aztec chain, %.1f s" % (done, spent)
    if g:
        out["full_chain_value"] = g["site_updates_per_s"]
        out["full_chain_note"] = ("the same oracle over the whole 10^4-sweep chain (%.0f s) on the machine that "
                                  "stored the result: %s" % (g["wall_s"], g["host"]["cpu"]))
    return out


def _mt_chain(item):
    """One full chain of the batched workload in a worker process (oracle only)."""
    import oracle
    from fractions import Fraction
    i, n, sweeps = item
    thr = oracle.table_from_ratios(oracle.domino_ratios("two_periodic", 1, Fraction(1, 2)), False)
    o = oracle.DominoOracle(n, thr, seed=i)
    t0 = time.perf_counter()
    o.sweep(sweeps)
    return i, (2 * n * n - 2 * n + 1) * sweeps, time.perf_counter() - t0, oracle.canonical_hash(o.export())


def cpu_baseline_mt(max_procs):
    """Multi-process oracle figure ("oracle-mt"): independent chains of the
    batched workload (two-periodic, 5000 sweeps, seed = chain index), whole,
    one per process, over up to max_procs host cores; the chains are ones the
    oracle's stored results cover (orders near the median), so each result is
    also checked against them."""
    import multiprocessing as mp
    g = golden("batch4096")
    if not g:
        return None
    procs = max(1, min(max_procs, host_cpu()["nproc"] or 1))
    chains = sorted((c for c in g["chains"] if 200 <= c["order"] <= 330), key=lambda c: c["chain"])[:procs]
    items = [(c["chain"], c["order"], g["sweeps"]) for c in chains]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(items)) as pool:
        res = pool.map(_mt_chain, items)
    wall = time.perf_counter() - t0
    want = {c["chain"]: c["hash"] for c in chains}
    return {"value": sum(r[1] for r in res) / wall, "unit": "site-updates/s", "cores": len(items),
            "kind": "oracle-mt", "host": host_cpu(),
            "oracle_match": "%d/%d" % (sum(1 for r in res if r[3] == want[r[0]]), len(res)),
            "sample": "%d whole chains of the batched workload (orders %s, two-periodic a=1 b=1/2, %d sweeps), one "
                      "per process, %.1f s wall" % (len(items), [c["order"] for c in chains], g["sweeps"], wall)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    # the CPU oracle legs run first, before anything touches the GPU (the
    # multi-process one forks its workers)
    cpu = cpu_mt = None
    if (not args.no_cpu_baseline and not args.sweeps_only and not args.copy_calibration
            and args.workload == "aztec2048"):
        cpu = cpu_baseline(args.cpu_seconds)
        print("cpu baseline done", file=sys.stderr, flush=True)
        cpu_mt = cpu_baseline_mt(args.cpu_procs)
        print("cpu multi-process baseline done", file=sys.stderr, flush=True)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 5}))
        return
    import paper_1804_07250_amd as tl
    wl = WORKLOADS[args.workload]
    r = plain_leg(tl, args.workload, args, args.steps, args.warmup)
    if args.sweeps_only:
        print(json.dumps({"sweeps_only_s_per_step": r["el"] / args.steps, "kernel_ms": r["kernel_ms"],
                          "launches": r["launches"]}))
        return
    avg_s = r["avg_launch_s"]
    achieved = r["bytes_per_launch"] / avg_s / 1e9 if r["launches"] else 0.0
    rec = r["rec"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": rec["bytes_per_launch"] if rec else None,
            "kernel": r["kernel"], "avg_launch_us": round(avg_s * 1e6, 3), "launches": r["launches"],
            "algorithmic_bytes_per_launch": r["bytes_per_launch"],
            "lds": lds_roofline(rec, avg_s), "valu": valu_summary(rec, avg_s), "alu": alu_roofline(rec, avg_s)}
    out = {"metric": "site-updates/sec on 1 MI355X (plain vs batched vs served p50/p99), bit-exact",
           "value": r["value"], "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": r["workload"],
                      "sites": r["sites"], "colours": r["colours"], "sweeps": wl["sweeps"],
                      "kernel": "tiled" if args.kernel != 1 else "streaming",
                      "hash": r["hash"], "oracle_match": r["oracle_match"]},
           "roofline": roof}
    headline = args.workload == "aztec2048"
    if headline and not args.no_models:
        out["models"] = run_models(tl, args)
        print("models done", file=sys.stderr, flush=True)
    if not args.no_variants and wl["model"] == "domino":
        out["variants"] = run_variants(tl, wl, args)
        print("variants done", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = run_batched(tl, args)
        print("batched done", file=sys.stderr, flush=True)
    if not args.no_served:
        out["served"] = run_served(tl, args, args.served_budget_mib)
        print("served done", file=sys.stderr, flush=True)
        if args.served_tight_mib:
            out["served_budget_bound"] = run_served(tl, args, args.served_tight_mib)
            print("served (budget-bound) done", file=sys.stderr, flush=True)
    if not args.no_cftp:
        out["cftp"] = run_cftp(tl, args)
        print("cftp done", file=sys.stderr, flush=True)
    if cpu:
        out["cpu_baseline"] = cpu
    if cpu_mt:
        out["cpu_baseline_mt"] = cpu_mt
    print(json.dumps(out))


if __name__ == "__main__":
    main()
