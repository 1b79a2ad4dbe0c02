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
kernel, timed per launch by its own dispatch events) and the serial CPU
oracle's rate on a bounded sample of the same workload.
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
    p.add_argument("--sweeps-only", action="store_true",
                   help="time only the sweeps (for profiler runs); no JSON contract line")
    p.add_argument("--copy-calibration", type=int, default=0,
                   help="run a plain device copy of this many MiB (profiler calibration) and exit")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-served", action="store_true")
    p.add_argument("--batched-chains", type=int, default=4096)
    p.add_argument("--batched-sweeps", type=int, default=5000)
    p.add_argument("--served-requests", type=int, default=2000)
    p.add_argument("--served-rate", type=float, default=200.0)
    p.add_argument("--served-sweeps", type=int, default=2000)
    p.add_argument("--served-budget-mib", type=int, default=1024)
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


def run_batched(tl, args):
    """Batched form: Aztec chains of orders uniform in [16, 512], two-periodic
    weights a = 1, b = 1/2, seeds 0..count-1, args.batched_sweeps sweeps in one
    graph-replayed persistent launch; work-group size from the autotuner."""
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
    rec = traffic_record("domino_batch_batched4096") if (len(orders), args.batched_sweeps) == (4096, 5000) else None
    avg_s = kms * 1e-3 / max(1, launches)
    updates = info["sites"] * args.batched_sweeps
    h0 = b.hash(0)
    b.destroy()
    # algorithmic bytes: the packed state of every chain read and written per colour step
    alg = 2.0 * info["state_bytes"] * 2 * args.batched_sweeps
    return {"value": updates / el, "unit": "site-updates/s", "ms_per_step": el * 1e3,
            "chains": len(orders), "sweeps": args.batched_sweeps, "sites": info["sites"],
            "state_bytes": info["state_bytes"], "threads": threads, "workgroups": info["workgroups"],
            "autotune_probe_ms": round(probe_ms, 3), "launch_ms": round(kms, 3),
            "roofline": {"bound": "hbm", "achieved": round(alg / (kms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": rec["bytes_per_launch"] if rec else None, "launches": launches,
                         "lds": lds_roofline(rec, avg_s), "valu": valu_summary(rec, avg_s)},
            "chain0_hash": h0,
            "workload": "batched: %d domino chains, Aztec orders uniform in [16,512] (PCG64 seed 0x5EED), "
                        "two-periodic a=1 b=1/2, %d sweeps, seeds 0..%d, one graph-replayed persistent launch"
                        % (len(orders), args.batched_sweeps, len(orders) - 1)}


def run_served(tl, args):
    """Served form: six-vertex domain-wall requests, N uniform over
    {64,...,1024}, weights (1,1,sqrt 2) / (1,1,1) alternating as lazy Metropolis
    thresholds, 2000 sweeps, Poisson arrivals; admitted by a device-memory budget."""
    from paper_1804_07250_amd import workloads
    from paper_1804_07250_amd.serving import Server
    reqs = workloads.serve_requests(args.served_requests, args.served_rate)
    sv = Server(args.served_budget_mib << 20, args.served_slots, tl.options(sweeps_per_launch=args.served_quantum))
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
    ok = all(x["status"] == tl.TL_OK for x, _ in res)
    updates = sum((r["N"] - 1) ** 2 * args.served_sweeps for _, r in res)
    return {"value": updates / (end - start), "unit": "site-updates/s", "requests": len(res), "all_ok": ok,
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3), "span_s": round(end - start, 3),
            "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"],
            "workload": "served: six-vertex DWBC, N uniform over {64,128,256,512,1024}, weights (1,1,sqrt2) and "
                        "(1,1,1) alternating (lazy Metropolis), %d sweeps per request, Poisson %.0f/s, %d requests, budget %d MiB, "
                        "%d slots, ticks of %d sweeps (x4 for one-bit jobs)"
                        % (args.served_sweeps, args.served_rate, len(res), args.served_budget_mib, args.served_slots,
                           args.served_quantum)}


def run_cftp(tl, args):
    """Exact samples by coupling from the past: the six-vertex DWBC square with
    (a,b,c) = (1,1,1) and the uniform Aztec diamond, seeds 0..k-1."""
    out = {}
    cases = [("sixv", tl.domain(tl.TL_SIXVERTEX, n=args.cftp_n), tl.weights(tl.TL_W_UNIFORM),
              (args.cftp_n - 1) ** 2),
             ("aztec", tl.domain(tl.TL_DOMINO, n=args.cftp_aztec), tl.weights(tl.TL_W_UNIFORM),
              2 * args.cftp_aztec ** 2 - 2 * args.cftp_aztec + 1)]
    for name, dom, w, sites in cases:
        secs, logs, total = [], [], 0
        for seed in range(args.cftp_samples):
            s = tl.Sampler(dom, w, seed)
            s.sync()
            t0 = time.perf_counter()
            info = s.cftp(30)
            secs.append(time.perf_counter() - t0)
            logs.append(info["log2_sweeps"])
            total += info["total_sweeps"]
            s.destroy()
        out[name] = {"seconds_per_sample": round(sum(secs) / len(secs), 4), "log2_sweeps": logs,
                     "site_updates_per_s": sites * total / sum(secs)}
    out["workload"] = ("coupling from the past: six-vertex DWBC %dx%d with (a,b,c) = (1,1,1) and the uniform "
                       "Aztec diamond of order %d, seeds 0..%d, doubling from 2 sweeps"
                       % (args.cftp_n, args.cftp_n, args.cftp_aztec, args.cftp_samples - 1))
    return out


def run_variants(tl, wl, args):
    """The plain domino workload under the random colour order, and the same
    sweeps on a square domain given by a mask (start T_min), each timed over
    args.steps jobs after one warm-up job."""
    import numpy as np
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


def cpu_baseline(wl, budget_s):
    """The serial oracle on the same workload from its start, for a bounded
    number of sweeps (about budget_s seconds)."""
    import oracle
    from fractions import Fraction
    if wl["model"] == "domino":
        n = wl["n"]
        thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
        o = oracle.DominoOracle(n, thr, seed=wl["seed"])
        sites = 2 * n * n - 2 * n + 1
    elif wl["model"] == "lozenge":
        thr = oracle.table_from_ratios(oracle.lozenge_ratios(Fraction(*wl["q"])), False)
        o = oracle.LozengeOracle(wl["a"], wl["b"], wl["c"], thr, seed=wl["seed"])
        sites = len(o.sites())
        n = "%dx%dx%d" % (wl["a"], wl["b"], wl["c"])
    else:
        a2, b2, c2 = wl["w2"]
        thr = oracle.table_from_ratios(oracle.sixv_ratios(int(a2 ** 0.5), int(b2 ** 0.5), int(c2)), False)
        o = oracle.SixVertexOracle(wl["n"], thr, seed=wl["seed"])
        sites = (wl["n"] - 1) ** 2
        n = wl["n"]
    done = 0
    t0 = time.perf_counter()
    chunk = 1
    while time.perf_counter() - t0 < budget_s and done < wl["sweeps"]:
        o.sweep(chunk)
        done += chunk
        el = time.perf_counter() - t0
        if el < budget_s / 8:
            chunk *= 2
    el = time.perf_counter() - t0
    return {"value": sites * done / el, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": "serial C oracle, first %d of %d sweeps of the same %s chain (size %s, seed %d, from its "
                      "extremal start), %.1f s" % (done, wl["sweeps"], wl["model"], n, wl["seed"], el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
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

    for _ in range(args.warmup):
        step()
    s.sync()
    s.kernel_time()          # discard warm-up launches
    s.set_timing(0 if args.no_timing else args.timing_period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        obs, digest = step()
        print("step %d done" % i, file=sys.stderr, flush=True)
    s.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kms, launches, csteps, bpc = s.kernel_time()
    updates = sites * wl["sweeps"] * args.steps
    value = updates / el
    avg_ms = kms / max(1, launches)
    bytes_per_launch = bpc * csteps / max(1, launches)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    kname = ("domino" if wl["model"] == "domino" else "height") + ("_tiled" if args.kernel != 1 else "_streaming")
    rec = traffic_record("%s_%s" % (kname, args.workload))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": rec["bytes_per_launch"] if rec else None,
            "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 3), "launches": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "lds": lds_roofline(rec, avg_ms * 1e-3), "valu": valu_summary(rec, avg_ms * 1e-3)}
    out = {"metric": "site-updates/sec on 1 MI355X (plain vs batched vs served p50/p99), bit-exact",
           "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": describe(wl),
                      "sites": sites, "colours": colours, "sweeps": wl["sweeps"],
                      "kernel": "tiled" if args.kernel != 1 else "streaming",
                      "hash": digest},
           "roofline": roof}
    if args.sweeps_only:
        print(json.dumps({"sweeps_only_s_per_step": el / args.steps, "kernel_ms": kms, "launches": launches}))
        return
    s.destroy()
    if not args.no_variants and wl["model"] == "domino":
        out["variants"] = run_variants(tl, wl, args)
        print("variants done", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = run_batched(tl, args)
        print("batched done", file=sys.stderr, flush=True)
    if not args.no_served:
        out["served"] = run_served(tl, args)
        print("served done", file=sys.stderr, flush=True)
    if not args.no_cftp:
        out["cftp"] = run_cftp(tl, args)
        print("cftp done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
