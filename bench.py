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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "aztec2048": dict(model="domino", n=2048, sweeps=10000, seed=7, obs_every=100, obs_bin=64),
    "aztec64": dict(model="domino", n=64, sweeps=1000, seed=1, obs_every=1, obs_bin=1),
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
    return p.parse_args()


def make_sampler(tl, wl, args):
    opt = tl.options(obs_every=wl["obs_every"], obs_bin=wl["obs_bin"], kernel=args.kernel,
                     sweeps_per_launch=args.sweeps_per_launch, tile_rows=args.tile_rows,
                     tile_groups=args.tile_groups)
    if wl["model"] == "domino":
        dom = tl.domain(tl.TL_DOMINO, n=wl["n"])
        w = tl.weights(tl.TL_W_UNIFORM)
    else:
        raise ValueError(wl["model"])
    return tl.Sampler(dom, w, wl["seed"], opt)


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


def cpu_baseline(wl, budget_s):
    """The serial oracle on the same workload from its start, for a bounded
    number of sweeps (about budget_s seconds)."""
    import oracle
    if wl["model"] != "domino":
        return None
    n = wl["n"]
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    o = oracle.DominoOracle(n, thr, seed=wl["seed"])
    sites = 2 * n * n - 2 * n + 1
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
            "sample": "serial C oracle, first %d of %d sweeps of the same chain (order %d, seed %d, from the "
                      "brick tiling), %.1f s" % (done, wl["sweeps"], n, wl["seed"], el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md, sharding)",
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
    kname = "domino_tiled" if args.kernel != 1 else "domino_streaming"
    rec = traffic_record("%s_%s" % (kname, args.workload))
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": rec["bytes_per_launch"] if rec else None,
            "kernel": kname, "avg_launch_us": round(avg_ms * 1e3, 3), "launches": launches,
            "algorithmic_bytes_per_launch": bytes_per_launch}
    out = {"metric": "site-updates/sec on 1 MI355X (plain vs batched vs served p50/p99), bit-exact",
           "value": value, "unit": "site-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "plain: domino tilings of the order-%d Aztec diamond, uniform, brick start, "
                                  "%d sweeps, seed %d, 2 bits/face, %dx%d-face density bins every %d sweeps, row hash"
                                  % (wl["n"], wl["sweeps"], wl["seed"], wl["obs_bin"], wl["obs_bin"],
                                     wl["obs_every"]),
                      "sites": sites, "colours": colours, "sweeps": wl["sweeps"],
                      "kernel": "tiled" if args.kernel != 1 else "streaming",
                      "hash": digest},
           "roofline": roof}
    if args.sweeps_only:
        print(json.dumps({"sweeps_only_s_per_step": el / args.steps, "kernel_ms": kms, "launches": launches}))
        return
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
