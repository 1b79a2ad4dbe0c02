"""Stored expected values of the benchmark workloads, computed by the oracle only.

TEST INFRASTRUCTURE ONLY: this script calls nothing but ``oracle/`` (and the
seeded input generators of ``paper_1804_07250_amd/workloads.py``, loaded from
their file so that no part of the HIP binding is imported).  It runs the
serial chains of the paper's RandomWalk (Section 2.2: a tiling, a seed and a
step count in, a tiling out) over the full length of each workload and writes
``tests/golden/<name>.json``:

  aztec2048    domino tilings of the order-2048 Aztec diamond, uniform weights,
               brick start, seed 7, 10^4 sweeps; horizontal-domino counts in
               bins of 64 x 64 faces sampled every 100 sweeps; the canonical
               hash after 2500, 5000, 7500 and 10^4 sweeps; oracle checkpoints
               (canonical exports) at the intermediate times
  aztec2048r   the same chain under the random colour choice per step
               (Section 2.2's RandomWalk draws the colour of every step)
  square2048   the same chain on the 2048 x 2048 square given as a mask, from
               its T_min (closed form, checked against the general algorithm)
  hexagon1024  lozenge tilings of the 1024^3 hexagon, q^volume with
               q = 1999/2000 (heat-bath), empty-box start, seed 11, 2 x 10^4
               sweeps; volume bins of 64 x 64 vertices every 200 sweeps; hashes
               every 5000 sweeps
  sixv1024     six-vertex model, domain-wall N = 1024, (a^2, b^2, c^2) =
               (1, 1, 2) heat-bath, seed 0, 2000 sweeps; c-vertex bins of
               64 x 64 every 100 sweeps (sixv1024u: (1, 1, 1), seed 1)
  batch4096    chains of the 4096-chain batched workload (Aztec orders from the
               seeded generator, two-periodic weights a = 1, b = 1/2, seed of
               chain i = i, 5000 sweeps): every 64th chain and the chains of
               the smallest and the largest order
  served       requests of the served six-vertex stream (2000 requests at
               200/s, lazy Metropolis, 2000 sweeps): the first ten requests of
               every size for each of the two weight sets
  cftp         exact samples by coupling from the past (Section 1.1.4, the
               CFTP host function of Section 2.2): the six-vertex domain-wall
               square N = 128 with (a, b, c) = (1, 1, 1) and the uniform Aztec
               diamond of order 64, seeds 0 and 1; the coalescence exponent R
               and the canonical hash of each sample

Usage: python -m oracle.goldens <name> [--jobs J] [--ckpt-dir DIR]

Every record also holds the wall time of the oracle run on the machine that
wrote it (for the CPU baseline beside the GPU figures).
"""
from __future__ import annotations

import argparse
import importlib.util
import json
import os
import platform
import subprocess
import time
from concurrent.futures import ProcessPoolExecutor
from fractions import Fraction

import numpy as np

import oracle

ROOT = os.path.dirname(oracle.HERE)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def workloads():
    """The seeded input generators, loaded from their own file."""
    path = os.path.join(ROOT, "paper_1804_07250_amd", "workloads.py")
    spec = importlib.util.spec_from_file_location("_tl_workloads", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def host():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count(), "threads_used": 1, "compiler": "gcc -O2 (serial)"}


def commit_of_oracle():
    try:
        out = subprocess.run(["git", "-C", ROOT, "log", "-1", "--format=%H", "--", "oracle"],
                             capture_output=True, text=True, check=True)
        return out.stdout.strip() or None
    except (OSError, subprocess.CalledProcessError):
        return None


def write(name, rec):
    os.makedirs(GOLDEN, exist_ok=True)
    rec["written_by"] = "python -m oracle.goldens %s" % name
    rec["oracle_commit"] = commit_of_oracle()
    rec["host"] = host()
    path = os.path.join(GOLDEN, name + ".json")
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(path + ".tmp", path)
    print("wrote", path, flush=True)


def save_checkpoint(ckpt_dir, name, t, export):
    """Canonical export after t sweeps, compressed (numpy, no pickle)."""
    if not ckpt_dir:
        return None
    os.makedirs(ckpt_dir, exist_ok=True)
    fn = "%s_t%d.npz" % (name, t)
    np.savez_compressed(os.path.join(ckpt_dir, fn), export=export, t=np.uint64(t))
    return fn


def run_plain(name, chain, sweeps, marks, ckpt_dir, sites):
    """Run one chain to `sweeps`, recording the hash at each mark."""
    out, t, t_all = [], 0, time.perf_counter()
    for m in list(marks) + [sweeps]:
        if m <= t:
            continue
        t0 = time.perf_counter()
        chain.sweep(m - t)
        el = time.perf_counter() - t0
        ex = chain.export()
        rec = {"t": m, "hash": oracle.canonical_hash(ex), "seconds": round(el, 3),
               "site_updates_per_s": sites * (m - t) / el}
        if m != sweeps:
            rec["checkpoint"] = save_checkpoint(ckpt_dir, name, m, ex)
        out.append(rec)
        print("%s: t=%d hash=%s %.1fs" % (name, m, rec["hash"][:16], el), flush=True)
        t = m
    return out, time.perf_counter() - t_all


def aztec2048(args):
    n, seed, sweeps, every, bin_ = 2048, 7, 10000, 100, 64
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    o = oracle.DominoOracle(n, thr, seed=seed, obs_every=every, bin_=bin_)
    sites = 2 * n * n - 2 * n + 1
    marks, wall = run_plain("aztec2048", o, sweeps, (2500, 5000, 7500), args.ckpt_dir, sites)
    write("aztec2048", {
        "workload": "domino tilings of the order-2048 Aztec diamond, uniform weights (T = 2^31), "
                    "all-horizontal brick start, Philox seed 7, 10^4 sweeps, fixed colour order",
        "model": "domino", "n": n, "seed": seed, "sweeps": sweeps, "obs_every": every, "bin": bin_,
        "sites": sites, "thresholds": [int(v) for v in thr],
        "hash": marks[-1]["hash"], "marks": marks,
        "samples": int(o.samples[0]), "scalar_sum": int(o.scalar_sum[0]),
        "bin_sum": [int(v) for v in o.bin_sum],
        "wall_s": round(wall, 2), "site_updates_per_s": sites * sweeps / wall})


def aztec2048r(args):
    """aztec2048 under the paper's random colour choice per step."""
    n, seed, sweeps, every, bin_ = 2048, 7, 10000, 100, 64
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    o = oracle.DominoOracle(n, thr, seed=seed, obs_every=every, bin_=bin_, random_colours=True)
    sites = 2 * n * n - 2 * n + 1
    marks, wall = run_plain("aztec2048r", o, sweeps, (2500, 5000, 7500), "", sites)
    write("aztec2048r", {
        "workload": "domino tilings of the order-2048 Aztec diamond, uniform weights (T = 2^31), "
                    "all-horizontal brick start, Philox seed 7, 10^4 sweeps, random colour per step",
        "model": "domino", "n": n, "seed": seed, "sweeps": sweeps, "obs_every": every, "bin": bin_,
        "colour_order": "random", "sites": sites, "thresholds": [int(v) for v in thr],
        "hash": marks[-1]["hash"], "marks": marks,
        "samples": int(o.samples[0]), "scalar_sum": int(o.scalar_sum[0]),
        "bin_sum": [int(v) for v in o.bin_sum],
        "wall_s": round(wall, 2), "site_updates_per_s": sites * sweeps / wall})


def square2048(args):
    """The plain domino job on the 2048 x 2048 square given as a mask, from
    T_min (closed form, oracle.square_tmin), embedded in the Aztec diamond of
    order 2048."""
    side, seed, sweeps, every, bin_ = 2048, 7, 10000, 100, 64
    thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
    o = oracle.DominoRegionOracle(np.ones((side, side), dtype=bool), thr, seed=seed, obs_every=every, bin_=bin_,
                                  init=None)
    o.load(oracle.square_tmin(side))
    sites = (side - 1) ** 2
    marks, wall = run_plain("square2048", o, sweeps, (2500, 5000, 7500), "", sites)
    write("square2048", {
        "workload": "domino tilings of the 2048 x 2048 square (a mask), uniform weights (T = 2^31), T_min start, "
                    "embedded in the Aztec diamond of order 2048, Philox seed 7, 10^4 sweeps, fixed colour order",
        "model": "domino", "side": side, "seed": seed, "sweeps": sweeps, "obs_every": every, "bin": bin_,
        "sites": sites, "thresholds": [int(v) for v in thr],
        "hash": marks[-1]["hash"], "marks": marks,
        "samples": int(o.samples[0]), "scalar_sum": int(o.scalar_sum[0]),
        "bin_sum": [int(v) for v in o.bin_sum],
        "wall_s": round(wall, 2), "site_updates_per_s": sites * sweeps / wall})


def hexagon1024(args):
    a = b = c = 1024
    seed, sweeps, every, bin_ = 11, 20000, 200, 64
    q = Fraction(1999, 2000)
    thr = oracle.table_from_ratios(oracle.lozenge_ratios(q), False)
    o = oracle.LozengeOracle(a, b, c, thr, seed=seed, obs_every=every, bin_=bin_)
    sites = 3 * a * a - 3 * a + 1   # interior vertices of the a = b = c hexagon
    marks, wall = run_plain("hexagon1024", o, sweeps, (5000, 10000, 15000), args.ckpt_dir, sites)
    write("hexagon1024", {
        "workload": "lozenge tilings of the 1024 x 1024 x 1024 hexagon, weight q^volume with q = 1999/2000 "
                    "(heat-bath), empty-box start, Philox seed 11, 2 x 10^4 sweeps, fixed colour order",
        "model": "lozenge", "a": a, "b": b, "c": c, "q": [1999, 2000], "seed": seed, "sweeps": sweeps,
        "obs_every": every, "bin": bin_, "sites": sites, "thresholds": [int(v) for v in thr],
        "hash": marks[-1]["hash"], "marks": marks,
        "samples": int(o.samples[0]), "scalar_sum": int(o.scalar_sum[0]),
        "bin_sum": [int(v) for v in o.bin_sum],
        "wall_s": round(wall, 2), "site_updates_per_s": sites * sweeps / wall})


def _sixv_plain(name, N, w2, seed, args):
    sweeps, every, bin_ = 2000, 100, 64
    thr = oracle.table_from_ratios(oracle.sixv_ratios(1, 1, w2[2]), False)
    o = oracle.SixVertexOracle(N, thr, seed=seed, obs_every=every, bin_=bin_)
    sites = (N - 1) ** 2
    marks, wall = run_plain(name, o, sweeps, (500, 1000, 1500), "", sites)
    write(name, {
        "workload": "six-vertex model with domain-wall boundary, N = %d, (a^2, b^2, c^2) = %s (heat-bath), "
                    "h_min start, Philox seed %d, 2000 sweeps, fixed colour order" % (N, list(w2), seed),
        "model": "sixvertex", "n": N, "w2": list(w2), "seed": seed, "sweeps": sweeps, "obs_every": every,
        "bin": bin_, "sites": sites, "thresholds": [int(v) for v in thr],
        "hash": marks[-1]["hash"], "marks": marks,
        "samples": int(o.samples[0]), "scalar_sum": int(o.scalar_sum[0]),
        "bin_sum": [int(v) for v in o.bin_sum],
        "wall_s": round(wall, 2), "site_updates_per_s": sites * sweeps / wall})


def sixv1024(args):
    _sixv_plain("sixv1024", 1024, (1, 1, 2), 0, args)


def sixv1024u(args):
    _sixv_plain("sixv1024u", 1024, (1, 1, 1), 1, args)


BATCH_SWEEPS = 5000


def _batch_chain(item):
    i, n = item
    thr = oracle.table_from_ratios(oracle.domino_ratios("two_periodic", 1, Fraction(1, 2)), False)
    o = oracle.DominoOracle(n, thr, seed=i)
    t0 = time.perf_counter()
    o.sweep(BATCH_SWEEPS)
    el = time.perf_counter() - t0
    return {"chain": i, "order": n, "seed": i, "hash": oracle.canonical_hash(o.export()),
            "seconds": round(el, 3), "sites": 2 * n * n - 2 * n + 1}


def batch4096(args):
    orders = workloads().batch_orders(4096)
    pick = set(range(0, 4096, 64))
    pick.add(int(np.argmin(orders)))
    pick.add(int(np.argmax(orders)))
    items = [(i, orders[i]) for i in sorted(pick)]
    thr = oracle.table_from_ratios(oracle.domino_ratios("two_periodic", 1, Fraction(1, 2)), False)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        chains = list(ex.map(_batch_chain, items))
    wall = time.perf_counter() - t0
    cpu = sum(c["seconds"] for c in chains)
    upd = sum(c["sites"] for c in chains) * BATCH_SWEEPS
    write("batch4096", {
        "workload": "batched domino chains: Aztec orders from the seeded generator (PCG64 seed 0x5EED, uniform "
                    "in [16, 512]), two-periodic edge weights a = 1, b = 1/2 (heat-bath), brick start, seed of "
                    "chain i = i, 5000 sweeps; every 64th chain and the chains of the smallest and largest order",
        "chains_total": 4096, "sweeps": BATCH_SWEEPS, "thresholds": [int(v) for v in thr],
        "chains": chains, "processes": args.jobs, "wall_s": round(wall, 2), "cpu_s": round(cpu, 2),
        "site_updates_per_s_per_core": upd / cpu})


SERVE_SWEEPS = 2000


def _served_request(r):
    c2 = int(r["w2"][2])
    thr = oracle.table_from_ratios(oracle.sixv_ratios(1, 1, c2), True)
    o = oracle.SixVertexOracle(r["N"], thr, metropolis=True, seed=r["seed"])
    t0 = time.perf_counter()
    o.sweep(SERVE_SWEEPS)
    el = time.perf_counter() - t0
    return {"request": r["seed"], "N": r["N"], "w2": list(r["w2"]), "metropolis": True, "seed": r["seed"],
            "hash": oracle.canonical_hash(o.export()), "scalar_now": o.observe()[0],
            "seconds": round(el, 3), "sites": (r["N"] - 1) ** 2}


def served(args):
    wl = workloads()
    reqs = wl.serve_requests(2000, 200.0)
    pick = []
    for N in wl.SERVE_SIZES:
        for parity in (0, 1):
            idx = [r for r in reqs if r["N"] == N and r["seed"] % 2 == parity][:10]
            pick.extend(idx)
    pick.sort(key=lambda r: -r["N"])          # longest first
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        res = list(ex.map(_served_request, pick))
    wall = time.perf_counter() - t0
    res.sort(key=lambda r: r["request"])
    cpu = sum(r["seconds"] for r in res)
    upd = sum(r["sites"] for r in res) * SERVE_SWEEPS
    write("served", {
        "workload": "served six-vertex requests: domain-wall N x N, N uniform over {64, 128, 256, 512, 1024}, "
                    "(a^2, b^2, c^2) = (1, 1, 2) for even and (1, 1, 1) for odd request indices, lazy "
                    "Metropolis thresholds, h_min start, 2000 sweeps, request seed = request index (stream of "
                    "2000 requests, PCG64 seed 0x5E4E); the first ten requests of each size and weight set",
        "sweeps": SERVE_SWEEPS, "requests": res, "processes": args.jobs, "wall_s": round(wall, 2),
        "cpu_s": round(cpu, 2), "site_updates_per_s_per_core": upd / cpu})


CFTP_CASES = [("sixvertex", 128, 0), ("sixvertex", 128, 1), ("domino", 64, 0), ("domino", 64, 1)]


def _cftp_case(case):
    model, n, seed = case
    if model == "sixvertex":
        thr = oracle.table_from_ratios(oracle.sixv_ratios(1, 1, 1), False)
        make = lambda init: oracle.SixVertexOracle(n, thr, seed=seed, init=init)
    else:
        thr = oracle.table_from_ratios(oracle.domino_ratios(), False)
        make = lambda init: oracle.DominoOracle(n, thr, seed=seed, init=init)
    t0 = time.perf_counter()
    R, sample = oracle.cftp(make, max_log2=30)
    el = time.perf_counter() - t0
    return {"model": model, "n": n, "seed": seed, "log2_sweeps": R, "hash": oracle.canonical_hash(sample),
            "seconds": round(el, 3)}


def cftp(args):
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=args.jobs) as ex:
        cases = list(ex.map(_cftp_case, CFTP_CASES))
    wall = time.perf_counter() - t0
    write("cftp", {
        "workload": "coupling from the past, uniform weights (every threshold 2^31), heat-bath, rounds "
                    "doubling from 2 sweeps with the draws of each time step fixed for all rounds: the "
                    "six-vertex domain-wall square N = 128 and the Aztec diamond of order 64, seeds 0 and 1",
        "cases": cases, "processes": args.jobs, "wall_s": round(wall, 2),
        "cpu_s": round(sum(c["seconds"] for c in cases), 2)})


JOBS = {"aztec2048": aztec2048, "aztec2048r": aztec2048r, "square2048": square2048, "hexagon1024": hexagon1024, "sixv1024": sixv1024, "sixv1024u": sixv1024u,
        "batch4096": batch4096, "served": served, "cftp": cftp}


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("name", choices=sorted(JOBS))
    p.add_argument("--jobs", type=int, default=2, help="worker processes for the chain lists")
    p.add_argument("--ckpt-dir", default=os.path.join(GOLDEN, "ckpt"),
                   help="where the intermediate oracle states go ('' for none)")
    args = p.parse_args()
    oracle.build(force=False)
    JOBS[args.name](args)


if __name__ == "__main__":
    main()
