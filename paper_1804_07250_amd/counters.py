"""Counter records for the roofline figures of bench.py.

Reads the CSV output of rocprofv3 ``--pmc`` runs (``counter_collection.csv``
under each run's ``-d`` folder) and writes ``profiles/<name>_traffic.json``:
HBM bytes per launch of one kernel from FETCH_SIZE and WRITE_SIZE, each scaled
by what the same counter reads for a device copy of known size, LDS bytes and
busy / bank-conflict cycles from the SQ LDS counters, and VALU use from the SQ
VALU counters.  The record carries a SHA-256 of the kernel sources it was
measured on; bench.py ignores it once they change.

    python -m paper_1804_07250_amd.counters summary DIR
    python -m paper_1804_07250_amd.counters record NAME --kernel 'domino_tiled_kernel<2, false>' \\
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-mib 256 \\
        [--lds DIR] [--valu DIR] [--trace DIR] [--sources domino.hip device_common.hpp] [--largest N]

Each DIR is the output folder of one rocprofv3 run (one counter block per run:
FETCH_SIZE and WRITE_SIZE cannot share a pass); --trace is a
``--kernel-trace`` run of the same workload, whose mean dispatch duration of
the kernel the record keeps (the launch time its figures are stated at).  The copy runs profile
``bench.py --copy-calibration MIB``, whose copies the runtime issues as
``__amd_rocclr_copyBuffer``.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
COPY_KERNEL = "__amd_rocclr_copyBuffer"
LDS_COUNTERS = ("SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH", "SQ_INSTS_LDS_ATOMIC_BANDWIDTH",
                "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE")
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU")


def kernel_label(name):
    """A kernel's name without its return type, namespaces and parameter list
    (template arguments kept): 'domino_tiled_kernel<2, false>'."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("tl::", "").strip()
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i].strip()
    return name


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of the columns %s in the counter CSV" % (names,))


def counter_values(folder):
    """{(kernel label, counter): [value per dispatch]} over every
    counter_collection.csv under folder."""
    files = sorted(glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % folder)
    out = defaultdict(list)
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                out[(kernel_label(_col(r, "Kernel_Name", "KERNEL_NAME")), _col(r, "Counter_Name", "COUNTER_NAME"))] \
                    .append(float(_col(r, "Counter_Value", "COUNTER_VALUE")))
    return out


def mean_of(values, kernel, counter, largest=None):
    """Mean of a counter over a kernel's dispatches, or over its `largest`
    largest values (a run that also launches the kernel on small probe inputs
    keeps only the full launches that way)."""
    v = values.get((kernel, counter))
    if not v:
        raise KeyError("no %s for kernel %s" % (counter, kernel))
    if largest:
        if len(v) < largest:
            raise KeyError("%d dispatches of %s for %s, %d asked for" % (len(v), kernel, counter, largest))
        v = sorted(v, reverse=True)[:largest]
    return statistics.fmean(v), len(v)


def trace_durations(folder):
    """{kernel label: [dispatch duration in us]} over every kernel_trace.csv
    under folder."""
    files = sorted(glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True))
    if not files:
        raise FileNotFoundError("no kernel_trace.csv under %s" % folder)
    out = defaultdict(list)
    for f in files:
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                start = int(_col(r, "Start_Timestamp", "START_TIMESTAMP"))
                end = int(_col(r, "End_Timestamp", "END_TIMESTAMP"))
                out[kernel_label(_col(r, "Kernel_Name", "KERNEL_NAME"))].append((end - start) / 1000.0)
    return out


def sources_sha256(sources):
    h = hashlib.sha256()
    for s in sources:
        with open(os.path.join(PKG, "csrc", s), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def make_record(kernel, fetch, write, copy_fetch, copy_write, copy_mib, sources, lds=None, valu=None, base=None,
                largest=None, trace=None):
    """The record as a dict.  fetch / write / copy_* / lds / valu are the
    counter_values() of the corresponding runs, trace the trace_durations()
    of a kernel-trace run; base supplies the fields kept from an existing
    record (workload, commands)."""
    rec = dict(base or {})
    rec.pop("trace_avg_launch_us", None)   # a trace time belongs to the runs it came with
    rec.pop("trace_launches", None)
    rec["kernel"] = kernel
    rec["sources"] = list(sources)
    rec["sources_sha256"] = sources_sha256(sources)
    f, launches = mean_of(fetch, kernel, "FETCH_SIZE", largest)
    w, _ = mean_of(write, kernel, "WRITE_SIZE", largest)
    copy_kib = copy_mib * 1024.0
    fs = copy_kib / mean_of(copy_fetch, COPY_KERNEL, "FETCH_SIZE")[0]
    ws = copy_kib / mean_of(copy_write, COPY_KERNEL, "WRITE_SIZE")[0]
    rec["bytes_per_launch"] = int(round(f * 1024 * fs + w * 1024 * ws))
    rec["fetch_kib_per_launch_raw"] = round(f, 1)
    rec["write_kib_per_launch_raw"] = round(w, 1)
    rec["fetch_scale"] = round(fs, 5)
    rec["write_scale"] = round(ws, 5)
    rec["launches_profiled"] = launches
    if lds is not None:
        raw = {c: round(mean_of(lds, kernel, c, largest)[0], 1) for c in LDS_COUNTERS}
        rec["lds_counters_raw"] = raw
        rec["lds_bytes_per_launch"] = int(round(64 * (raw["SQ_INSTS_LDS_LOAD_BANDWIDTH"] +
                                                      raw["SQ_INSTS_LDS_STORE_BANDWIDTH"] +
                                                      raw["SQ_INSTS_LDS_ATOMIC_BANDWIDTH"])))
        rec["lds_active_cycles_per_launch"] = raw["SQ_LDS_IDX_ACTIVE"]
        rec["lds_bank_conflict_cycles_per_launch"] = raw["SQ_LDS_BANK_CONFLICT"]
    if valu is not None:
        raw = {c: round(mean_of(valu, kernel, c, largest)[0], 1) for c in VALU_COUNTERS}
        rec["valu_counters_raw"] = raw
        rec["valu_active_per_launch"] = raw["SQ_ACTIVE_INST_VALU"]
        rec["valu_lane_util"] = round(raw["SQ_THREAD_CYCLES_VALU"] / (64.0 * raw["SQ_ACTIVE_INST_VALU"]), 4)
    if trace is not None:
        d = trace.get(kernel)
        if not d:
            raise KeyError("no dispatches of kernel %s in the kernel trace" % kernel)
        if largest:
            if len(d) < largest:
                raise KeyError("%d traced dispatches of %s, %d asked for" % (len(d), kernel, largest))
            d = sorted(d, reverse=True)[:largest]
        rec["trace_avg_launch_us"] = round(statistics.fmean(d), 3)
        rec["trace_launches"] = len(d)
    return rec


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = p.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summary", help="mean of every counter per kernel")
    s.add_argument("folder")
    r = sub.add_parser("record", help="write profiles/<name>_traffic.json")
    r.add_argument("name")
    r.add_argument("--kernel", required=True)
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        r.add_argument("--" + k, required=True)
    r.add_argument("--copy-mib", type=float, required=True)
    r.add_argument("--lds")
    r.add_argument("--valu")
    r.add_argument("--trace", help="rocprofv3 --kernel-trace folder of the same workload")
    r.add_argument("--sources", nargs="+")
    r.add_argument("--largest", type=int, help="use only the N dispatches with the largest value of each counter")
    r.add_argument("--out", help="record path (default profiles/<name>_traffic.json, whose workload, commands\n"
                                  "and sources a new record keeps)")
    a = p.parse_args(argv)
    if a.cmd == "summary":
        for (k, c), v in sorted(counter_values(a.folder).items()):
            print("%-60s %-30s n=%6d mean=%14.1f" % (k[:60], c, len(v), statistics.fmean(v)))
        return 0
    committed = os.path.join(ROOT, "profiles", a.name + "_traffic.json")
    out = a.out or committed
    base = {}
    for path in (out, committed):   # fields kept from an existing record
        if os.path.exists(path):
            with open(path) as fh:
                base = json.load(fh)
            break
    base.setdefault("workload", a.name.split("_")[-1])
    sources = a.sources or base.get("sources")
    if not sources:
        p.error("--sources is needed for a new record")
    rec = make_record(a.kernel, counter_values(a.fetch), counter_values(a.write), counter_values(a.copy_fetch),
                      counter_values(a.copy_write), a.copy_mib, sources,
                      counter_values(a.lds) if a.lds else None, counter_values(a.valu) if a.valu else None, base,
                      a.largest, trace_durations(a.trace) if a.trace else None)
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("%s: %d bytes per launch%s" % (out, rec["bytes_per_launch"],
                                         ", %d LDS bytes" % rec["lds_bytes_per_launch"] if "lds_bytes_per_launch"
                                         in rec else ""))
    return 0


if __name__ == "__main__":
    sys.exit(main())
