"""Host logic of bench.py, no GPU: the one-GPU refusal, the counter records in
profiles/ (their derived figures follow from the raw counters they store, and
a record stops counting once a kernel source it names changes), the LDS and
VALU summaries built from them, and the tool that writes the records from
rocprofv3 counter CSV output."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def committed_records():
    d = os.path.join(ROOT, "profiles")
    return sorted(f for f in os.listdir(d) if f.endswith("_traffic.json"))


@pytest.mark.parametrize("fname", committed_records())
def test_record_figures_follow_from_raw_counters(fname):
    rec = json.load(open(os.path.join(ROOT, "profiles", fname)))
    assert rec["sources"] and len(rec["sources_sha256"]) == 64
    assert rec["launches_profiled"] > 0 and len(rec["commands"]) >= 4
    kib = rec["fetch_kib_per_launch_raw"] * rec["fetch_scale"] + rec["write_kib_per_launch_raw"] * rec["write_scale"]
    assert abs(rec["bytes_per_launch"] - kib * 1024) <= 1e-4 * rec["bytes_per_launch"]
    # the copy calibration: FETCH_SIZE sees about half of a device copy's bytes
    assert 1.9 < rec["fetch_scale"] < 2.1 and rec["write_scale"] == 1.0
    if "lds_counters_raw" in rec:
        c = rec["lds_counters_raw"]
        units = c["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + c["SQ_INSTS_LDS_STORE_BANDWIDTH"] + c["SQ_INSTS_LDS_ATOMIC_BANDWIDTH"]
        assert rec["lds_bytes_per_launch"] == int(round(64 * units))
        assert rec["lds_active_cycles_per_launch"] == c["SQ_LDS_IDX_ACTIVE"]
        assert rec["lds_bank_conflict_cycles_per_launch"] == c["SQ_LDS_BANK_CONFLICT"] <= c["SQ_LDS_IDX_ACTIVE"]
    if "valu_counters_raw" in rec:
        c = rec["valu_counters_raw"]
        assert rec["valu_active_per_launch"] == c["SQ_ACTIVE_INST_VALU"]
        assert rec["valu_lane_util"] == round(c["SQ_THREAD_CYCLES_VALU"] / (64.0 * c["SQ_ACTIVE_INST_VALU"]), 4)
        assert 0.0 < rec["valu_lane_util"] <= 1.0


def write_tree(root, files, record):
    csrc = root / "paper_1804_07250_amd" / "csrc"
    csrc.mkdir(parents=True)
    (root / "profiles").mkdir()
    for name, text in files.items():
        (csrc / name).write_bytes(text)
    if record is not None:
        (root / "profiles" / "k_traffic.json").write_text(json.dumps(record))


def test_record_tracks_its_kernel_sources(tmp_path, monkeypatch):
    files = {"a.hip": b"kernel a\n", "b.hpp": b"header b\n"}
    h = hashlib.sha256(files["a.hip"] + files["b.hpp"]).hexdigest()
    rec = {"sources": ["a.hip", "b.hpp"], "sources_sha256": h, "bytes_per_launch": 10}
    write_tree(tmp_path, files, rec)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_record("k")["bytes_per_launch"] == 10
    assert bench.traffic_record("other") is None
    # order matters: the hash is over the sources in the order the record names
    (tmp_path / "profiles" / "k_traffic.json").write_text(json.dumps(dict(rec, sources=["b.hpp", "a.hip"])))
    assert bench.traffic_record("k") is None
    (tmp_path / "profiles" / "k_traffic.json").write_text(json.dumps(rec))
    (tmp_path / "paper_1804_07250_amd" / "csrc" / "b.hpp").write_bytes(b"header b, edited\n")
    assert bench.traffic_record("k") is None
    os.remove(tmp_path / "paper_1804_07250_amd" / "csrc" / "b.hpp")
    assert bench.traffic_record("k") is None


def test_lds_and_valu_summaries():
    rec = {"lds_bytes_per_launch": 3.0e8, "lds_active_cycles_per_launch": 1.8432e6,
           "lds_bank_conflict_cycles_per_launch": 4.608e5, "valu_active_per_launch": 3.6864e6,
           "valu_lane_util": 0.75}
    t = 25e-6                                   # 256 CUs x 2.4 GHz x 25 us = 1.536e7 CU-cycles
    lds = bench.lds_roofline(rec, t)
    assert lds["achieved"] == pytest.approx(12000.0)                 # 3e8 B / 25 us in GB/s
    assert lds["peak"] == pytest.approx(157286.4)                    # 256 B/clk x 256 CUs x 2.4 GHz
    assert lds["frac"] == pytest.approx(12000.0 / 157286.4, abs=1e-4)
    assert lds["busy_frac"] == pytest.approx(0.12)
    assert lds["bank_conflict_frac"] == pytest.approx(0.25)
    v = bench.valu_summary(rec, t)
    assert v == {"busy_frac": pytest.approx(0.24), "lane_util": 0.75}
    for bad in ({}, None):
        assert bench.lds_roofline(bad, t) is None and bench.valu_summary(bad, t) is None
    assert bench.lds_roofline(rec, 0.0) is None and bench.valu_summary(rec, -1.0) is None


def test_alu_roofline_is_busy_share_times_lane_use():
    # lane throughput = SQ_THREAD_CYCLES_VALU per launch / launch time against
    # 64 lanes x 256 CUs x 2.4 GHz; equal to VALU busy share x lane use
    active = 3.6864e6
    rec = {"valu_counters_raw": {"SQ_ACTIVE_INST_VALU": active, "SQ_THREAD_CYCLES_VALU": 0.75 * 64 * active},
           "valu_active_per_launch": active, "valu_lane_util": 0.75}
    t = 25e-6
    a = bench.alu_roofline(rec, t)
    assert a["bound"] == "alu" and a["peak"] == pytest.approx(39.32, abs=0.01)
    v = bench.valu_summary(rec, t)
    assert a["frac"] == pytest.approx(v["busy_frac"] * v["lane_util"], abs=1e-4)
    assert 0.0 < a["frac"] <= 1.0
    assert a["achieved"] == pytest.approx(a["frac"] * a["peak"], rel=1e-3)
    assert bench.alu_roofline({}, t) is None and bench.alu_roofline(rec, 0.0) is None


@pytest.mark.parametrize("fname", committed_records())
def test_committed_records_give_no_fraction_above_one(fname):
    # any roofline the bench builds from a committed record stays at or below
    # its peak (at the launch time the record's own kernel trace measured)
    rec = json.load(open(os.path.join(ROOT, "profiles", fname)))
    if "trace_avg_launch_us" not in rec:
        pytest.skip("record without its kernel trace time")
    t = rec["trace_avg_launch_us"] * 1e-6
    for fig in (bench.alu_roofline(rec, t), bench.lds_roofline(rec, t)):
        if fig is not None:
            assert 0.0 < fig["frac"] <= 1.0
    assert rec["bytes_per_launch"] / t / 1e9 <= bench.HBM_PEAK_GBS


def write_trace(folder, rows):
    """A rocprofv3-style kernel_trace.csv: rows of (kernel, start ns, end ns)."""
    d = folder / "host" / "123"
    d.mkdir(parents=True)
    with open(d / "123_kernel_trace.csv", "w") as fh:
        fh.write("Kind,Agent_Id,Queue_Id,Kernel_Id,Kernel_Name,Correlation_Id,Start_Timestamp,End_Timestamp\n")
        for i, (k, s, e) in enumerate(rows):
            fh.write('KERNEL_DISPATCH,1,1,%d,"%s",%d,%d,%d\n' % (i, k, i, s, e))
    return str(folder)


def write_counters(folder, rows):
    """A rocprofv3-style counter_collection.csv: rows of (kernel, counter, value)."""
    d = folder / "host" / "123"
    d.mkdir(parents=True)
    with open(d / "123_counter_collection.csv", "w") as fh:
        fh.write("Correlation_Id,Dispatch_Id,Agent_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            fh.write('%d,%d,1,"%s",%s,%r\n' % (i, i, k, c, v))
    return str(folder)


def test_counter_tool_builds_the_record(tmp_path):
    from paper_1804_07250_amd import counters
    k = "void tl::domino_tiled_kernel<2, false>(unsigned int const*, unsigned int*, unsigned long, int)"
    assert counters.kernel_label(k) == "domino_tiled_kernel<2, false>"
    assert counters.kernel_label("(anonymous namespace)::f<(x)>(int)") == "f<(x)>"
    copy = "__amd_rocclr_copyBuffer"
    fetch = write_counters(tmp_path / "f", [(k, "FETCH_SIZE", 1000.0), (k, "FETCH_SIZE", 1002.0),
                                            ("other_kernel", "FETCH_SIZE", 5.0)])
    write = write_counters(tmp_path / "w", [(k, "WRITE_SIZE", 500.0), (k, "WRITE_SIZE", 500.0)])
    cf = write_counters(tmp_path / "cf", [(copy, "FETCH_SIZE", 131072.0)] * 5)
    cw = write_counters(tmp_path / "cw", [(copy, "WRITE_SIZE", 262144.0)] * 5)
    lds = write_counters(tmp_path / "l", [(k, c, v) for c, v in (
        ("SQ_INSTS_LDS_LOAD_BANDWIDTH", 100.0), ("SQ_INSTS_LDS_STORE_BANDWIDTH", 20.0),
        ("SQ_INSTS_LDS_ATOMIC_BANDWIDTH", 4.0), ("SQ_LDS_BANK_CONFLICT", 30.0), ("SQ_LDS_IDX_ACTIVE", 120.0),
        ("SQ_INSTS_LDS", 9.0))])
    valu = write_counters(tmp_path / "v", [(k, "SQ_INSTS_VALU", 10.0), (k, "SQ_ACTIVE_INST_VALU", 10.0),
                                           (k, "SQ_THREAD_CYCLES_VALU", 480.0)])
    trace = write_trace(tmp_path / "t", [(k, 1000, 26000), (k, 30000, 54000), ("other_kernel", 0, 5)])
    out = tmp_path / "rec.json"
    rc = counters.main(["record", "x_aztec9", "--kernel", "domino_tiled_kernel<2, false>", "--fetch", fetch,
                        "--write", write, "--copy-fetch", cf, "--copy-write", cw, "--copy-mib", "256",
                        "--lds", lds, "--valu", valu, "--trace", trace, "--sources", "domino.hip",
                        "device_common.hpp", "--out", str(out)])
    assert rc == 0
    rec = json.load(open(out))
    assert rec["trace_avg_launch_us"] == 24.5 and rec["trace_launches"] == 2
    assert rec["launches_profiled"] == 2 and rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["bytes_per_launch"] == (1001 * 2 + 500) * 1024
    assert rec["lds_bytes_per_launch"] == 124 * 64
    assert rec["lds_bank_conflict_cycles_per_launch"] == 30.0 and rec["lds_active_cycles_per_launch"] == 120.0
    assert rec["valu_lane_util"] == 0.75 and rec["workload"] == "aztec9"
    h = hashlib.sha256()
    for s in ("domino.hip", "device_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1804_07250_amd", "csrc", s), "rb").read())
    assert rec["sources_sha256"] == h.hexdigest()
    # probe launches of the same kernel are left out with largest=N
    probe = write_counters(tmp_path / "p", [(k, "FETCH_SIZE", 7.0), (k, "FETCH_SIZE", 1000.0), (k, "FETCH_SIZE", 3.0),
                                            (k, "FETCH_SIZE", 1002.0)])
    assert counters.mean_of(counters.counter_values(probe), "domino_tiled_kernel<2, false>", "FETCH_SIZE", 2) == (1001.0, 2)
    with pytest.raises(KeyError):
        counters.mean_of(counters.counter_values(probe), "domino_tiled_kernel<2, false>", "FETCH_SIZE", 5)
    with pytest.raises(KeyError):
        counters.make_record("missing_kernel", counters.counter_values(fetch), counters.counter_values(write),
                             counters.counter_values(cf), counters.counter_values(cw), 256, ["domino.hip"])
