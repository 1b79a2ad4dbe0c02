"""Host logic of bench.py, no GPU: the one-GPU refusal, the counter records in
profiles/ (their derived figures follow from the raw counters they store, and
a record stops counting once a kernel source it names changes), and the LDS and
VALU summaries built from them."""
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
