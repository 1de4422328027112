"""Host-side measurement logic of bench.py (CPU only): bytes from request
counts by size, the counter summary built from rocprofv3 CSV files with its
calibration against known bytes, the traffic lookup keyed by the kernel
sources, and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys
import types

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_request_bytes_by_size():
    # 10 reads of 128 bytes, 4 of 64, 2 of 32, 1 other (counted as 64);
    # 6 writes of 64 bytes and 3 of 32
    c = {"TCC_EA0_RDREQ_sum": 17, "TCC_EA0_RDREQ_32B_sum": 2, "TCC_EA0_RDREQ_64B_sum": 4,
         "TCC_EA0_RDREQ_128B_sum": 10, "TCC_EA0_WRREQ_sum": 9, "TCC_EA0_WRREQ_64B_sum": 6}
    rd, wr = bench.request_bytes(c)
    assert rd == 10 * 128 + 4 * 64 + 2 * 32 + 1 * 64
    assert wr == 6 * 64 + 3 * 32


def _write_pass(d, rows):
    """A rocprofv3 counter-collection CSV: rows of (dispatch, kernel, counter, value, ns)."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "c_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for disp, name, ctr, val, ns in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": ctr, "Counter_Value": val,
                        "Start_Timestamp": 1000, "End_Timestamp": 1000 + ns})


def _reads(disp, name, n128, ns):
    return [(disp, name, "TCC_EA0_RDREQ_sum", n128, ns), (disp, name, "TCC_EA0_RDREQ_32B_sum", 0, ns),
            (disp, name, "TCC_EA0_RDREQ_64B_sum", 0, ns), (disp, name, "TCC_EA0_RDREQ_128B_sum", n128, ns)]


def _writes(disp, name, n64, ns):
    return [(disp, name, "TCC_EA0_WRREQ_sum", n64, ns), (disp, name, "TCC_EA0_WRREQ_64B_sum", n64, ns)]


def test_counter_summary_and_calibration(tmp_path, monkeypatch):
    """Exact request counts of the calibration stream give ratio 1 to its
    known bytes; a library kernel's per-dispatch bytes are the mean over its
    dispatches; the summary records the sources' digest."""
    rank = "void spg::k_rank_num<spg::PackedB<spg::SrMinPlusI32>, false>(spg::Operands, int)"
    w_rd, w_wr = str(tmp_path / "w_rd"), str(tmp_path / "w_wr")
    _write_pass(w_rd, _reads(1, rank, 1000, 2_000_000) + _reads(2, rank, 3000, 4_000_000))
    _write_pass(w_wr, _writes(1, rank, 500, 2_000_000) + _writes(2, rank, 700, 4_000_000))
    n = (1 << 30) // 4  # the calibration stream: 1 GiB read, 1 GiB written
    cal_rd = _reads(1, "void at::native::neg_kernel(float*)", 4 * n // 128, 1_000_000)
    cal_wr = _writes(1, "void at::native::neg_kernel(float*)", 4 * n // 64, 1_000_000)
    _write_pass(str(tmp_path / "c_rd"), cal_rd)
    _write_pass(str(tmp_path / "c_wr"), cal_wr)
    out = str(tmp_path / "sum.json")
    args = types.SimpleNamespace(counter_dirs=",".join([w_rd, w_wr, str(tmp_path / "c_rd"), str(tmp_path / "c_wr")]),
                                 counter_out=out, counter_workload="t", counter_command="cmd")
    rec = bench.run_counters(args)
    k = rec["kernels"]["k_rank_num<min_plus_i32>"]
    assert k["dispatches"] == 2
    assert k["read_bytes"] == pytest.approx(128 * 2000)
    assert k["write_bytes"] == pytest.approx(64 * 600)
    assert k["avg_ms"] == pytest.approx(3.0)
    assert rec["calibration_measured"]["calib_stream"]["read_ratio"] == pytest.approx(1.0)
    assert rec["calibration_measured"]["calib_stream"]["write_ratio"] == pytest.approx(1.0)
    assert rec["sources_sha256"] == bench.kernel_sources_digest()
    assert json.load(open(out))["kernels"].keys() == rec["kernels"].keys()


def test_traffic_lookup_follows_the_sources(tmp_path, monkeypatch):
    """The stored traffic is used only while the kernel sources match; a
    phase of several launches counts each; a two-semiring name sums both."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = bench.kernel_sources_digest()
    rec = {"sources_sha256": sha,
           "kernels": {"k_esc_num<plus_times_f32>": {"read_bytes": 10.0, "write_bytes": 5.0},
                       "k_dense_num_b<plus_times_f64>": {"read_bytes": 100.0, "write_bytes": 1.0},
                       "k_dense_num_b<min_plus_i32>": {"read_bytes": 200.0, "write_bytes": 2.0}}}
    (prof / "hbm_traffic_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: sha)
    assert bench.measured_traffic("k_esc_num<plus_times_f32>", "w", 9) == 135
    assert bench.measured_traffic("k_dense_num_b<plus_times_f64+min_plus_i32>", "w") == 303
    assert bench.measured_traffic("k_rank_num<min_plus_i32>", "w") is None
    rec["sources_sha256"] = "0" * 64
    (prof / "hbm_traffic_w.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("k_esc_num<plus_times_f32>", "w", 9) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
