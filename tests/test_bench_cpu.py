"""CPU checks of the benchmark's measurement helpers: the algorithmic bytes
per SpMV against the figures the measurement plan publishes for its
workloads, the byte-counter calibration (FETCH_SIZE / WRITE_SIZE scaled by
a plain copy of known size) and its tie to the kernel sources, and the
kernel-trace summary."""
import csv
import json
import os

import pytest

import bench

M3, NNZ3 = 256 ** 3, 7 * 256 ** 3 - 6 * 256 ** 2  # the 256^3 7-point stencil
M2, NNZ2 = 1 << 20, 16_086_387                     # R-MAT scale 20, duplicates merged


def test_alg_bytes_match_the_published_figures():
    # values + indices + pointer (or row indices) + x read once + y written once
    assert bench.alg_bytes("csr", M3, M3, NNZ3, 8, 8) == 1_740_111_876   # "1,740 MB"
    assert bench.alg_bytes("coo", M3, M3, NNZ3, 8, 8) == 2_141_192_192   # "2,141 MB"
    assert bench.alg_bytes("csr", M3, M3, NNZ3, 4, 4) == 1_137_704_964   # FP32 "1,138 MB"
    assert bench.alg_bytes("csr", M3, M3, NNZ3, 2, 4) == 903_610_372     # BF16 "904 MB"
    assert bench.alg_bytes("csc", M2, M2, NNZ2, 8, 8) == 214_008_168
    # the pointer is per row (CSR) or per column (CSC); beta != 0 reads y too
    assert bench.alg_bytes("csc", 10, 30, 7, 8, 8) - bench.alg_bytes("csr", 10, 30, 7, 8, 8) == 80
    assert bench.alg_bytes("csr", 10, 30, 7, 8, 8, beta0=False) - \
        bench.alg_bytes("csr", 10, 30, 7, 8, 8) == 80


def _counters(d, rows):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerows(rows)


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """Bytes per launch = the kernel's median reading times the factor that
    makes the largest copy of the run read 256 MiB; the record is used only
    while the kernel sources hash the same."""
    k = "void msrep::spmv_coo_seg<0, 4, true>(int const*)"
    cp = "__amd_rocclr_copyBuffer"
    _counters(tmp_path / "f", [(k, "FETCH_SIZE", 1000), (k, "FETCH_SIZE", 1200),
                               (k, "FETCH_SIZE", 1100), (cp, "FETCH_SIZE", 100),
                               (cp, "FETCH_SIZE", 131072)])   # the copy reads as 128 MiB
    _counters(tmp_path / "w", [(k, "WRITE_SIZE", 500), (cp, "WRITE_SIZE", 262144)])
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h1")
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), "spmv_coo_seg", "key/a", "cmd")
    rec = [json.loads(l) for l in open(tmp_path / "profiles" / "traffic.txt") if l.startswith("{")]
    assert len(rec) == 1
    assert rec[0]["fetch_bytes"] == 1100 * 1024 * 2 and rec[0]["write_bytes"] == 500 * 1024
    assert bench.load_traffic("key/a") == 1100 * 1024 * 2 + 500 * 1024
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h2")  # the kernels changed
    assert bench.load_traffic("key/a") is None
    # a second summary of the same key replaces the first
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), "spmv_coo_seg", "key/a", "cmd")
    rec = [json.loads(l) for l in open(tmp_path / "profiles" / "traffic.txt") if l.startswith("{")]
    assert [r["source_hash"] for r in rec] == ["h2"]


def test_pmc_summary_needs_the_kernel_and_the_copy(tmp_path, monkeypatch):
    _counters(tmp_path / "f", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072)])
    _counters(tmp_path / "w", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144)])
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    with pytest.raises(SystemExit):
        bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), "spmv_csr_seg", "k", "c")


def test_trace_summary(tmp_path, monkeypatch):
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["void msrep::(anonymous namespace)::spmv_coo_seg<0, 4, true>(int)", 3, 1500000,
                    500000, 90.0])
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])
        for g in range(50):  # 50 launch grids: the table keeps the 40 busiest
            w.writerow(["void msrep::k<%d>(int)" % g, 64 * (g + 1), 0, 1000 * (g + 1)])
    rec = {"metric": "m", "value": 1.0, "unit": "u", "ms_per_step": 2.0,
           "roofline": {"kernel": "spmv_coo_seg", "kernel_avg_us": 500.0, "achieved": 4000.0,
                        "frac": 0.5, "peak": 8000.0},
           "per_format": {"coo": {"kernels_us": {"spmv_coo_seg": 500.0}}}}
    (tmp_path / "b.json").write_text("log line\n" + json.dumps(rec) + "\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    bench.trace_summary(str(d), "t.txt", "the command", str(tmp_path / "b.json"))
    text = (tmp_path / "profiles" / "t.txt").read_text()
    assert "# command: the command" in text
    assert "void msrep::spmv_coo_seg<0, 4, true>" in text and "anonymous" not in text
    assert "the 40 of 50 with the most time" in text
    grid_rows = [l for l in text.splitlines() if l.startswith("void msrep::k<")]
    assert len(grid_rows) == 40 and grid_rows[0].startswith("void msrep::k<49>")
    assert "roofline kernel spmv_coo_seg, 500.00 us per launch" in text
