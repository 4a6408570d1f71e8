"""Host-side checks of bench.py (no GPU): the one-GPU rule, the rocprofv3
summary parser on small synthetic CSV files, and the counter-traffic loader's
digest check."""

import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stdout


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_rocprof_summary_scales_counters_by_the_copy(tmp_path):
    n = 4096
    sym_r = "void cssar::" + bench.kind_symbol("col_residual", n) + "(cssar::ColArgs)"
    sym_m = "void cssar::" + bench.kind_symbol("row_M", n) + "(cssar::RowArgs)"
    _write(str(tmp_path / "s" / "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[sym_r, 10, 1e6, 1e5, 60.0, 9e4, 1.1e5], [sym_m, 10, 7e5, 7e4, 40.0, 6e4, 8e4]])
    copy = "__amd_rocclr_copyBuffer"
    cal = bench.CAL_MIB * 1024  # KiB read and written by the calibration copy
    for d, counter, scale in (("f", "FETCH_SIZE", 2.0), ("w", "WRITE_SIZE", 1.0)):
        # the copy counts cal / scale: the summary multiplies kernel counts by scale
        _write(str(tmp_path / d / "run_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value"],
               [[copy, counter, cal / scale], [sym_r, counter, 1000.0], [sym_r, counter, 1000.0],
                [sym_m, counter, 500.0]])
    text = bench.rocprof_summary(str(tmp_path / "s"), str(tmp_path / "f"), str(tmp_path / "w"), n,
                                 ["cmd"])
    lines = {l.split()[1]: l.split() for l in text.splitlines() if l.strip().startswith("traffic ")}
    assert float(lines["col_residual"][2]) == pytest.approx(1000 * 1024 * 2.0)
    assert float(lines["col_residual"][3]) == pytest.approx(1000 * 1024 * 1.0)
    assert float(lines["row_M"][2]) == pytest.approx(500 * 1024 * 2.0)
    assert "kernel_sources_sha256 " + bench.kernel_source_digest() in text
    # durations only
    short = bench.rocprof_summary(str(tmp_path / "s"), "-", "-", n, ["cmd"], "x")
    assert sym_r[:60] in short and "traffic" not in short


def test_traffic_is_null_for_other_kernel_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.md"
    f.write_text("    traffic col_residual 1 2\n    kernel_sources_sha256 deadbeef\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic() is None
    f.write_text("    traffic col_residual 1 2\n    kernel_sources_sha256 %s\n" % bench.kernel_source_digest())
    assert bench.load_traffic() == {"col_residual": 3.0}
