"""Host-side checks of bench.py (no GPU): the one-GPU rule, the rocprofv3
summary parsers on small synthetic CSV files (the calibration copy, the roctx
ranges), and the counter-traffic loader's digest check."""

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


def test_calibration_takes_the_buffer_copy_over_larger_copies(tmp_path):
    # at 8192 x 8192 the scene set-up runs elementwise copies larger than the
    # 256 MiB calibration copy; the runtime's buffer copy is the calibration
    n = 8192
    sym_r = "void cssar::" + bench.kind_symbol("col_residual", n) + "(cssar::ColArgs)"
    _write(str(tmp_path / "s" / "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"],
           [[sym_r, 10, 1e6, 1e5, 100.0, 9e4, 1.1e5]])
    cal = bench.CAL_MIB * 1024
    big = "void at::native::elementwise_kernel<128, 4, direct_copy_kernel_cuda>"
    for d, counter in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        _write(str(tmp_path / d / "run_counter_collection.csv"),
               ["Kernel_Name", "Counter_Name", "Counter_Value"],
               [["__amd_rocclr_copyBuffer", counter, cal / 2.0], [big, counter, 4 * cal],
                [sym_r, counter, 1000.0]])
    text = bench.rocprof_summary(str(tmp_path / "s"), str(tmp_path / "f"), str(tmp_path / "w"), n,
                                 ["cmd"])
    assert "scale factor 2.0000" in text
    lines = {l.split()[1]: l.split() for l in text.splitlines() if l.strip().startswith("traffic ")}
    assert float(lines["col_residual"][2]) == pytest.approx(1000 * 1024 * 2.0)


def test_marker_summary_lists_ranges_by_total_time(tmp_path):
    _write(str(tmp_path / "m" / "run_marker_api_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [["cssar row M", 4, 2000.0, 500.0, 20.0, 400.0, 600.0, 1.0],
            ["cssar_ita_solve", 1, 8000.0, 8000.0, 80.0, 8000.0, 8000.0, 0.0]])
    text = bench.marker_summary(str(tmp_path / "m"), 4096, ["cmd"])
    rows = [l for l in text.splitlines() if l.startswith("| cssar")]
    assert rows[0].startswith("| cssar_ita_solve | 1 | 8.0 |")
    assert rows[1].startswith("| cssar row M | 4 | 2.0 | 0.5 |")
    assert "    cmd" in text
