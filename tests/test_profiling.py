"""The rocprofv3 summary tools and the bench's traffic lookup, on small
synthetic CSV files (no GPU): calibration against the copy kernel, the
dominant kernel's bytes per launch, and the source-hash guard that keeps a
stale counter file from being reported."""
import csv
import json
import os

import pytest

from paper_2207_08716_amd import profiling

SWEEP = "void ptk::(anonymous namespace)::k_sweep<double, 0, false, 0>(ptk::Geom, ptk::Coef, ptk::SweepPtrs<double>)"
SWEEP_NORMS = "void ptk::(anonymous namespace)::k_sweep<double, 0, true, 0>(ptk::Geom, ptk::Coef, ptk::SweepPtrs<double>)"
COPY = "ptk::(anonymous namespace)::k_copy(ptk::dvec2 const*, ptk::dvec2*, long)"


def _counters(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, (name, value) in enumerate(rows):
            w.writerow([d, name, counter, value])


def test_traffic_summary_calibrates_with_the_copy(tmp_path):
    n = 7
    pitch = 32
    copy_bytes = (n + 1) * (n + 1) * pitch * 8
    # the copy reads its bytes but the counter shows half of them (factor 2),
    # and writes them with factor 1; two dispatches of the sweep are averaged
    fetch = [(COPY, copy_bytes / 2 / 1024), (SWEEP, 1000.0), (SWEEP, 1200.0), (SWEEP_NORMS, 9e9)]
    write = [(COPY, copy_bytes / 1024), (SWEEP, 400.0), (SWEEP, 400.0), (SWEEP_NORMS, 9e9)]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _counters(fcsv, "FETCH_SIZE", fetch)
    _counters(wcsv, "WRITE_SIZE", write)
    out_json, out_md = tmp_path / "t.json", tmp_path / "t.md"
    profiling.traffic_summary(str(fcsv), str(wcsv), n, str(out_json), str(out_md), "cmd")
    rec = json.load(open(out_json))
    assert rec["kernel"] == "k_sweep<double, 0, false, 0>"
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["fetch_bytes"] == pytest.approx(1100.0 * 1024 * 2.0)
    assert rec["write_bytes"] == pytest.approx(400.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["a_eff_bytes"] == 25.0 * n ** 3 * 8
    assert "Dominant kernel k_sweep<double, 0, false, 0>" in open(out_md).read()


def test_trace_summary_rows(tmp_path):
    stats = tmp_path / "s.csv"
    with open(stats, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow([SWEEP, 3, 30000.0, 10000.0, 75.0, 9000.0, 11000.0, 1.0])
    out = tmp_path / "s.md"
    profiling.trace_summary(str(stats), str(out), "cmd")
    text = open(out).read()
    assert "| k_sweep<double, 0, false, 0> | 3 | 10.0 | 9.0 | 11.0 | 75.00 |" in text


def test_bench_reports_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    import bench
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    rec = {"n": 511, "kernel_source_sha": bench.kernel_source_sha(), "bytes_per_launch": 3.2e10}
    json.dump(rec, open(path, "w"))
    assert bench.measured_traffic(511) == 3.2e10
    assert bench.measured_traffic(255) is None              # other grid
    rec["kernel_source_sha"] = "0" * 16
    json.dump(rec, open(path, "w"))
    assert bench.measured_traffic(511) is None              # counters of another source
    os.remove(path)
    assert bench.measured_traffic(511) is None              # no counter file
