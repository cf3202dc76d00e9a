"""Host-side parts of bench.py, no GPU: the single-GPU guard and the two
summarisers that turn rocprofv3 CSV output into the files kept under
profiles/ (checked on small synthetic CSVs whose totals are worked by hand).
"""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _run(*args):
    return subprocess.run([sys.executable, BENCH, *args], capture_output=True, text=True, timeout=120)


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


COUNTER_HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _counter_rows(counter, calls, copy_kib):
    """Two count calls (root_key, resolve, heavy x2, stats) and a 1 GiB copy;
    the kernel of the second call reads 10x what the first reads."""
    rows, did, t = [], 1, 0
    for call in range(2):
        for name, kib, ns in (("root_key_kernel", 1.0, 1000), ("resolve_kernel", 100.0, 2000),
                              ("heavy_kernel", 300.0, 4000), ("heavy_kernel", 200.0, 3000),
                              ("stats_kernel", 0.5, 500)):
            val = kib * (10 if call else 1)
            rows.append([did, name, counter, val, t, t + ns])
            did, t = did + 1, t + ns + 100
    rows.append([did, "__amd_rocclr_copyBuffer", counter, copy_kib, t, t + 200000])
    return rows


def test_summarize_kernels_synthetic(tmp_path):
    fd, wd = tmp_path / "fetch", tmp_path / "write"
    # the copy's 1 GiB reads show as 0.5 GiB of FETCH_SIZE (factor 2), its
    # writes as 1 GiB of WRITE_SIZE (factor 1)
    _write(str(fd / "run_counter_collection.csv"), COUNTER_HEADER, _counter_rows("FETCH_SIZE", 2, 524288.0))
    _write(str(wd / "run_counter_collection.csv"), COUNTER_HEADER, _counter_rows("WRITE_SIZE", 2, 1048576.0))
    out = tmp_path / "summary"
    r = _run("--summarize-kernels", "--fetch-dir", str(fd), "--write-dir", str(wd), "--out", str(out),
             "--title", "t", "--cmd", "c")
    assert r.returncode == 0, r.stderr
    rec = json.load(open(str(out) + ".json"))
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]
    # only the last call counts: its heavy kernel read (300 + 200) * 10 KiB
    assert k["heavy_kernel"]["dispatches"] == 2
    assert k["heavy_kernel"]["fetch_bytes"] == pytest.approx(5000 * 1024 * 2)
    assert k["heavy_kernel"]["write_bytes"] == pytest.approx(5000 * 1024 * 1)
    assert k["heavy_kernel"]["ms"] == pytest.approx(0.007)
    assert k["resolve_kernel"]["fetch_bytes"] == pytest.approx(1000 * 1024 * 2)
    assert "__amd_rocclr_copyBuffer" not in k
    total_kib = (1 + 100 + 300 + 200 + 0.5) * 10
    assert rec["bytes"] == pytest.approx(total_kib * 1024 * 3)
    assert rec["kernel_ms"] == pytest.approx((1000 + 2000 + 4000 + 3000 + 500) / 1e6)
    md = open(str(out) + ".md").read()
    assert md.startswith("# t") and "| heavy_kernel | 2 |" in md


def test_summarize_heavy_stage_synthetic(tmp_path):
    """Heavy-stage record: per call the four bin kernels' FETCH_SIZE and
    WRITE_SIZE (KiB) summed and scaled by the copy's factors; traffic is the
    mean over the calls after the first."""
    fd, wd, td = tmp_path / "fetch", tmp_path / "write", tmp_path / "trace"
    rows_f, rows_w, did = [], [], 1
    for call, kib in enumerate((100.0, 200.0, 300.0)):
        for b in range(4):
            rows_f.append([did, "heavy_kernel", "FETCH_SIZE", kib, 0, 1])
            rows_w.append([did, "heavy_kernel", "WRITE_SIZE", kib / 10, 0, 1])
            did += 1
    rows_f.append([did, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0, 0, 1])
    rows_w.append([did, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0, 0, 1])
    _write(str(fd / "run_counter_collection.csv"), COUNTER_HEADER, rows_f)
    _write(str(wd / "run_counter_collection.csv"), COUNTER_HEADER, rows_w)
    _write(str(td / "run_kernel_stats.csv"), ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [["heavy_kernel", 8, 8000000, 1000000, 90.0], ["resolve_kernel", 2, 800000, 400000, 10.0]])
    trace = []
    for call in range(2):
        base = call * 10_000_000
        for b in range(4):  # bins in sequence, 1 ms each
            trace.append(["heavy_kernel", base + b * 1_000_000, base + (b + 1) * 1_000_000])
    _write(str(td / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    out = tmp_path / "heavy"
    r = _run("--summarize", "--trace-dir", str(td), "--fetch-dir", str(fd), "--write-dir", str(wd),
             "--out", str(out), "--title", "t", "--cmd", "c")
    assert r.returncode == 0, r.stderr
    rec = json.load(open(str(out) + ".json"))
    assert rec["heavy_span_ms"] == pytest.approx([4.0, 4.0])
    assert rec["fetch_bytes_per_launch"] == pytest.approx([4 * k * 1024 * 2 for k in (100, 200, 300)])
    assert rec["write_bytes_per_launch"] == pytest.approx([4 * k / 10 * 1024 for k in (100, 200, 300)])
    mean_after_first = (4 * 250 * 1024 * 2) + (4 * 25 * 1024)
    assert rec["traffic_bytes"] == pytest.approx(mean_after_first)
    assert len(rec["source_sha256"]) == 64
