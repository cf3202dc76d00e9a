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


COUNTER_HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp",
                  "LDS_Block_Size"]
CALLS = (("root_key_kernel", 1.0, 1000), ("resolve_kernel", 100.0, 2000), ("heavy_kernel", 300.0, 4000),
         ("heavy_kernel", 200.0, 3000), ("stats_kernel", 0.5, 500))


def _counter_rows(counter, copy_value, scale=1.0):
    """Two count calls (root_key, resolve, heavy x2, stats) and a 1 GiB
    copy; the second call's kernels read 10x what the first's read.  Each
    value is split over two rows (two cache instances) to check the sum."""
    rows, did, t = [], 1, 0
    for call in range(2):
        for name, v, ns in CALLS:
            val = v * scale * (10 if call else 1)
            lds = 131072 if name == "heavy_kernel" else 0
            rows.append([did, name, counter, val / 2, t, t + ns, lds])
            rows.append([did, name, counter, val / 2, t, t + ns, lds])
            did, t = did + 1, t + ns + 100
    rows.append([did, "__amd_rocclr_copyBuffer", counter, copy_value, t, t + 200000, 0])
    return rows


def test_summarize_counters_synthetic(tmp_path):
    """DRAM bytes per kernel of the last call, scaled by the copy (whose
    reads show as half their size: factor 2; writes as their size: factor
    1), the L2 hit share, and occupancy from a synthetic kernel trace."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", BENCH)
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rd, wr, l2 = tmp_path / "rd", tmp_path / "wr", tmp_path / "l2"
    _write(str(rd / "run_counter_collection.csv"), COUNTER_HEADER,
           _counter_rows("TCC_EA0_RDREQ_DRAM_32B", 2**30 / 32 / 2))
    _write(str(wr / "run_counter_collection.csv"), COUNTER_HEADER,
           _counter_rows("TCC_EA0_WRREQ_WRITE_DRAM_32B", 2**30 / 32, scale=0.1))
    _write(str(l2 / "run_counter_collection.csv"), COUNTER_HEADER,
           _counter_rows("TCC_HIT", 0.0, scale=3.0) + _counter_rows("TCC_MISS", 0.0, scale=1.0))
    td = tmp_path / "trace"
    trace, t = [], 0
    for call in range(2):
        for name, _, ns in CALLS:
            lds = 131072 if name == "heavy_kernel" else 0
            trace.append([name, t, t + ns, 52, 0, lds, 1024])
            t += ns + 100
    _write(str(td / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "VGPR_Count",
                                              "Accum_VGPR_Count", "LDS_Block_Size", "Workgroup_Size_X"], trace)
    out = tmp_path / "summary"
    r = _run("--summarize-counters", "--trace-dir", str(td), "--pmc-dir", str(rd), "--pmc-dir", str(wr),
             "--pmc-dir", str(l2), "--out", str(out), "--title", "t", "--cmd", "c")
    assert r.returncode == 0, r.stderr
    rec = json.load(open(str(out) + ".json"))
    assert rec["calibration"]["TCC_EA0_RDREQ_DRAM_32B"]["factor"] == pytest.approx(2.0)
    assert rec["calibration"]["TCC_EA0_WRREQ_WRITE_DRAM_32B"]["factor"] == pytest.approx(1.0)
    k = rec["kernels"]
    # only the last call counts: its heavy kernels read (300 + 200) * 10 units
    assert k["heavy_kernel[lds=131072]"]["n"] == 2
    assert k["heavy_kernel[lds=131072]"]["dram_read"] == pytest.approx(5000 * 32 * 2)
    assert k["heavy_kernel[lds=131072]"]["dram_write"] == pytest.approx(500 * 32)
    assert k["heavy_kernel[lds=131072]"]["ms"] == pytest.approx(0.007)
    assert k["heavy_kernel[lds=131072]"]["l2_hit_frac"] == pytest.approx(0.75)
    # a trace VGPR_Count of 52 is 104 registers (pairs on gfx950) -> 4 waves
    # by registers; 128 KB LDS -> 1 block of 16 waves per CU -> 4 waves per
    # SIMD too; resolve (no LDS) is limited by its registers
    assert k["heavy_kernel[lds=131072]"]["vgpr"] == pytest.approx(104)
    assert k["heavy_kernel[lds=131072]"]["theo_waves_simd"] == pytest.approx(4.0)
    assert k["heavy_kernel[lds=131072]"]["theo_limit"] == "lds"
    assert k["resolve_kernel"]["theo_waves_simd"] == pytest.approx(4.0)
    assert k["resolve_kernel"]["theo_limit"] == "vgpr"
    assert "__amd_rocclr_copyBuffer" not in k
    assert rec["heavy"]["traffic_bytes"] == pytest.approx(5000 * 32 * 2 + 500 * 32)
    assert len(rec["heavy"]["source_sha256"]) == 64
    md = open(str(out) + ".md").read()
    assert md.startswith("# t") and "| heavy_kernel[lds=131072] | 2 |" in md
    assert bench.theoretical_waves_per_simd(128, 0, 0, 256) == (4, "vgpr")
    assert bench.theoretical_waves_per_simd(24, 0, 65536, 256) == (2.0, "lds")
