"""The C-ABI library loads and exports every entry point of include/tc.h;
host-side logic that needs no GPU (workspace sizing, status strings)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2210_00389_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2210_00389_amd import build
        build.build()
    return _lib.load()


def header_functions():
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)))


def test_exports_match_header(lib):
    from paper_2210_00389_amd import _lib
    names = header_functions()
    assert names, "no functions found in tc.h"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tc_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n)


def test_status_strings(lib):
    from paper_2210_00389_amd import _lib
    for code in _lib.STATUS_NAMES:
        s = lib.tc_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.tc_status_string(12345).decode() == "unknown status"


def test_workspace_sizes(lib):
    from paper_2210_00389_amd import _lib
    for op in (_lib.OP_BUILD_CSR, _lib.OP_BFS_LEVELS, _lib.OP_COVER_EDGES, _lib.OP_COUNT,
               _lib.OP_EDGE_BASELINE, _lib.OP_VALIDATE, _lib.OP_COUNT_BATCH):
        small = lib.tc_workspace_bytes(op, 1000, 20000, 4)
        big = lib.tc_workspace_bytes(op, 100000, 2000000, 400)
        assert 0 < small <= big
        assert lib.tc_workspace_bytes(op, 0, 0, 0) > 0
    assert lib.tc_workspace_bytes(99, 10, 10, 0) == 0
    assert lib.tc_workspace_bytes(_lib.OP_COUNT, -1, 10, 0) == 0
    # R-MAT scale 24 (16.7 M vertices, ~0.52 G entries): the workspace (about
    # 115 B per entry, most of it the stream records of the heavy anchors)
    # stays well inside one GPU's 288 GB
    assert lib.tc_workspace_bytes(_lib.OP_COUNT, 1 << 24, 520_000_000, 0) < 64 * 2**30


def test_argument_errors_without_gpu(lib):
    """Argument checks run before any device work."""
    import ctypes
    from paper_2210_00389_amd import _lib
    assert lib.tc_count(None, -1, 0, None, None, None, None, None, 0, None) == -1
    csr = _lib.TcCsr(-1, 0, None, None)
    assert lib.tc_bfs_levels(ctypes.byref(csr), -1, 0, None, None, None, 0, None) == -1
    csr = _lib.TcCsr(1 << 31, 0, 1, None)
    assert lib.tc_count(ctypes.byref(csr), -1, 0, 1, None, None, None, None, 0, None) == -8
    csr = _lib.TcCsr(10, 20, 1, 1)
    t = ctypes.c_int64(0)
    # workspace too small
    assert lib.tc_count(ctypes.byref(csr), -1, 0, ctypes.byref(t), None, None, None, None, 16, None) == -2
    assert "workspace" in lib.tc_last_error().decode()
    # root out of range
    assert lib.tc_count(ctypes.byref(csr), 10, 0, ctypes.byref(t), None, None, None, None, 1 << 30, None) == -1
    # a degree could reach 2^29 (n - 1 and nnz / 2 both at least 2^29): refused
    # by the counting calls, before the workspace is looked at
    big = _lib.TcCsr((1 << 29) + 1, 1 << 30, 1, 1)
    assert lib.tc_count(ctypes.byref(big), -1, 0, ctypes.byref(t), None, None, None, None, 0, None) == -8
    assert "2^29" in lib.tc_last_error().decode()
    assert lib.tc_count_edge_baseline(ctypes.byref(big), 0, ctypes.byref(t), None, 0, None) == -8
    assert lib.tc_list_triangles(ctypes.byref(big), -1, 0, None, 0, ctypes.byref(t), None, None, None, 0, None) == -8
    # one entry fewer (nnz / 2 below 2^29), or one vertex fewer: past this check
    for n, nnz in (((1 << 29) + 1, (1 << 30) - 2), (1 << 29, 1 << 30)):
        ok = _lib.TcCsr(n, nnz, 1, 1)
        assert lib.tc_count(ctypes.byref(ok), -1, 0, ctypes.byref(t), None, None, None, None, 16, None) == -2


def test_batch_argument_errors_without_gpu(lib):
    """tc_count_batch rejects a declared graph size above TC_BATCH_MAX_N, a
    NULL batch and negative sizes before any device work."""
    import ctypes
    from paper_2210_00389_amd import _lib
    t = ctypes.c_int64(0)
    b = _lib.TcBatch(1, 70000, 10, 1, 1, 1, 70000)
    assert lib.tc_count_batch(ctypes.byref(b), None, 0, ctypes.byref(t), None, None, None, 1 << 30, None) == -8
    assert "65536" in lib.tc_last_error().decode()
    assert lib.tc_count_batch(None, None, 0, ctypes.byref(t), None, None, None, 0, None) == -1
    b = _lib.TcBatch(-1, 0, 0, None, None, None, 0)
    assert lib.tc_count_batch(ctypes.byref(b), None, 0, ctypes.byref(t), None, None, None, 0, None) == -1


def test_tuning_out_of_range_without_gpu(lib):
    """Out-of-range knobs of tc_tuning are refused before any device work."""
    import ctypes
    from paper_2210_00389_amd import _lib
    from paper_2210_00389_amd.batch import make_tuning
    csr = _lib.TcCsr(1000, 20000, 1, 1)
    t = ctypes.c_int64(0)
    for bad in (dict(light_max=33), dict(light_max=-1), dict(dn_light=-2), dict(item_log2=11), dict(item_log2=25),
                dict(bitmap_desc_words=2000), dict(bin0_mode=3), dict(bins_mode=-1), dict(bin0_max_desc=-2),
                dict(up_anchor_min=31), dict(up_anchor_min=-2), dict(degree_groups=3)):
        tu = make_tuning(dict(bad, small_max_n=-1))
        rc = lib.tc_count_tuned(ctypes.byref(csr), -1, 0, ctypes.byref(tu), ctypes.byref(t), None, None, None,
                                ctypes.c_void_p(256), 1 << 40, None)
        assert rc == -1 and "tuning" in lib.tc_last_error().decode(), bad
        rc = lib.tc_count_edge_baseline_tuned(ctypes.byref(csr), 0, ctypes.byref(tu), ctypes.byref(t),
                                              ctypes.c_void_p(256), 1 << 40, None)
        assert rc == -1, bad
    import pytest
    with pytest.raises(ValueError):
        make_tuning(dict(no_such_knob=1))
