"""ctypes binding of libtc (include/tc.h): structs, signatures, loading.

Argument marshalling only -- every step of the method runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libtc.so")

TC_OK = 0
TC_VALIDATE = 1
TC_PER_VERTEX = 2

OP_BUILD_CSR = 1
OP_BFS_LEVELS = 2
OP_COVER_EDGES = 3
OP_COUNT = 4
OP_COUNT_BATCH = 5
OP_EDGE_BASELINE = 6
OP_VALIDATE = 7
OP_SELECT_ROOT = 8
MAX_ROOT_CANDIDATES = 64

STATUS_NAMES = {
    0: "TC_OK", -1: "TC_ERR_INVALID_ARG", -2: "TC_ERR_WORKSPACE", -3: "TC_ERR_NOT_SORTED",
    -4: "TC_ERR_DUPLICATE", -5: "TC_ERR_SELF_LOOP", -6: "TC_ERR_NOT_SYMMETRIC",
    -7: "TC_ERR_OUT_OF_RANGE", -8: "TC_ERR_TOO_LARGE", -9: "TC_ERR_HIP", -10: "TC_ERR_BAD_OFFSETS",
}

EXPORTS = [
    "tc_workspace_bytes", "tc_build_csr", "tc_validate_csr", "tc_bfs_levels", "tc_cover_edges",
    "tc_count", "tc_count_tuned", "tc_list_triangles", "tc_edge_support", "tc_select_root", "tc_count_edge_baseline",
    "tc_count_batch", "tc_count_batch_noalloc", "tc_noalloc_scratch_bytes",
    "tc_count_edge_baseline_tuned", "tc_status_string", "tc_last_error",
    "tc_profile_enable", "tc_profile_read", "tc_read_stats",
]


class TcCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p)]


class TcBatch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("total_vertices", ctypes.c_int64),
                ("total_nnz", ctypes.c_int64), ("vbase", ctypes.c_void_p),
                ("row_offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p),
                ("max_graph_vertices", ctypes.c_int32)]


TUNING_FIELDS = ("batch_block", "batch_piece", "batch_blocks_per_cu", "small_max_n", "small_max_nnz",
                 "light_max", "dn_light", "bitmap_member_words", "bitmap_desc_words", "item_log2", "bin0_mode",
                 "bins_mode", "twolevel_sparsity", "bin0_max_desc", "up_anchor_min", "degree_groups")


class TcTuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in TUNING_FIELDS]


class TcProfile(ctypes.Structure):
    _fields_ = [("num_stages", ctypes.c_int32), ("names", (ctypes.c_char * 24) * 32),
                ("ms", ctypes.c_float * 32)]


class TcStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("h", ctypes.c_int64),
                ("num_levels", ctypes.c_int64), ("stream_elems", ctypes.c_int64),
                ("light_tasks", ctypes.c_int64), ("heavy_items", ctypes.c_int64),
                ("heavy_desc", ctypes.c_int64), ("heavy_elems", ctypes.c_int64),
                ("heavy_builds", ctypes.c_int64), ("light_elems", ctypes.c_int64),
                ("bin_elems", ctypes.c_int64 * 4), ("bin_items", ctypes.c_int64 * 4),
                ("descriptors", ctypes.c_int64), ("twolevel_elems", ctypes.c_int64)]


_lib = None


def load(path: str | None = None):
    """Load libtc.so (built by paper_2210_00389_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libtc is not built ({p} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    P, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    c_int = ctypes.c_int
    lib.tc_workspace_bytes.argtypes = [c_int, i64, i64, i32]
    lib.tc_workspace_bytes.restype = sz
    lib.tc_build_csr.argtypes = [i64, i64, P, P, P, P, P, P, sz, P]
    lib.tc_build_csr.restype = c_int
    lib.tc_validate_csr.argtypes = [ctypes.POINTER(TcCsr), P, sz, P]
    lib.tc_validate_csr.restype = c_int
    lib.tc_bfs_levels.argtypes = [ctypes.POINTER(TcCsr), i64, u32, P, P, P, sz, P]
    lib.tc_bfs_levels.restype = c_int
    lib.tc_cover_edges.argtypes = [ctypes.POINTER(TcCsr), P, P, P, P, P, sz, P]
    lib.tc_cover_edges.restype = c_int
    lib.tc_count.argtypes = [ctypes.POINTER(TcCsr), i64, u32, P, P, P, P, P, sz, P]
    lib.tc_count.restype = c_int
    lib.tc_count_tuned.argtypes = [ctypes.POINTER(TcCsr), i64, u32, ctypes.POINTER(TcTuning), P, P, P, P, P, sz, P]
    lib.tc_count_tuned.restype = c_int
    lib.tc_list_triangles.argtypes = [ctypes.POINTER(TcCsr), i64, u32, P, i64, P, P, P, P, sz, P]
    lib.tc_list_triangles.restype = c_int
    lib.tc_select_root.argtypes = [ctypes.POINTER(TcCsr), i32, u32, P, P, P, P, sz, P]
    lib.tc_select_root.restype = c_int
    lib.tc_edge_support.argtypes = [ctypes.POINTER(TcCsr), P, i64, P, P]
    lib.tc_edge_support.restype = c_int
    lib.tc_count_edge_baseline.argtypes = [ctypes.POINTER(TcCsr), u32, P, P, sz, P]
    lib.tc_count_edge_baseline.restype = c_int
    lib.tc_count_edge_baseline_tuned.argtypes = [ctypes.POINTER(TcCsr), u32, ctypes.POINTER(TcTuning), P, P, sz, P]
    lib.tc_count_edge_baseline_tuned.restype = c_int
    lib.tc_count_batch.argtypes = [ctypes.POINTER(TcBatch), ctypes.POINTER(TcTuning), u32, P, P, P, P, sz, P]
    lib.tc_count_batch.restype = c_int
    lib.tc_count_batch_noalloc.argtypes = [ctypes.POINTER(TcBatch), ctypes.POINTER(TcTuning), u32, P, P, P, P]
    lib.tc_count_batch_noalloc.restype = c_int
    lib.tc_noalloc_scratch_bytes.argtypes = []
    lib.tc_noalloc_scratch_bytes.restype = sz
    lib.tc_status_string.argtypes = [c_int]
    lib.tc_status_string.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = []
    lib.tc_last_error.restype = ctypes.c_char_p
    lib.tc_profile_enable.argtypes = [c_int]
    lib.tc_profile_enable.restype = None
    lib.tc_profile_read.argtypes = [ctypes.POINTER(TcProfile)]
    lib.tc_profile_read.restype = c_int
    lib.tc_read_stats.argtypes = [P, ctypes.POINTER(TcStats), P]
    lib.tc_read_stats.restype = c_int
    if path is None:
        _lib = lib
    return lib
