"""Exact triangle counting through cover edges on AMD Instinct MI355X.

The computation lives in libtc (HIP kernels for gfx950, C ABI in
include/tc.h); this package is its Python binding plus the batched and
serving front ends.  Importing it loads nothing: the library is loaded on
first use and raises if it has not been built (see build.py).
"""
from .api import (CountResult, Graph, ListResult, TcError, Workspace, bfs_levels, build_csr, count,  # noqa: F401
                  count_edge_baseline, cover_edges, default_workspace, edge_support, from_host_csr, from_host_pairs,
                  list_triangles, profile_enable, profile_read, read_stats, select_root, validate, workspace_bytes)
from .batch import Batch, BatchResult, CapturedBatch, autotune, count_batch  # noqa: F401,E402
from .tune import autotune_count  # noqa: F401,E402
