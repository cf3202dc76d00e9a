"""Batched counting: many small graphs per tc_count_batch call.

A :class:`Batch` is the concatenated device CSR of the ``tc_batch`` ABI:
``vbase`` (int64, G+1 vertex bases), global ``row_offsets`` (int64) and
``cols`` holding local vertex ids (int32, < 65536).  :func:`count_batch`
runs the library's two kernels; :class:`CapturedBatch` records that call
once in a CUDA/HIP graph and replays it; :func:`autotune` times the tuning
knobs of the counting kernel on a given batch and keeps the fastest.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .api import TcError, Workspace, _check, _on_stream, _ptr, _stream, build_csr, default_workspace, workspace_bytes

MAX_N = 65536


@dataclass
class Batch:
    vbase: torch.Tensor        # int64 [G+1]
    row_offsets: torch.Tensor  # int64 [sum n + 1], positions in cols
    cols: torch.Tensor         # int32 [sum nnz], local ids
    sizes: list = field(default_factory=list)  # per graph (n, nnz)

    @property
    def num_graphs(self) -> int:
        return int(self.vbase.numel()) - 1

    @property
    def total_vertices(self) -> int:
        return int(self.row_offsets.numel()) - 1

    @property
    def total_nnz(self) -> int:
        return int(self.cols.numel())

    @property
    def total_edges(self) -> int:
        return self.total_nnz // 2

    def tc(self, max_graph_vertices: int | None = None) -> L.TcBatch:
        mx = max((n for n, _ in self.sizes), default=0) if max_graph_vertices is None else max_graph_vertices
        return L.TcBatch(self.num_graphs, self.total_vertices, self.total_nnz,
                         self.vbase.data_ptr(), self.row_offsets.data_ptr(),
                         self.cols.data_ptr() if self.total_nnz else None, mx)

    @staticmethod
    def from_graphs(graphs, device="cuda", ws: Workspace | None = None, max_n: int = MAX_N) -> "Batch":
        """Concatenate raw graphs (graphgen.Graph: n, src, dst) into one
        batch: the union is built as one CSR by tc_build_csr (vertex ids of
        graph g shifted by its base), then columns are made local.  Graphs
        above `max_n` vertices are refused (the library's limit is MAX_N;
        a larger `max_n` lets a caller hand the library an oversize graph,
        which it flags instead of counting)."""
        ns = np.array([g.n for g in graphs], dtype=np.int64)
        if (ns > max_n).any():
            raise ValueError(f"batched graphs must have at most {max_n} vertices")
        vb = np.zeros(len(graphs) + 1, dtype=np.int64)
        np.cumsum(ns, out=vb[1:])
        total = int(vb[-1])
        src = np.concatenate([np.asarray(g.src, dtype=np.int64) + vb[i] for i, g in enumerate(graphs)]
                             or [np.zeros(0, np.int64)])
        dst = np.concatenate([np.asarray(g.dst, dtype=np.int64) + vb[i] for i, g in enumerate(graphs)]
                             or [np.zeros(0, np.int64)])
        if total >= 2**31:
            raise ValueError("batch too large for int32 ids")
        dev = torch.device(device)
        s = torch.from_numpy(src.astype(np.int32)).to(dev)
        d = torch.from_numpy(dst.astype(np.int32)).to(dev)
        G = build_csr(total, s, d, ws=ws)
        del s, d
        vbase = torch.from_numpy(vb).to(dev)
        # local column ids: subtract the base of each entry's graph (graph of
        # an entry = graph of its row; a CSR entry never leaves its graph)
        deg = G.row_offsets[1:] - G.row_offsets[:-1]
        graph_of_row = torch.repeat_interleave(torch.arange(len(graphs), device=dev), torch.from_numpy(ns).to(dev))
        base_of_entry = torch.repeat_interleave(vbase[:-1][graph_of_row], deg)
        cols = (G.cols.to(torch.int64) - base_of_entry).to(torch.int32)
        nnz_g = (G.row_offsets[vbase[1:]] - G.row_offsets[vbase[:-1]]).cpu().numpy()
        return Batch(vbase, G.row_offsets, cols, [(int(n), int(z)) for n, z in zip(ns, nnz_g)])


@dataclass
class BatchResult:
    triangles: torch.Tensor  # int64 [G]
    h_count: torch.Tensor | None  # int64 [G] (None when not asked for)
    levels: torch.Tensor | None = None  # int32 [sum n]


def make_tuning(t: dict | None) -> L.TcTuning | None:
    """A tc_tuning from a dict of its fields (missing ones: 0 = default)."""
    if not t:
        return None
    unknown = set(t) - set(L.TUNING_FIELDS)
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    return L.TcTuning(*[int(t.get(f, 0)) for f in L.TUNING_FIELDS])


@_on_stream
def count_batch(b: Batch, tuning: dict | None = None, return_levels: bool = False,
                ws: Workspace | None = None, stream=None, out: BatchResult | None = None,
                with_h: bool = True, validate: bool = False,
                max_graph_vertices: int | None = None, noalloc: bool = False) -> BatchResult:
    """tc_count_batch: exact T and (with_h) |H| of every graph (device
    tensors).  validate=True checks the batch's structure first (the call
    then synchronises).  max_graph_vertices overrides the bound the batch
    declares (tests of the library's own checks).  noalloc=True calls
    tc_count_batch_noalloc (scratch in the library's static device array, no
    workspace; outputs are still allocated here unless `out` is given)."""
    lib = L.load()
    dev = b.cols.device
    G = b.num_graphs
    res = out or BatchResult(torch.empty(max(G, 1), dtype=torch.int64, device=dev),
                             torch.empty(max(G, 1), dtype=torch.int64, device=dev) if with_h else None,
                             torch.empty(max(b.total_vertices, 1), dtype=torch.int32, device=dev)
                             if return_levels else None)
    tb = b.tc(max_graph_vertices)
    tu = make_tuning(tuning)
    if noalloc:
        _check(lib.tc_count_batch_noalloc(ctypes.byref(tb), ctypes.byref(tu) if tu is not None else None,
                                          L.TC_VALIDATE if validate else 0, _ptr(res.triangles), _ptr(res.h_count),
                                          _ptr(res.levels), _stream(stream)), "tc_count_batch_noalloc")
        return res
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_COUNT_BATCH, b.total_vertices, b.total_nnz, G))
    _check(lib.tc_count_batch(ctypes.byref(tb), ctypes.byref(tu) if tu is not None else None,
                              L.TC_VALIDATE if validate else 0,
                              _ptr(res.triangles), _ptr(res.h_count), _ptr(res.levels), _ptr(buf), buf.numel(),
                              _stream(stream)), "tc_count_batch")
    return res


class CapturedBatch:
    """tc_count_batch recorded once in a graph and replayed (no host work per
    launch beyond the replay).  Inputs and outputs stay at fixed addresses."""

    def __init__(self, b: Batch, tuning: dict | None = None, ws: Workspace | None = None):
        self.batch = b
        self.tuning = tuning
        dev = b.cols.device
        self.ws = ws or Workspace(dev)
        self.ws.get(workspace_bytes(L.OP_COUNT_BATCH, b.total_vertices, b.total_nnz, b.num_graphs))
        self.out = BatchResult(torch.empty(max(b.num_graphs, 1), dtype=torch.int64, device=dev),
                               torch.empty(max(b.num_graphs, 1), dtype=torch.int64, device=dev))
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):  # warm-up outside capture
            count_batch(b, tuning, ws=self.ws, stream=side, out=self.out)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            count_batch(b, tuning, ws=self.ws, stream=torch.cuda.current_stream(dev), out=self.out)

    def replay(self) -> BatchResult:
        self.graph.replay()
        return self.out


_TUNE_CANDIDATES = [
    dict(batch_block=256, batch_piece=4096), dict(batch_block=256, batch_piece=16384),
    dict(batch_block=256, batch_piece=65536), dict(batch_block=512, batch_piece=4096),
    dict(batch_block=512, batch_piece=16384), dict(batch_block=512, batch_piece=65536),
    dict(batch_block=256, batch_piece=16384, batch_blocks_per_cu=2),
    dict(batch_block=64, batch_piece=1024), dict(batch_block=64, batch_piece=2048),
    dict(batch_block=64, batch_piece=4096),
]


def _cache_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "autotune.json")


def shape_key(b: Batch) -> str:
    """Coarse batch shape: graph count, total vertices and entries (log2)."""
    lg = lambda v: int(np.log2(max(v, 1)))  # noqa: E731
    return f"G{b.num_graphs}-n{lg(b.total_vertices)}-z{lg(b.total_nnz)}"


def autotune(b: Batch, candidates=None, reps: int = 3, use_cache: bool = True, verbose: bool = False) -> dict:
    """Time every candidate tuning on `b` (median of `reps` launches, HIP
    events on the launch stream) and return the fastest; results are
    checked equal across candidates.  The choice is cached per shape_key."""
    key = shape_key(b)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["tuning"])
    cands = candidates or _TUNE_CANDIDATES
    stream = torch.cuda.current_stream()
    ws = Workspace(b.cols.device)
    ref = None
    best, best_ms, table = None, float("inf"), []
    for t in cands:
        times = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            r = count_batch(b, t, ws=ws, stream=stream)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times[1:]))
        tri = r.triangles.cpu()
        if ref is None:
            ref = tri
        elif not torch.equal(ref, tri):
            raise TcError(-1, f"autotune: tuning {t} changed the counts")
        table.append((t, ms))
        if verbose:
            print(f"[autotune] {t}: {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = t, ms
    if use_cache:
        cache[key] = dict(tuning=best, ms=best_ms, table=[[t, ms] for t, ms in table])
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(best)
