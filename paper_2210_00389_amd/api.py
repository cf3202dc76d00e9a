"""Torch-facing wrappers of libtc.

PyTorch provides device memory and streams; every computation is a libtc
entry point (include/tc.h).  Graphs live on the device as int64 row offsets
and int32 sorted columns.
"""
from __future__ import annotations

import ctypes
import functools
import inspect
from dataclasses import dataclass

import torch

from . import _lib as L


class TcError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = L.load()
        detail = lib.tc_last_error().decode(errors="replace")
        name = L.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {name}: {detail}")
        self.status = status


def _check(rc: int, where: str):
    if rc != L.TC_OK:
        raise TcError(rc, where)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Runs fn with its `stream` argument (when given) as torch's current
    stream, so that the buffers it allocates -- workspace growth, outputs --
    belong to the stream the library enqueues on, and the caching allocator
    never hands a freed block to other work before that stream is done."""
    idx = list(inspect.signature(fn).parameters).index("stream")

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = kwargs.get("stream") if "stream" in kwargs else (args[idx] if len(args) > idx else None)
        if stream is None:
            return fn(*args, **kwargs)
        with torch.cuda.stream(stream):
            return fn(*args, **kwargs)
    return wrapper


class Workspace:
    """A growable device byte buffer (torch allocation) handed to libtc."""

    def __init__(self, device=None):
        self.device = torch.device(device or "cuda")
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def default_workspace(device=None) -> Workspace:
    dev = torch.device(device or "cuda")
    key = (dev.type, dev.index if dev.index is not None else torch.cuda.current_device())
    if key not in _default_ws:
        _default_ws[key] = Workspace(dev)
    return _default_ws[key]


@dataclass
class Graph:
    """A simple undirected graph in device CSR form."""
    n: int
    row_offsets: torch.Tensor  # int64 [n+1]
    cols: torch.Tensor         # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.cols.numel())

    @property
    def m(self) -> int:
        return self.nnz // 2

    def csr(self) -> L.TcCsr:
        return L.TcCsr(self.n, self.nnz, self.row_offsets.data_ptr() if self.n > 0 else None,
                       self.cols.data_ptr() if self.nnz > 0 else None)

    def nbytes(self) -> int:
        return self.row_offsets.numel() * 8 + self.cols.numel() * 4


def workspace_bytes(op: int, n: int, nnz: int, num_graphs: int = 0) -> int:
    return int(L.load().tc_workspace_bytes(op, n, nnz, num_graphs))


@_on_stream
def build_csr(n: int, src: torch.Tensor, dst: torch.Tensor, ws: Workspace | None = None,
              stream=None) -> Graph:
    """Simple undirected CSR from raw device pairs (tc_build_csr)."""
    lib = L.load()
    src = src.to(torch.int32).contiguous()
    dst = dst.to(torch.int32).contiguous()
    dev = src.device
    P = int(src.numel())
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    cols = torch.empty(max(2 * P, 1), dtype=torch.int32, device=dev)
    nnz = ctypes.c_int64(0)
    need = workspace_bytes(L.OP_BUILD_CSR, n, P)
    buf = (ws or default_workspace(dev)).get(need)
    _check(lib.tc_build_csr(n, P, _ptr(src), _ptr(dst), _ptr(off), _ptr(cols), ctypes.byref(nnz),
                            _ptr(buf), buf.numel(), _stream(stream)), "tc_build_csr")
    return Graph(n, off, cols[: nnz.value])


@_on_stream
def from_host_pairs(n: int, src, dst, device="cuda", ws=None, stream=None) -> Graph:
    s = torch.as_tensor(src, dtype=torch.int32).to(device)
    d = torch.as_tensor(dst, dtype=torch.int32).to(device)
    return build_csr(n, s, d, ws, stream)


def from_host_csr(n: int, row_offsets, cols, device="cuda") -> Graph:
    off = torch.as_tensor(row_offsets, dtype=torch.int64).to(device)
    c = torch.as_tensor(cols, dtype=torch.int32).to(device)
    return Graph(n, off, c)


@_on_stream
def validate(g: Graph, ws: Workspace | None = None, stream=None) -> int:
    """0 if g is a simple undirected CSR, else the negative status."""
    lib = L.load()
    buf = (ws or default_workspace(g.cols.device)).get(workspace_bytes(L.OP_VALIDATE, g.n, g.nnz))
    csr = g.csr()
    return int(lib.tc_validate_csr(ctypes.byref(csr), _ptr(buf), buf.numel(), _stream(stream)))


@_on_stream
def bfs_levels(g: Graph, root: int = -1, validate: bool = False, ws: Workspace | None = None,
               stream=None):
    """(levels int32 tensor, num_levels) as in Alg. 1 (tc_bfs_levels)."""
    lib = L.load()
    levels = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.cols.device)
    nl = ctypes.c_int32(0)
    buf = (ws or default_workspace(g.cols.device)).get(workspace_bytes(L.OP_BFS_LEVELS, g.n, g.nnz))
    csr = g.csr()
    _check(lib.tc_bfs_levels(ctypes.byref(csr), root, L.TC_VALIDATE if validate else 0, _ptr(levels),
                             ctypes.byref(nl), _ptr(buf), buf.numel(), _stream(stream)), "tc_bfs_levels")
    return levels[: g.n], int(nl.value)


@_on_stream
def cover_edges(g: Graph, levels: torch.Tensor, ws: Workspace | None = None, stream=None):
    """(h_u, h_v): the cover edges of `levels`, lexicographic (tc_cover_edges)."""
    lib = L.load()
    dev = g.cols.device
    cap = max(g.nnz // 2, 1)
    hu = torch.empty(cap, dtype=torch.int32, device=dev)
    hv = torch.empty(cap, dtype=torch.int32, device=dev)
    hc = torch.zeros(1, dtype=torch.int64, device=dev)
    levels = levels.to(torch.int32).contiguous()
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_COVER_EDGES, g.n, g.nnz))
    csr = g.csr()
    _check(lib.tc_cover_edges(ctypes.byref(csr), _ptr(levels), _ptr(hu), _ptr(hv), _ptr(hc), _ptr(buf),
                              buf.numel(), _stream(stream)), "tc_cover_edges")
    h = int(hc.item())
    return hu[:h], hv[:h]


@dataclass
class CountResult:
    triangles: torch.Tensor        # int64 [1], device
    h_count: torch.Tensor          # int64 [1], device
    levels: torch.Tensor | None
    per_vertex: torch.Tensor | None

    @property
    def T(self) -> int:
        return int(self.triangles.item())

    @property
    def h(self) -> int:
        return int(self.h_count.item())


@_on_stream
def count(g: Graph, root: int = -1, per_vertex: bool = False, validate: bool = False,
          return_levels: bool = False, ws: Workspace | None = None, stream=None,
          out: CountResult | None = None, tuning: dict | None = None) -> CountResult:
    """Cover-edge triangle count (tc_count_tuned; tuning=None gives
    tc_count's defaults); results stay on the device."""
    from .batch import make_tuning
    lib = L.load()
    dev = g.cols.device
    res = out or CountResult(torch.zeros(1, dtype=torch.int64, device=dev),
                             torch.zeros(1, dtype=torch.int64, device=dev),
                             torch.empty(max(g.n, 1), dtype=torch.int32, device=dev) if return_levels else None,
                             torch.empty(max(g.n, 1), dtype=torch.int64, device=dev) if per_vertex else None)
    flags = (L.TC_VALIDATE if validate else 0) | (L.TC_PER_VERTEX if per_vertex else 0)
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_COUNT, g.n, g.nnz))
    csr = g.csr()
    tu = make_tuning(tuning)
    _check(lib.tc_count_tuned(ctypes.byref(csr), root, flags, ctypes.byref(tu) if tu is not None else None,
                              _ptr(res.triangles), _ptr(res.h_count), _ptr(res.levels), _ptr(res.per_vertex),
                              _ptr(buf), buf.numel(), _stream(stream)),
           "tc_count")
    if res.levels is not None:
        res.levels = res.levels[: g.n]
    if res.per_vertex is not None:
        res.per_vertex = res.per_vertex[: g.n]
    return res


@dataclass
class ListResult:
    tri: torch.Tensor        # int32 [min(T, cap), 3], each row ascending; row order unspecified
    triangles: torch.Tensor  # int64 [1]: T
    h_count: torch.Tensor    # int64 [1]: |H|
    tri_buf: torch.Tensor | None = None  # the whole output buffer [max(cap, 1), 3]

    @property
    def T(self) -> int:
        return int(self.triangles.item())


@_on_stream
def list_triangles(g: Graph, root: int = -1, cap: int | None = None, validate: bool = False,
                   ws: Workspace | None = None, stream=None, out: ListResult | None = None) -> ListResult:
    """Triangle finding (tc_list_triangles).  With cap=None the triangles are
    counted first (tc_count) and the buffer is sized exactly; `out` (from an
    earlier call with the same cap) reuses its buffers."""
    lib = L.load()
    dev = g.cols.device
    if cap is None:
        cap = out.tri_buf.shape[0] if out is not None else count(g, root=root, validate=validate, ws=ws,
                                                                  stream=stream).T
    if out is not None and out.tri_buf.shape[0] >= max(cap, 1):
        res = out
    else:
        res = ListResult(torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev),
                         torch.zeros(1, dtype=torch.int64, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
        res.tri_buf = res.tri
    flags = L.TC_VALIDATE if validate else 0
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_COUNT, g.n, g.nnz))
    csr = g.csr()
    _check(lib.tc_list_triangles(ctypes.byref(csr), root, flags, _ptr(res.tri_buf), cap, _ptr(res.triangles),
                                 _ptr(res.h_count), None, _ptr(buf), buf.numel(), _stream(stream)),
           "tc_list_triangles")
    res.tri = res.tri_buf[: min(cap, res.T)]
    return res


@dataclass
class RootChoice:
    root: int                 # the candidate with the smallest |H|
    candidates: list[int]     # largest degree first (smallest id on ties)
    h: list[int]              # |H| with each candidate as root


@_on_stream
def select_root(g: Graph, num_candidates: int = 8, validate: bool = False, ws: Workspace | None = None,
                stream=None) -> RootChoice:
    """Root choice for a small cover-edge set (tc_select_root)."""
    lib = L.load()
    dev = g.cols.device
    k = max(0, min(num_candidates, L.MAX_ROOT_CANDIDATES))
    root = ctypes.c_int64(-1)
    cand = (ctypes.c_int64 * max(k, 1))()
    hs = (ctypes.c_int64 * max(k, 1))()
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_SELECT_ROOT, g.n, g.nnz))
    csr = g.csr()
    _check(lib.tc_select_root(ctypes.byref(csr), num_candidates, L.TC_VALIDATE if validate else 0,
                              ctypes.byref(root), cand, hs, _ptr(buf), buf.numel(), _stream(stream)),
           "tc_select_root")
    used = min(k, g.n)
    return RootChoice(int(root.value), list(cand[:used]), list(hs[:used]))


@_on_stream
def edge_support(g: Graph, tri: torch.Tensor, stream=None) -> torch.Tensor:
    """Triangles per CSR entry from a triangle list (tc_edge_support)."""
    lib = L.load()
    tri = tri.contiguous()
    if tri.dtype != torch.int32 or (tri.dim() != 2 or tri.shape[1] != 3) and tri.numel() > 0:
        raise ValueError("tri must be an int32 [k, 3] tensor")
    sup = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=g.cols.device)
    csr = g.csr()
    _check(lib.tc_edge_support(ctypes.byref(csr), _ptr(tri) if tri.numel() else None, tri.shape[0] if tri.numel() else 0,
                               _ptr(sup), _stream(stream)), "tc_edge_support")
    return sup[: g.nnz]


@_on_stream
def count_edge_baseline(g: Graph, validate: bool = False, ws: Workspace | None = None, stream=None,
                        out: torch.Tensor | None = None, tuning: dict | None = None) -> torch.Tensor:
    """Plain direction-oriented edge-iterator count
    (tc_count_edge_baseline_tuned; tuning=None gives the defaults)."""
    from .batch import make_tuning
    lib = L.load()
    dev = g.cols.device
    t = out if out is not None else torch.zeros(1, dtype=torch.int64, device=dev)
    buf = (ws or default_workspace(dev)).get(workspace_bytes(L.OP_EDGE_BASELINE, g.n, g.nnz))
    csr = g.csr()
    tu = make_tuning(tuning)
    _check(lib.tc_count_edge_baseline_tuned(ctypes.byref(csr), L.TC_VALIDATE if validate else 0,
                                            ctypes.byref(tu) if tu is not None else None, _ptr(t),
                                            _ptr(buf), buf.numel(), _stream(stream)), "tc_count_edge_baseline")
    return t


def read_stats(ws: Workspace | None = None, device=None, stream=None) -> dict:
    """Work statistics of the last tc_count / tc_count_edge_baseline call
    that used this workspace."""
    lib = L.load()
    w = ws or default_workspace(device)
    st = L.TcStats()
    _check(lib.tc_read_stats(_ptr(w.buf), ctypes.byref(st), _stream(stream)), "tc_read_stats")
    out = {k: int(getattr(st, k)) for k in ("n", "nnz", "h", "num_levels", "stream_elems", "light_tasks",
                                             "heavy_items", "heavy_desc", "heavy_elems", "heavy_builds",
                                             "light_elems", "descriptors", "twolevel_elems")}
    out["bin_elems"] = [int(x) for x in st.bin_elems]
    out["bin_items"] = [int(x) for x in st.bin_items]
    return out


def profile_enable(on: bool = True):
    L.load().tc_profile_enable(1 if on else 0)


def profile_read() -> list:
    """[(stage name, ms)] of the calling thread's last libtc call."""
    lib = L.load()
    p = L.TcProfile()
    _check(lib.tc_profile_read(ctypes.byref(p)), "tc_profile_read")
    return [(bytes(p.names[i]).split(b"\0")[0].decode(), float(p.ms[i])) for i in range(p.num_stages)]
