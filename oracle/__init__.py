"""CPU oracle for cover-edge triangle counting -- TEST INFRASTRUCTURE ONLY.

This package is the test reference: a plain single-threaded C implementation
(``oracle.c``) of the paper's sequential algorithm (Alg. 1, CETC, of Bader et
al., "Triangle Counting Through Cover-Edges") plus an O(n^3) brute force
(``brute.py``).  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the GPU
library and never imports it.

All arrays are numpy; a CSR is ``(n, row_offsets int64[n+1], cols int32[nnz])``.

Parity status of every function (what pins it is in ``tests/test_oracle.py``):

* build_csr, validate_csr -- pinned (hand-built CSRs, scipy/networkx).
* bfs_levels -- pinned (scipy shortest paths from the same roots; path/star/
  complete closed forms; BFS invariants).
* cover_edges -- pinned (closed-form |H| for K_n, W_n, C_n; bipartite <=> 0;
  Lemma 1 and Lemma 2 against brute-force triangle lists).
* count -- pinned (brute force, networkx, closed forms, root and relabelling
  invariance, per-vertex sum = 3T, both intersection modes).
* edge_count -- pinned (brute force, closed forms).
* work_counters -- pinned (brute-force loops over adjacency sets, closed
  forms for K_n, zero for bipartite graphs; ``tests/test_oracle_work.py``).
* per-edge support -- pinned (sum over H = T; bounded by |N(u) ∩ N(v)|).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "liboracle.so")
_lib = None

STATUS = {
    0: "ok", -1: "invalid argument", -2: "out of memory", -3: "bad offsets",
    -4: "id out of range", -5: "row not sorted", -6: "duplicate entry",
    -7: "self loop", -8: "not symmetric",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}: {STATUS.get(code, 'unknown')}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O2 (single-threaded, no OpenMP)."""
    global _lib
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    _lib = None
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_SO))
    return _lib


def _use_library(path: str | None):
    """Load the oracle from another build of oracle.c (the mutation tests
    compile planted-mistake copies); None restores the normal build."""
    global _lib
    _lib = None if path is None else _bind(ctypes.CDLL(path))


def _bind(lib):
    i64, p, c_int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    lib.oracle_build_csr.argtypes = [i64, i64, p, p, p, p, p]
    lib.oracle_build_csr.restype = c_int
    lib.oracle_validate_csr.argtypes = [i64, p, p]
    lib.oracle_validate_csr.restype = c_int
    lib.oracle_default_root.argtypes = [i64, p]
    lib.oracle_default_root.restype = i64
    lib.oracle_bfs_levels.argtypes = [i64, p, p, i64, p, p, p]
    lib.oracle_bfs_levels.restype = c_int
    lib.oracle_cover_edges.argtypes = [i64, p, p, p, p, p]
    lib.oracle_cover_edges.restype = i64
    lib.oracle_count.argtypes = [i64, p, p, p, c_int, p, p, p]
    lib.oracle_count.restype = c_int
    lib.oracle_edge_support.argtypes = [p, p, p, ctypes.c_int32, ctypes.c_int32]
    lib.oracle_edge_support.restype = i64
    lib.oracle_edge_count.argtypes = [i64, p, p]
    lib.oracle_edge_count.restype = i64
    lib.oracle_count_rows.argtypes = [i64, p, p, p, c_int, i64, i64, p]
    lib.oracle_count_rows.restype = c_int
    lib.oracle_count_rows_strided.argtypes = [i64, p, p, p, c_int, i64, i64, i64, p]
    lib.oracle_count_rows_strided.restype = c_int
    lib.oracle_list_triangles.argtypes = [i64, p, p, p, p, i64, p]
    lib.oracle_list_triangles.restype = c_int
    lib.oracle_edge_supports.argtypes = [i64, p, p, p, p]
    lib.oracle_edge_supports.restype = c_int
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(rc):
    if rc != 0:
        raise OracleError(rc)


@dataclass
class CSR:
    n: int
    row_offsets: np.ndarray  # int64[n+1]
    cols: np.ndarray         # int32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_offsets[-1]) if self.n > 0 else 0

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_offsets)


def build_csr(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Simple undirected CSR from raw pairs (loops dropped, repeats merged)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    off = np.zeros(n + 1, dtype=np.int64)
    cols = np.empty(max(2 * src.shape[0], 1), dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    _check(_load().oracle_build_csr(n, src.shape[0], _p(src), _p(dst), _p(off), _p(cols),
                                    _p(nnz)))
    return CSR(n, off, cols[: int(nnz[0])].copy())


def from_graph(g) -> CSR:
    """CSR of a graphgen.Graph (raw pairs)."""
    return build_csr(g.n, g.src, g.dst)


def validate_csr(csr: CSR) -> int:
    """0 if the CSR is a simple undirected graph, else the oracle status."""
    off = np.ascontiguousarray(csr.row_offsets, dtype=np.int64)
    cols = np.ascontiguousarray(csr.cols, dtype=np.int32)
    if cols.size == 0:
        cols = np.zeros(1, dtype=np.int32)
    return int(_load().oracle_validate_csr(csr.n, _p(off), _p(cols)))


def default_root(csr: CSR) -> int:
    return int(_load().oracle_default_root(csr.n, _p(csr.row_offsets)))


@dataclass
class Levels:
    levels: np.ndarray  # int32[n]
    num_levels: int
    num_roots: int


def bfs_levels(csr: CSR, root: int = -1) -> Levels:
    """Alg. 1 levels: BFS from root (default: max degree, smallest id), then a
    new BFS from every vertex left unvisited, in increasing id order."""
    L = np.empty(max(csr.n, 1), dtype=np.int32)
    nl = np.zeros(1, dtype=np.int32)
    nr = np.zeros(1, dtype=np.int64)
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    _check(_load().oracle_bfs_levels(csr.n, _p(csr.row_offsets), _p(cols), root, _p(L), _p(nl),
                                     _p(nr)))
    return Levels(L[: csr.n].copy(), int(nl[0]), int(nr[0]))


def cover_edges(csr: CSR, levels: np.ndarray):
    """Horizontal edges (u < v, L(u) = L(v)) in lexicographic order."""
    lib = _load()
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    h = int(lib.oracle_cover_edges(csr.n, _p(csr.row_offsets), _p(cols), _p(L), None, None))
    hu = np.empty(max(h, 1), dtype=np.int32)
    hv = np.empty(max(h, 1), dtype=np.int32)
    lib.oracle_cover_edges(csr.n, _p(csr.row_offsets), _p(cols), _p(L), _p(hu), _p(hv))
    return hu[:h].copy(), hv[:h].copy()


@dataclass
class Count:
    triangles: int
    per_edge: np.ndarray | None
    per_vertex: np.ndarray | None


def count(csr: CSR, levels: np.ndarray, mode: int = 0, per_edge: bool = False,
          per_vertex: bool = False) -> Count:
    """Alg. 1 count over the horizontal edges of ``levels``.
    mode 0 = direct-address table intersection, 1 = two-pointer merge."""
    lib = _load()
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    pe = pv = None
    if per_edge:
        h = int(lib.oracle_cover_edges(csr.n, _p(csr.row_offsets), _p(cols), _p(L), None, None))
        pe = np.zeros(max(h, 1), dtype=np.int64)
    if per_vertex:
        pv = np.zeros(max(csr.n, 1), dtype=np.int64)
    T = np.zeros(1, dtype=np.int64)
    _check(lib.oracle_count(csr.n, _p(csr.row_offsets), _p(cols), _p(L), mode, _p(T), _p(pe),
                            _p(pv)))
    if per_edge:
        pe = pe[:h].copy()
    if per_vertex:
        pv = pv[: csr.n].copy()
    return Count(int(T[0]), pe, pv)


def count_rows(csr: CSR, levels: np.ndarray, u_begin: int, u_end: int, mode: int = 0) -> int:
    """Alg. 1 count restricted to cover edges (u, v) with u in [u_begin, u_end)."""
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    T = np.zeros(1, dtype=np.int64)
    _check(_load().oracle_count_rows(csr.n, _p(csr.row_offsets), _p(cols), _p(L), mode, u_begin, u_end,
                                     _p(T)))
    return int(T[0])


def count_rows_strided(csr: CSR, levels: np.ndarray, phase: int, stride: int, mode: int = 0) -> int:
    """Alg. 1 count restricted to cover edges (u, v) with u = phase (mod
    stride): the phases of one stride partition the rows."""
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    T = np.zeros(1, dtype=np.int64)
    _check(_load().oracle_count_rows_strided(csr.n, _p(csr.row_offsets), _p(cols), _p(L), mode,
                                             min(phase, csr.n), csr.n, stride, _p(T)))
    return int(T[0])


def edge_support(csr: CSR, levels: np.ndarray, u: int, v: int) -> int:
    """c(u, v) of one horizontal edge (u < v) by two-pointer merge."""
    L = np.ascontiguousarray(levels, dtype=np.int32)
    return int(_load().oracle_edge_support(_p(csr.row_offsets), _p(csr.cols), _p(L), u, v))


def list_triangles(csr: CSR, levels: np.ndarray) -> np.ndarray:
    """Triangle finding by Alg. 1's enumeration: int32 [T, 3], each row the
    three ids ascending, rows in the order the count finds them."""
    lib = _load()
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    T = np.zeros(1, dtype=np.int64)
    _check(lib.oracle_list_triangles(csr.n, _p(csr.row_offsets), _p(cols), _p(L), None, 0, _p(T)))
    tri = np.zeros((max(int(T[0]), 1), 3), dtype=np.int32)
    _check(lib.oracle_list_triangles(csr.n, _p(csr.row_offsets), _p(cols), _p(L), _p(tri), int(T[0]), _p(T)))
    return tri[: int(T[0])].copy()


def edge_supports(csr: CSR, levels: np.ndarray) -> np.ndarray:
    """Triangles on each edge, int64 per CSR entry (both orientations)."""
    lib = _load()
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    L = np.ascontiguousarray(levels, dtype=np.int32)
    if L.size == 0:
        L = np.zeros(1, dtype=np.int32)
    sup = np.zeros(max(csr.nnz, 1), dtype=np.int64)
    _check(lib.oracle_edge_supports(csr.n, _p(csr.row_offsets), _p(cols), _p(L), _p(sup)))
    return sup[: csr.nnz].copy()


def edge_count(csr: CSR) -> int:
    """Plain direction-oriented edge iterator (u < v < w); uses no levels."""
    cols = csr.cols if csr.cols.size else np.zeros(1, dtype=np.int32)
    return int(_load().oracle_edge_count(csr.n, _p(csr.row_offsets), _p(cols)))


def work_counters(csr: CSR, levels: np.ndarray) -> dict:
    """Work measures of the cost analysis (Sec. III), from their definitions:
    over the horizontal edges H (u < v, equal levels) |H|, the sum of
    min(d(u), d(v)) (Alg. 1 scans the shorter list and looks each id up in a
    hash table of the other) and the sum of d(u) + d(v) (both lists merged);
    for the plain edge iterator (every edge u < v, apexes w > v) the sum over
    all edges of min(d+(u), d+(v)), where d+(x) = |{w in N(x) : w > x}|."""
    deg = np.diff(csr.row_offsets)
    rows = np.repeat(np.arange(csr.n, dtype=np.int64), deg)
    cols = csr.cols.astype(np.int64)
    up = rows < cols
    u, v = rows[up], cols[up]
    lv = np.asarray(levels)
    hz = lv[u] == lv[v] if u.size else np.zeros(0, dtype=bool)
    fwd = np.bincount(u, minlength=csr.n)
    return dict(h=int(hz.sum()),
                h_min_deg=int(np.minimum(deg[u[hz]], deg[v[hz]]).sum()),
                h_sum_deg=int((deg[u[hz]] + deg[v[hz]]).sum()),
                edge_min_fwd=int(np.minimum(fwd[u], fwd[v]).sum()))


def triangle_count(csr: CSR, root: int = -1, mode: int = 0) -> int:
    """Alg. 1 end to end: levels, then the count over the horizontal edges."""
    return count(csr, bfs_levels(csr, root).levels, mode).triangles
