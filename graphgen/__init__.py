"""Seeded synthetic graph generators: the inputs shared by the CPU oracle and
the HIP library.

Every generator returns a :class:`Graph` holding ``n`` and two int32 endpoint
arrays (``src``, ``dst``).  The pairs are *raw*: they may contain self loops,
repeats and both orientations of one edge.  Turning them into a simple
undirected graph in CSR form is the consumer's job (the oracle and the
library each have their own builder), so this module holds no part of the
counting method.

Families and recipes:

* R-MAT (Graph500 quadrant recursion, a,b,c,d = 0.57,0.19,0.19,0.05 by
  default), ``2**scale * edge_factor`` pairs, then a seeded uniform relabel of
  the vertex ids.
* Erdos-Renyi G(n, p) by geometric skipping.
* Barabasi-Albert with ``m`` edges per new vertex.
* Chung-Lu with power-law expected degrees (exponent gamma, mean degree d).
* Closed-form families: complete, wheel, cycle, path, star, complete
  bipartite, grid, random bipartite.
* :func:`batch_mix` (4096 ER / BA graphs of log-uniform size) and
  :func:`serving_pool` (R-MAT / Chung-Lu request pool).

The C part (``graphgen.c``) is compiled with gcc into ``_build/`` on first use.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_BUILD = os.path.join(_HERE, "_build")
_SO = os.path.join(_BUILD, "libgraphgen.so")
_lib = None

RMAT_PROBS = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compile graphgen.c into _build/libgraphgen.so with gcc (-O2, OpenMP)."""
    global _lib
    if not force and os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(_SRC):
        return _SO
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    _lib = None
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        i64, u64, i32p, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, u64, u64, u64, u64, i32p, i32p]
        lib.gg_rmat.restype = None
        lib.gg_permutation.argtypes = [i64, u64, i32p]
        lib.gg_permutation.restype = None
        lib.gg_relabel.argtypes = [i64, i32p, i32p, i32p]
        lib.gg_relabel.restype = None
        lib.gg_er.argtypes = [i64, dbl, u64, i32p, i32p, i64]
        lib.gg_er.restype = i64
        lib.gg_ba.argtypes = [i64, i64, u64, i32p, i32p]
        lib.gg_ba.restype = i64
        lib.gg_chung_lu.argtypes = [i64, i32p, u64, i32p, i32p, i64]
        lib.gg_chung_lu.restype = i64
        lib.gg_stream_key.argtypes = [u64, u64]
        lib.gg_stream_key.restype = u64
        lib.gg_draw.argtypes = [u64, u64]
        lib.gg_draw.restype = u64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """Raw undirected pairs over vertex ids [0, n)."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_pairs(self) -> int:
        return int(self.src.shape[0])


def _mk(n, s, d, name, **meta) -> Graph:
    return Graph(int(n), np.ascontiguousarray(s, dtype=np.int32),
                 np.ascontiguousarray(d, dtype=np.int32), name, dict(meta))


def permutation(n: int, seed: int) -> np.ndarray:
    """Seeded uniform permutation of [0, n) (Fisher-Yates); perm[old] = new."""
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed & (2**64 - 1), _ptr(perm))
    return perm


def relabel(g: Graph, seed: int) -> Graph:
    """Apply a seeded uniform vertex relabelling to the pairs of ``g``."""
    perm = permutation(g.n, seed)
    s, d = g.src.copy(), g.dst.copy()
    _load().gg_relabel(s.shape[0], _ptr(perm), _ptr(s), _ptr(d))
    meta = dict(g.meta, relabel_seed=seed)
    return Graph(g.n, s, d, g.name, meta)


# ----------------------------------------------------------------- R-MAT
def rmat(scale: int, edge_factor: int = 16, probs=RMAT_PROBS, seed: int = 1,
         permute: bool = True) -> Graph:
    """R-MAT with ``2**scale`` vertices and ``edge_factor * 2**scale`` pairs.

    Quadrant per bit level from cumulative integer thresholds over 53 random
    bits; the vertex ids are then relabelled by a permutation drawn from the
    same seed (so hubs are not clustered at small ids).
    """
    a, b, c, d = probs
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    n = 1 << scale
    m = edge_factor * n
    two53 = float(1 << 53)
    ta = int(math.floor(a * two53))
    tab = int(math.floor((a + b) * two53))
    tabc = int(math.floor((a + b + c) * two53))
    s = np.empty(m, dtype=np.int32)
    t = np.empty(m, dtype=np.int32)
    lib = _load()
    lib.gg_rmat(scale, m, ta, tab, tabc, seed & (2**64 - 1), _ptr(s), _ptr(t))
    g = Graph(n, s, t, f"rmat{scale}", dict(family="rmat", scale=scale, edge_factor=edge_factor,
                                             probs=tuple(probs), seed=seed))
    if permute:
        perm = permutation(n, seed ^ 0x5EED5EED)
        lib.gg_relabel(m, _ptr(perm), _ptr(s), _ptr(t))
        g.meta["permuted"] = True
    return g


# ------------------------------------------------------------ Erdos-Renyi
def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    """G(n, p): every unordered pair independently with probability p."""
    lib = _load()
    exp = p * n * (n - 1) / 2.0
    cap = int(exp + 10.0 * math.sqrt(exp + 1.0) + 16)
    while True:
        s = np.empty(max(cap, 1), dtype=np.int32)
        t = np.empty(max(cap, 1), dtype=np.int32)
        k = lib.gg_er(n, float(p), seed & (2**64 - 1), _ptr(s), _ptr(t), cap)
        if k >= 0:
            return _mk(n, s[:k], t[:k], f"er{n}", family="er", p=p, seed=seed)
        cap = -k


# -------------------------------------------------------- Barabasi-Albert
def barabasi_albert(n: int, m: int, seed: int) -> Graph:
    """Preferential attachment, ``m`` pairs per new vertex (raw, with repeats)."""
    s = np.empty(n * m, dtype=np.int32)
    t = np.empty(n * m, dtype=np.int32)
    k = _load().gg_ba(n, m, seed & (2**64 - 1), _ptr(s), _ptr(t))
    return _mk(n, s[:k], t[:k], f"ba{n}", family="ba", m=m, seed=seed)


# --------------------------------------------------------------- Chung-Lu
def chung_lu_weights(n: int, gamma: float, mean_degree: float) -> np.ndarray:
    """Expected degrees w_i = c*(i+i0)^(-1/(gamma-1)), scaled to the given
    mean, with i0 chosen so that w_0 = sqrt(n*mean) (then every p_ij <= 1)."""
    beta = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)
    target = math.sqrt(n * mean_degree)

    def w0(i0):
        base = (idx + i0) ** (-beta)
        c = n * mean_degree / base.sum()
        return c * i0 ** (-beta), c

    lo, hi = 1e-6, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        v, _ = w0(mid)
        if v > target:
            lo = mid
        else:
            hi = mid
    i0 = hi
    _, c = w0(i0)
    return c * (idx + i0) ** (-beta)


def chung_lu(n: int, gamma: float = 2.1, mean_degree: float = 20.0, seed: int = 1,
             permute: bool = True) -> Graph:
    """Chung-Lu graph with power-law expected degrees; ids relabelled."""
    w = np.ascontiguousarray(chung_lu_weights(n, gamma, mean_degree))
    lib = _load()
    exp = n * mean_degree / 2.0
    cap = int(exp * 1.2 + 10.0 * math.sqrt(exp) + 64)
    while True:
        s = np.empty(cap, dtype=np.int32)
        t = np.empty(cap, dtype=np.int32)
        k = lib.gg_chung_lu(n, _ptr(w), seed & (2**64 - 1), _ptr(s), _ptr(t), cap)
        if k >= 0:
            break
        cap = -k
    g = _mk(n, s[:k], t[:k], f"cl{n}", family="chung_lu", gamma=gamma,
            mean_degree=mean_degree, seed=seed)
    if permute:
        g = relabel(g, seed ^ 0xC1C1C1C1)
    return g


# ----------------------------------------------------- closed-form families
def complete(n: int) -> Graph:
    """K_n."""
    i, j = np.triu_indices(n, k=1)
    return _mk(n, i, j, f"K{n}", family="complete")


def cycle(n: int) -> Graph:
    """C_n (n >= 3)."""
    i = np.arange(n)
    return _mk(n, i, (i + 1) % n, f"C{n}", family="cycle")


def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0))
    return _mk(n, i, i + 1, f"P{n}", family="path")


def star(n: int) -> Graph:
    """Hub 0 joined to leaves 1..n-1."""
    leaves = np.arange(1, n)
    return _mk(n, np.zeros_like(leaves), leaves, f"S{n}", family="star")


def wheel(n: int) -> Graph:
    """W_n with n vertices: hub 0 plus the rim cycle 1..n-1 (n >= 4)."""
    rim = np.arange(1, n)
    nxt = np.where(rim + 1 < n, rim + 1, 1)
    s = np.concatenate([np.zeros(n - 1, dtype=np.int64), rim])
    d = np.concatenate([rim, nxt])
    return _mk(n, s, d, f"W{n}", family="wheel")


def complete_bipartite(a: int, b: int) -> Graph:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return _mk(a + b, i.ravel(), j.ravel(), f"K{a},{b}", family="complete_bipartite")


def grid(rows: int, cols: int) -> Graph:
    vid = np.arange(rows * cols).reshape(rows, cols)
    s = np.concatenate([vid[:, :-1].ravel(), vid[:-1, :].ravel()])
    d = np.concatenate([vid[:, 1:].ravel(), vid[1:, :].ravel()])
    return _mk(rows * cols, s, d, f"grid{rows}x{cols}", family="grid")


def random_bipartite(a: int, b: int, p: float, seed: int) -> Graph:
    """Each of the a*b cross pairs kept with probability p (counter stream)."""
    lib = _load()
    key = lib.gg_stream_key(seed & (2**64 - 1), 0x42495054)
    keep = np.array([lib.gg_draw(key, k) >> 11 for k in range(a * b)], dtype=np.uint64)
    mask = keep < np.uint64(int(p * float(1 << 53)))
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return _mk(a + b, i.ravel()[mask], j.ravel()[mask], f"rbip{a},{b}", family="random_bipartite")


def disjoint_union(graphs) -> Graph:
    """Place graphs side by side (ids of graph i shifted by the sizes before)."""
    base = 0
    ss, dd = [], []
    for g in graphs:
        ss.append(g.src.astype(np.int64) + base)
        dd.append(g.dst.astype(np.int64) + base)
        base += g.n
    if not ss:
        return _mk(0, np.empty(0), np.empty(0), "union")
    return _mk(base, np.concatenate(ss), np.concatenate(dd), "union", family="union")


# ------------------------------------------------------ workload recipes
def _u01(key: int, ctr: int) -> float:
    return ((_load().gg_draw(key, ctr) >> 11) + 0.5) / float(1 << 53)


def batch_specs(num_graphs: int = 4096, seed_base: int = 4096, n_min: int = 64,
                n_max: int = 65536):
    """Parameters of the batched workload: the first half Erdos-Renyi with
    mean degree ~U[8, 64], the second half Barabasi-Albert with m ~U{2..16};
    n = floor(log-uniform[n_min, n_max]).  Returns a list of dicts."""
    lib = _load()
    specs = []
    half = num_graphs // 2
    for g in range(num_graphs):
        key = lib.gg_stream_key(seed_base + g, 0xBA7C4)
        n = int(math.floor(math.exp(math.log(n_min) + _u01(key, 0) *
                                    (math.log(n_max) - math.log(n_min)))))
        n = min(max(n, n_min), n_max)
        if g < half:
            dbar = 8.0 + 56.0 * _u01(key, 1)
            p = min(1.0, dbar / max(n - 1, 1))
            specs.append(dict(kind="er", n=n, p=p, mean_degree=dbar, seed=seed_base + g))
        else:
            mba = 2 + int(_u01(key, 2) * 15)
            specs.append(dict(kind="ba", n=n, m=mba, seed=seed_base + g))
    return specs


def from_spec(spec) -> Graph:
    if spec["kind"] == "er":
        return erdos_renyi(spec["n"], spec["p"], spec["seed"])
    if spec["kind"] == "ba":
        return barabasi_albert(spec["n"], spec["m"], spec["seed"])
    if spec["kind"] == "rmat":
        return rmat(spec["scale"], spec.get("edge_factor", 16), seed=spec["seed"])
    if spec["kind"] == "chung_lu":
        return chung_lu(spec["n"], spec.get("gamma", 2.1), spec.get("mean_degree", 20.0),
                        spec["seed"])
    raise ValueError(spec)


def batch_mix(num_graphs: int = 4096, seed_base: int = 4096, n_min: int = 64,
              n_max: int = 65536, threads: int = 8):
    """The batched workload as a list of raw graphs (see :func:`batch_specs`).
    Graphs are generated on `threads` host threads (the C generators release
    the interpreter lock and depend only on their own seeds)."""
    specs = batch_specs(num_graphs, seed_base, n_min, n_max)
    _load()
    if threads <= 1:
        return [from_spec(s) for s in specs]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(from_spec, specs))


def serving_specs(pool_size: int = 128, seed_base: int = 9000, scale_min: int = 12,
                  scale_max: int = 22, cl_n_min: int = 10**4, cl_n_max: int = 10**6):
    """Request pool of the serving workload: half R-MAT (scale uniform in
    [scale_min, scale_max], edge factor 16), half Chung-Lu (gamma 2.1, mean
    degree 20, n log-uniform in [cl_n_min, cl_n_max])."""
    lib = _load()
    specs = []
    for i in range(pool_size):
        key = lib.gg_stream_key(seed_base + i, 0x5E4E)
        if i % 2 == 0:
            sc = scale_min + int(_u01(key, 0) * (scale_max - scale_min + 1))
            specs.append(dict(kind="rmat", scale=min(sc, scale_max), edge_factor=16,
                              seed=seed_base + i))
        else:
            n = int(math.exp(math.log(cl_n_min) + _u01(key, 1) *
                             (math.log(cl_n_max) - math.log(cl_n_min))))
            specs.append(dict(kind="chung_lu", n=n, gamma=2.1, mean_degree=20.0,
                              seed=seed_base + i))
    return specs
