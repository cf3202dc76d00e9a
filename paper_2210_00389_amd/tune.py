"""Autotuner of the single-graph count (tc_count_tuned) and of the
comparator (tc_count_edge_baseline_tuned).

The knobs of tc_tuning that schedule the intersection stage -- the light /
heavy split of anchors, the bitmap-or-hash rule of the on-chip tables, the
work-item size, how the smallest-table bin hands out items and whether the
table bins run one after another or side by side -- are searched by
coordinate descent from the compiled defaults: each knob in turn takes every
value of its list with the others at their best so far, timed on the device
(median of `reps` calls, HIP events on the call's stream), and is kept when it
is faster by more than `min_gain`.  Every candidate must give the same count.
The choice is cached per graph class (path, log2 n, log2 nnz) in
_build/autotune.json beside the batch autotuner's entries.
"""
from __future__ import annotations

import json
import os
import statistics

import numpy as np
import torch

from .api import Graph, TcError, Workspace, count, count_edge_baseline

SPACE = {
    # which path: the one-workgroup path for graphs within 65536 vertices
    # never, or whatever their entry count (no effect on larger graphs)
    "small_max_n": [-1],
    "small_max_nnz": [2**31 - 1],
    "item_log2": [16, 17, 18, 19, 20, 21],
    "light_max": [16, 24, 32],
    "dn_light": [8, 16, 32, 64],
    "bitmap_member_words": [2, 4, 8, 32, 64],
    "bitmap_desc_words": [8, 16, 32, 64, 128],
    "bin0_mode": [1, 2],
    "bins_mode": [1, 2],
    "twolevel_sparsity": [-1, 16, 256],
    "bin0_max_desc": [-1, 256, 4096],
    "up_anchor_min": [-1, 256],
    "degree_groups": [2, 4],
}
# the comparator has no down class and no one-workgroup path
EDGE_SPACE = {k: v for k, v in SPACE.items() if k not in ("dn_light", "small_max_n", "small_max_nnz", "up_anchor_min",
                                                          "degree_groups")}
# a shorter search for graphs whose calls take long (the benchmark's
# comparator at R-MAT scale 24): the knobs that moved it in measurements
EDGE_SPACE_SHORT = {"item_log2": [16, 17, 18], "bitmap_desc_words": [32], "bins_mode": [1],
                    "twolevel_sparsity": [-1, 16, 256]}


def _cache_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "autotune.json")


def graph_key(g: Graph, path: str) -> str:
    lg = lambda v: int(np.log2(max(v, 1)))  # noqa: E731
    return f"{path}:n{lg(g.n)}-z{lg(g.nnz)}"


def _timed(fn, reps: int):
    """(median ms of `reps` calls after one warm-up, the last call's result)."""
    stream = torch.cuda.current_stream()
    fn()
    ts = []
    out = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        out = fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts), out


def autotune_count(g: Graph, path: str = "cover", reps: int = 3, space: dict | None = None, min_gain: float = 0.01,
                   use_cache: bool = True, ws: Workspace | None = None, verbose: bool = False) -> dict:
    """The fastest tuning found for graph g on `path` ("cover": tc_count;
    "edge": the comparator), as a dict of tc_tuning fields ({} = defaults)."""
    key = graph_key(g, path)
    cpath = _cache_path()
    cache = {}
    if use_cache and os.path.exists(cpath):
        try:
            cache = json.load(open(cpath))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return dict(cache[key]["tuning"])
    space = space or (SPACE if path == "cover" else EDGE_SPACE)
    ws = ws or Workspace(g.cols.device)
    if path == "cover":
        res = count(g, ws=ws)

        def run(t):
            count(g, ws=ws, tuning=t, out=res)
            return res.triangles
    else:
        out = torch.zeros(1, dtype=torch.int64, device=g.cols.device)

        def run(t):
            return count_edge_baseline(g, ws=ws, tuning=t, out=out)
    best: dict = {}
    best_ms, out0 = _timed(lambda: run(None), reps)
    ref = int(out0.item())
    table = [[{}, best_ms]]
    if verbose:
        print(f"[autotune] {key} defaults: {best_ms:.3f} ms", flush=True)
    for knob, values in space.items():
        for v in values:
            cand = dict(best, **{knob: v})
            if cand == best:
                continue
            ms, got = _timed(lambda: run(cand), reps)
            if int(got.item()) != ref:
                raise TcError(-1, f"autotune: tuning {cand} changed the count")
            table.append([cand, ms])
            if verbose:
                print(f"[autotune] {key} {cand}: {ms:.3f} ms", flush=True)
            if ms < best_ms * (1.0 - min_gain):
                best, best_ms = cand, ms
    if use_cache:
        cache[key] = dict(tuning=best, ms=best_ms, default_ms=table[0][1], table=table)
        os.makedirs(os.path.dirname(cpath), exist_ok=True)
        with open(cpath, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(best)
