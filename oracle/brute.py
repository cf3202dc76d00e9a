"""Brute-force checks for tiny graphs -- TEST INFRASTRUCTURE ONLY.

* :func:`triangles` lists every vertex triple {a < b < c} whose three edges
  exist, by trying all triples (the naive method of the related-work section,
  Omega(n^3)).
* :func:`all_pairs_hops` gives hop distances by Floyd-Warshall, so BFS levels
  can be pinned without any BFS code.

Pure Python loops; meant for n up to about 200.
"""
from __future__ import annotations

import numpy as np


def adjacency(n: int, src, dst) -> list[set[int]]:
    """Neighbour sets of the simple graph on raw pairs (loops dropped)."""
    adj = [set() for _ in range(n)]
    for s, d in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if s != d:
            adj[s].add(d)
            adj[d].add(s)
    return adj


def triangles(adj: list[set[int]]) -> list[tuple[int, int, int]]:
    """Every triple a < b < c with all three edges present."""
    n = len(adj)
    out = []
    for a in range(n):
        for b in range(a + 1, n):
            if b not in adj[a]:
                continue
            for c in range(b + 1, n):
                if c in adj[a] and c in adj[b]:
                    out.append((a, b, c))
    return out


def per_vertex(n: int, tris) -> np.ndarray:
    t = np.zeros(n, dtype=np.int64)
    for a, b, c in tris:
        t[a] += 1
        t[b] += 1
        t[c] += 1
    return t


def all_pairs_hops(adj: list[set[int]]) -> np.ndarray:
    """Hop distance between every pair (-1 when unreachable), Floyd-Warshall."""
    n = len(adj)
    inf = n + 1
    d = [[inf] * n for _ in range(n)]
    for i in range(n):
        d[i][i] = 0
        for j in adj[i]:
            d[i][j] = 1
    for k in range(n):
        dk = d[k]
        for i in range(n):
            dik = d[i][k]
            if dik == inf:
                continue
            di = d[i]
            for j in range(n):
                if dik + dk[j] < di[j]:
                    di[j] = dik + dk[j]
    out = np.array(d, dtype=np.int64)
    out[out == inf] = -1
    return out
