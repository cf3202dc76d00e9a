"""Pins of oracle.work_counters (the work measures of the cost analysis in
Sec. III): brute-force loops over adjacency sets on small random graphs,
closed forms for K_n, and zero horizontal work on bipartite graphs."""
from math import comb

import numpy as np
import pytest

import graphgen
import oracle


def _brute(c, L):
    adj = [set(c.cols[c.row_offsets[x]:c.row_offsets[x + 1]].tolist()) for x in range(c.n)]
    fwd = [sum(1 for w in adj[x] if w > x) for x in range(c.n)]
    h = hmin = hsum = emin = 0
    for u in range(c.n):
        for v in adj[u]:
            if v <= u:
                continue
            emin += min(fwd[u], fwd[v])
            if L[u] == L[v]:
                h += 1
                hmin += min(len(adj[u]), len(adj[v]))
                hsum += len(adj[u]) + len(adj[v])
    return dict(h=h, h_min_deg=hmin, h_sum_deg=hsum, edge_min_fwd=emin)


@pytest.mark.parametrize("seed", range(6))
def test_work_counters_brute_force(seed):
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        g = graphgen.erdos_renyi(int(rng.integers(20, 80)), 0.15, seed)
    elif kind == 1:
        g = graphgen.barabasi_albert(int(rng.integers(20, 80)), 3, seed)
    else:
        g = graphgen.rmat(6, 8, seed=seed)
    c = oracle.from_graph(g)
    L = oracle.bfs_levels(c).levels
    got = oracle.work_counters(c, L)
    assert got == _brute(c, L)
    assert got["h"] == len(oracle.cover_edges(c, L)[0])


@pytest.mark.parametrize("n", [4, 9, 30])
def test_work_counters_complete(n):
    """K_n from root 0: H is every pair of the other n - 1 vertices, all of
    degree n - 1; d+(x) = n - 1 - x, and each edge (u, v) takes d+(v)."""
    c = oracle.from_graph(graphgen.complete(n))
    got = oracle.work_counters(c, oracle.bfs_levels(c, 0).levels)
    assert got["h"] == comb(n - 1, 2)
    assert got["h_min_deg"] == comb(n - 1, 2) * (n - 1)
    assert got["h_sum_deg"] == 2 * comb(n - 1, 2) * (n - 1)
    assert got["edge_min_fwd"] == sum(v * (n - 1 - v) for v in range(n))


def test_work_counters_bipartite():
    c = oracle.from_graph(graphgen.grid(7, 9))
    got = oracle.work_counters(c, oracle.bfs_levels(c).levels)
    assert got["h"] == 0 and got["h_min_deg"] == 0 and got["h_sum_deg"] == 0
    assert got["edge_min_fwd"] > 0
