"""Pins of the oracle's triangle finding and per-edge supports (the
enumeration of Alg. 1, each accepted (u, v, w) reported once).

* the listed triangles are exactly the brute-force triangles (all triples
  with three edges, the naive method of the related-work section), with no
  repeats, on random and structured small graphs;
* closed forms: K_n lists all C(n, 3) triples, the wheel its n - 1 rim
  triangles, bipartite graphs none;
* the set does not depend on the BFS root (Thm. 2: T is root-independent,
  and the triangles themselves are the graph's);
* the support of every edge equals |N(u) ∩ N(v)| (each common neighbour
  closes exactly one triangle on that edge), is the same in both
  orientations, and sums to 6T.
"""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute


def _tris(g, root=-1):
    c = oracle.from_graph(g)
    L = oracle.bfs_levels(c, root).levels
    return c, L, oracle.list_triangles(c, L)


GRAPHS = [graphgen.erdos_renyi(40, 0.25, 1), graphgen.erdos_renyi(60, 0.1, 2), graphgen.barabasi_albert(50, 4, 3),
          graphgen.rmat(6, 8, seed=4), graphgen.disjoint_union([graphgen.complete(6), graphgen.wheel(8),
                                                                 graphgen.cycle(5), graphgen.path(4)]),
          graphgen.grid(5, 6)]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_listing_equals_brute_force(g):
    c, L, tri = _tris(g)
    got = [tuple(t) for t in tri.tolist()]
    assert all(a < b < cc for a, b, cc in got)
    assert len(set(got)) == len(got)
    assert sorted(got) == brute.triangles(brute.adjacency(g.n, g.src, g.dst))
    assert len(got) == oracle.count(c, L).triangles


def test_listing_closed_forms():
    _, _, t = _tris(graphgen.complete(9))
    assert sorted(map(tuple, t.tolist())) == list(itertools.combinations(range(9), 3))
    w = graphgen.wheel(12)
    _, _, t = _tris(w)
    assert len(t) == 11
    hub = int(np.bincount(np.concatenate([w.src, w.dst])).argmax())
    assert all(hub in row for row in t.tolist())
    for g in (graphgen.complete_bipartite(5, 7), graphgen.grid(6, 6), graphgen.cycle(8), graphgen.star(10)):
        assert _tris(g)[2].shape == (0, 3)
    _, _, t = _tris(graphgen.cycle(3))
    assert t.tolist() == [[0, 1, 2]]


def test_listing_root_invariant():
    g = graphgen.barabasi_albert(80, 5, 7)
    ref = sorted(map(tuple, _tris(g)[2].tolist()))
    for r in (0, 17, 79):
        assert sorted(map(tuple, _tris(g, r)[2].tolist())) == ref


@pytest.mark.parametrize("g", [graphgen.erdos_renyi(300, 0.05, 5), graphgen.barabasi_albert(1500, 6, 6),
                               graphgen.rmat(10, 16, seed=1)], ids=lambda g: g.name)
def test_supports_are_common_neighbour_counts(g):
    c = oracle.from_graph(g)
    L = oracle.bfs_levels(c).levels
    sup = oracle.edge_supports(c, L)
    off, cols = c.row_offsets, c.cols
    rows = np.repeat(np.arange(c.n), np.diff(off))
    common = np.array([np.intersect1d(cols[off[u]:off[u + 1]], cols[off[v]:off[v + 1]], assume_unique=True).size
                       for u, v in zip(rows.tolist(), cols.tolist())], dtype=np.int64)
    assert np.array_equal(sup, common)
    T = oracle.count(c, L).triangles
    assert int(sup.sum()) == 6 * T
    # both orientations agree
    rev = np.array([np.searchsorted(cols[off[v]:off[v + 1]], u) + off[v] for u, v in zip(rows.tolist(), cols.tolist())])
    assert np.array_equal(sup, sup[rev])


def test_empty_and_edgeless():
    c = oracle.from_graph(graphgen.path(1))
    assert oracle.list_triangles(c, oracle.bfs_levels(c).levels).shape == (0, 3)
    assert oracle.edge_supports(c, oracle.bfs_levels(c).levels).size == 0
    assert math.comb(3, 3) == 1
