"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: brute force
over all triples, Floyd-Warshall hop counts, networkx and scipy library
routines, closed forms, and the invariants the paper proves (Lemma 1: every
triangle has a horizontal edge; Lemma 2: exactly one or three; Thm. 2: the
count does not depend on the BFS roots).
"""
import itertools
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import graphgen
import oracle
from oracle import brute


def csr_of(g):
    return oracle.from_graph(g)


def small_graph(kind, n, seed):
    if kind == "er":
        return graphgen.erdos_renyi(n, 0.25, seed)
    if kind == "ba":
        return graphgen.barabasi_albert(n, 3, seed)
    if kind == "rmat":
        return graphgen.rmat(max(2, int(math.log2(max(n, 4)))), 4, seed=seed)
    if kind == "union":
        return graphgen.disjoint_union([graphgen.erdos_renyi(n // 2, 0.3, seed),
                                        graphgen.cycle(5), graphgen.complete(4),
                                        graphgen.Graph(3, np.zeros(0, np.int32),
                                                       np.zeros(0, np.int32))])
    raise ValueError(kind)


# ----------------------------------------------------------------- CSR
def test_build_csr_literal():
    # loops, repeats and both orientations collapse to one simple graph
    src = np.array([0, 1, 1, 2, 3, 2, 0, 3], dtype=np.int32)
    dst = np.array([1, 0, 1, 0, 3, 3, 2, 0], dtype=np.int32)
    c = oracle.build_csr(5, src, dst)
    assert c.row_offsets.tolist() == [0, 3, 4, 6, 8, 8]
    assert c.cols.tolist() == [1, 2, 3, 0, 0, 3, 0, 2]
    assert oracle.validate_csr(c) == 0


def test_build_csr_matches_networkx():
    import networkx as nx
    g = graphgen.rmat(8, 8, seed=3)
    c = csr_of(g)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(g.src, g.dst) if a != b)
    assert c.m == G.number_of_edges()
    for v in range(g.n):
        assert c.cols[c.row_offsets[v]:c.row_offsets[v + 1]].tolist() == sorted(G.neighbors(v))


def test_build_csr_out_of_range():
    with pytest.raises(oracle.OracleError) as e:
        oracle.build_csr(3, np.array([0], np.int32), np.array([3], np.int32))
    assert e.value.code == -4


@pytest.mark.parametrize("mutate,code", [
    ("offsets", -3), ("range", -4), ("unsorted", -5), ("dup", -6), ("self", -7), ("asym", -8)])
def test_validate_errors(mutate, code):
    off = np.array([0, 2, 4, 6], dtype=np.int64)
    cols = np.array([1, 2, 0, 2, 0, 1], dtype=np.int32)  # triangle
    c = oracle.CSR(3, off.copy(), cols.copy())
    assert oracle.validate_csr(c) == 0
    if mutate == "offsets":
        c.row_offsets[1] = 5
        c.row_offsets[2] = 4
    elif mutate == "range":
        c.cols[0] = 7
    elif mutate == "unsorted":
        c.cols[0], c.cols[1] = 2, 1
    elif mutate == "dup":
        c.cols[1] = 1
    elif mutate == "self":
        c.cols[0] = 0
    elif mutate == "asym":
        c = oracle.CSR(3, np.array([0, 1, 1, 1], np.int64), np.array([1], np.int32))
    assert oracle.validate_csr(c) == code


# ------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", range(3, 14))
def test_complete(n):
    c = csr_of(graphgen.complete(n))
    lv = oracle.bfs_levels(c)
    assert oracle.triangle_count(c) == math.comb(n, 3)
    assert oracle.edge_count(c) == math.comb(n, 3)
    hu, _ = oracle.cover_edges(c, lv.levels)
    assert len(hu) == math.comb(n - 1, 2)  # every edge not at the root
    # any root: K_n is vertex transitive, so |H| and T do not move
    for r in range(n):
        lr = oracle.bfs_levels(c, r).levels
        assert lr[r] == 0 and (lr[np.arange(n) != r] == 1).all()
        assert oracle.count(c, lr).triangles == math.comb(n, 3)


@pytest.mark.parametrize("n", range(5, 16))
def test_wheel(n):
    c = csr_of(graphgen.wheel(n))
    lv = oracle.bfs_levels(c)
    assert oracle.default_root(c) == 0  # the hub has the largest degree
    assert oracle.triangle_count(c) == n - 1
    hu, hv = oracle.cover_edges(c, lv.levels)
    assert len(hu) == n - 1  # the rim
    assert (hu > 0).all() and (hv > 0).all()


def test_wheel4_is_k4():
    assert oracle.triangle_count(csr_of(graphgen.wheel(4))) == 4


@pytest.mark.parametrize("n", range(3, 20))
def test_cycle(n):
    c = csr_of(graphgen.cycle(n))
    lv = oracle.bfs_levels(c)
    assert oracle.triangle_count(c) == (1 if n == 3 else 0)
    hu, _ = oracle.cover_edges(c, lv.levels)
    assert len(hu) == (n % 2)  # one horizontal edge closes an odd cycle
    # root 0 (all degrees tie): levels are the cycle distances
    d = np.minimum(np.arange(n), n - np.arange(n))
    assert (lv.levels == d).all()


@pytest.mark.parametrize("g", [graphgen.complete_bipartite(3, 5), graphgen.complete_bipartite(7, 7),
                               graphgen.grid(6, 9), graphgen.star(12), graphgen.path(17),
                               graphgen.random_bipartite(20, 25, 0.3, 7)])
def test_bipartite_has_no_cover_edges(g):
    c = csr_of(g)
    lv = oracle.bfs_levels(c)
    hu, _ = oracle.cover_edges(c, lv.levels)
    assert len(hu) == 0  # BFS levels 2-colour a bipartite graph
    assert oracle.triangle_count(c) == 0
    assert oracle.edge_count(c) == 0


def test_star_and_path_levels():
    c = csr_of(graphgen.star(9))
    lv = oracle.bfs_levels(c).levels
    assert lv[0] == 0 and (lv[1:] == 1).all()
    c = csr_of(graphgen.path(9))
    # all degrees 2 except the ends; the smallest id of degree 2 is vertex 1
    lv = oracle.bfs_levels(c).levels
    assert lv.tolist() == [1, 0, 1, 2, 3, 4, 5, 6, 7]


def test_empty_and_edgeless():
    c = oracle.build_csr(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert c.n == 0 and oracle.triangle_count(c) == 0
    c = oracle.build_csr(6, np.zeros(0, np.int32), np.zeros(0, np.int32))
    lv = oracle.bfs_levels(c)
    assert (lv.levels == 0).all() and lv.num_roots == 6
    assert oracle.triangle_count(c) == 0


# ------------------------------------------------ random small graphs
def component_roots(adj, r0):
    """Alg. 1 roots from brute-force reachability: r0, then the smallest id of
    every other component."""
    n = len(adj)
    hops = brute.all_pairs_hops(adj)
    roots = np.full(n, -1)
    if n == 0:
        return roots, hops
    for v in range(n):
        if hops[r0, v] >= 0:
            roots[v] = r0
    for v in range(n):
        if roots[v] < 0:
            for w in range(n):
                if hops[v, w] >= 0 and roots[w] < 0:
                    roots[w] = v
    return roots, hops


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(kind=st.sampled_from(["er", "ba", "rmat", "union"]), n=st.integers(2, 40),
       seed=st.integers(0, 10**6))
def test_random_small_against_brute_force(kind, n, seed):
    g = small_graph(kind, n, seed)
    c = csr_of(g)
    adj = brute.adjacency(g.n, g.src, g.dst)
    tris = brute.triangles(adj)
    lv = oracle.bfs_levels(c)
    L = lv.levels
    # levels: hop distance from the Alg. 1 root of each component
    r0 = oracle.default_root(c)
    if g.n:
        roots, hops = component_roots(adj, r0)
        assert all(L[v] == hops[roots[v], v] for v in range(g.n))
        assert lv.num_roots == len(set(roots.tolist()))
    # counts: both intersection modes, the edge iterator and brute force
    r_hash = oracle.count(c, L, 0, per_edge=True, per_vertex=True)
    r_merge = oracle.count(c, L, 1, per_edge=True, per_vertex=True)
    assert r_hash.triangles == r_merge.triangles == len(tris) == oracle.edge_count(c)
    assert (r_hash.per_vertex == brute.per_vertex(g.n, tris)).all()
    assert (r_merge.per_vertex == r_hash.per_vertex).all()
    assert r_hash.per_vertex.sum() == 3 * len(tris)
    assert r_hash.per_edge.sum() == len(tris)
    assert (r_hash.per_edge == r_merge.per_edge).all()
    # Lemma 1 / Lemma 2: one or three horizontal edges per triangle
    hu, hv = oracle.cover_edges(c, L)
    hset = set(zip(hu.tolist(), hv.tolist()))
    for a, b, cc in tris:
        k = sum(e in hset for e in [(a, b), (a, cc), (b, cc)])
        assert k in (1, 3)
    # H is exactly the same-level edges, u < v, sorted
    expect = sorted((u, v) for u in range(g.n) for v in adj[u] if u < v and L[u] == L[v])
    assert list(zip(hu.tolist(), hv.tolist())) == expect
    # per-edge support: c(u,v) <= |N(u) ∩ N(v)|, and matches the one-edge call
    for i, (u, v) in enumerate(zip(hu.tolist(), hv.tolist())):
        assert 0 <= r_hash.per_edge[i] <= len(adj[u] & adj[v])
        assert oracle.edge_support(c, L, u, v) == r_hash.per_edge[i]


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10**6), n=st.integers(5, 60))
def test_root_and_relabel_invariance(seed, n):
    g = graphgen.disjoint_union([graphgen.erdos_renyi(n, 0.2, seed), graphgen.barabasi_albert(n, 2, seed)])
    c = csr_of(g)
    T = oracle.triangle_count(c)
    rng = np.random.default_rng(seed)
    for r in rng.integers(0, g.n, size=4):
        L = oracle.bfs_levels(c, int(r)).levels
        assert oracle.count(c, L, 0).triangles == T  # Thm. 2 holds for any BFS root
        assert oracle.count(c, L, 1).triangles == T
    perm_g = graphgen.relabel(g, seed + 1)
    assert oracle.triangle_count(csr_of(perm_g)) == T


def test_levels_match_scipy_shortest_paths():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path, connected_components
    g = graphgen.rmat(11, 4, seed=5)
    c = csr_of(g)
    A = csr_matrix((np.ones(c.nnz), c.cols, c.row_offsets), shape=(c.n, c.n))
    ncomp, lab = connected_components(A, directed=False)
    r0 = oracle.default_root(c)
    roots = {lab[r0]: r0}
    for v in range(c.n):
        roots.setdefault(lab[v], v)
    rl = sorted(set(roots.values()))
    D = shortest_path(A, unweighted=True, directed=False, indices=rl)
    row_of = {r: i for i, r in enumerate(rl)}
    lv = oracle.bfs_levels(c)
    expect = np.array([D[row_of[roots[lab[v]]], v] for v in range(c.n)])
    assert (lv.levels == expect).all()
    assert lv.num_roots == ncomp


def test_rmat_matches_networkx():
    import networkx as nx
    g = graphgen.rmat(10, 16, seed=1)
    c = csr_of(g)
    G = nx.Graph()
    G.add_nodes_from(range(c.n))
    rows = np.repeat(np.arange(c.n), np.diff(c.row_offsets))
    G.add_edges_from(zip(rows.tolist(), c.cols.tolist()))
    tri = nx.triangles(G)
    res = oracle.count(c, oracle.bfs_levels(c).levels, 0, per_vertex=True)
    assert res.triangles == sum(tri.values()) // 3
    assert res.per_vertex.tolist() == [tri[v] for v in range(c.n)]


def test_bfs_invariants_rmat():
    c = csr_of(graphgen.rmat(12, 16, seed=2))
    L = oracle.bfs_levels(c).levels
    rows = np.repeat(np.arange(c.n), np.diff(c.row_offsets))
    assert (np.abs(L[rows] - L[c.cols]) <= 1).all()  # BFS levels move by at most one
    # every vertex at level > 0 has a neighbour one level up
    has_parent = np.zeros(c.n, bool)
    has_parent[rows[L[c.cols] == L[rows] - 1]] = True
    assert (has_parent | (L == 0)).all()


def test_golden_rmat_s10_reproduces():
    """The stored S10 values (written by tests/golden/make_golden.py from the
    oracle) still come out of the generator + oracle on this machine."""
    import json
    import os
    import hashlib
    path = os.path.join(os.path.dirname(__file__), "golden", "rmat_s10.json")
    gold = json.load(open(path))
    c = csr_of(graphgen.rmat(10, 16, seed=1))
    lv = oracle.bfs_levels(c)
    assert (c.n, c.m) == (gold["n"], gold["m"])
    assert hashlib.sha256(lv.levels.astype("<i4").tobytes()).hexdigest() == gold["levels_sha256"]
    assert oracle.count(c, lv.levels).triangles == gold["triangles"] == gold["edge_iterator_triangles"]


def test_count_rows_partition_sums_to_T():
    c = csr_of(graphgen.rmat(11, 16, seed=4))
    L = oracle.bfs_levels(c).levels
    T = oracle.count(c, L).triangles
    cuts = [0, 100, 700, 1500, c.n]
    parts = [oracle.count_rows(c, L, a, b) for a, b in zip(cuts, cuts[1:])]
    assert sum(parts) == T
    assert oracle.count_rows(c, L, 0, c.n, mode=1) == T


def test_count_rows_strided_phases_sum_to_T():
    """The strided row samples of one stride partition the rows: their
    counts sum to T (pinned against brute force) for several strides, in
    both intersection modes, and stride 1 is the full count."""
    g = graphgen.rmat(9, 16, seed=4)
    c = oracle.from_graph(g)
    L = oracle.bfs_levels(c).levels
    T = len(brute.triangles(brute.adjacency(g.n, g.src, g.dst)))
    assert oracle.count(c, L).triangles == T
    for stride in (1, 2, 7, 64, c.n + 5):
        for mode in (0, 1):
            parts = [oracle.count_rows_strided(c, L, ph, stride, mode) for ph in range(stride)]
            assert sum(parts) == T, (stride, mode)
    assert oracle.count_rows_strided(c, L, 0, 1) == T
    # one phase equals the sum of its rows counted one by one
    rows = range(3, c.n, 11)
    assert oracle.count_rows_strided(c, L, 3, 11) == sum(oracle.count_rows(c, L, u, u + 1) for u in rows)
