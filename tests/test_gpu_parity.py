"""GPU parity: every libtc entry point against the CPU oracle, element by
element, on seeded inputs (bit-exact: all outputs are integers)."""
import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tc():
    import torch
    from paper_2210_00389_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2210_00389_amd import build
        build.build()
    import paper_2210_00389_amd as tc
    torch.cuda.set_device(0)
    return tc


SMALL_ON = dict(small_max_n=65536, small_max_nnz=2**31 - 1)
SMALL_OFF = dict(small_max_n=-1)


def to_gpu(tc, g):
    return tc.from_host_pairs(g.n, g.src, g.dst, device="cuda")


def check_graph(tc, g, name="", root=-1, baseline=True, per_vertex=True):
    """Full parity of one raw graph: CSR, levels, |H|, H list, T, per-vertex
    counts and the comparator."""
    say(f"[parity] {name} n={g.n} pairs={g.num_pairs} root={root}")
    c = oracle.from_graph(g)
    G = to_gpu(tc, g)
    assert G.n == c.n and G.nnz == c.nnz
    assert np.array_equal(G.row_offsets.cpu().numpy(), c.row_offsets)
    assert np.array_equal(G.cols.cpu().numpy(), c.cols)
    lv = oracle.bfs_levels(c, root)
    L, nl = tc.bfs_levels(G, root)
    assert np.array_equal(L.cpu().numpy(), lv.levels), name
    assert nl == lv.num_levels
    hu, hv = oracle.cover_edges(c, lv.levels)
    gu, gv = tc.cover_edges(G, L)
    assert np.array_equal(gu.cpu().numpy(), hu) and np.array_equal(gv.cpu().numpy(), hv)
    want = oracle.count(c, lv.levels, per_vertex=per_vertex)
    res = tc.count(G, root=root, per_vertex=per_vertex, return_levels=True)
    assert res.T == want.triangles, (name, res.T, want.triangles)
    assert res.h == len(hu)
    assert np.array_equal(res.levels.cpu().numpy(), lv.levels)
    if per_vertex:
        assert np.array_equal(res.per_vertex.cpu().numpy(), want.per_vertex)
    # both paths of tc_count on every graph: the one-workgroup path forced on
    # (every graph within TC_BATCH_MAX_N vertices takes it) and forced off
    for tun in (SMALL_ON, SMALL_OFF):
        r2 = tc.count(G, root=root, return_levels=True, tuning=tun)
        assert (r2.T, r2.h) == (want.triangles, len(hu)), (name, tun)
        assert np.array_equal(r2.levels.cpu().numpy(), lv.levels), (name, tun)
    if baseline:
        assert int(tc.count_edge_baseline(G).item()) == want.triangles
    return c, G, want.triangles


# ---------------------------------------------------------- CSR build
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_build_csr_matches_oracle(tc, seed):
    for g in [graphgen.rmat(9, 8, seed=seed), graphgen.erdos_renyi(700, 0.01, seed),
              graphgen.barabasi_albert(900, 5, seed),
              graphgen.Graph(5, np.array([0, 1, 1, 2, 3, 2, 0, 3], np.int32),
                             np.array([1, 0, 1, 0, 3, 3, 2, 0], np.int32))]:
        say(f"[build] {g.name} seed={seed}")
        c = oracle.from_graph(g)
        G = to_gpu(tc, g)
        assert np.array_equal(G.row_offsets.cpu().numpy(), c.row_offsets)
        assert np.array_equal(G.cols.cpu().numpy(), c.cols)
        assert tc.validate(G) == 0


def test_build_csr_empty_and_out_of_range(tc):
    import torch
    G = tc.from_host_pairs(7, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert G.nnz == 0 and G.row_offsets.cpu().tolist() == [0] * 8
    G = tc.from_host_pairs(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert G.n == 0 and G.nnz == 0
    with pytest.raises(tc.TcError) as e:
        tc.from_host_pairs(4, np.array([0, 1], np.int32), np.array([2, 9], np.int32))
    assert e.value.status == -7
    torch.cuda.synchronize()


# ----------------------------------------------------------- validate
@pytest.mark.parametrize("mutate,code", [
    ("offsets", -10), ("range", -7), ("unsorted", -3), ("dup", -4), ("self", -5), ("asym", -6)])
def test_validate_errors(tc, mutate, code):
    off = np.array([0, 2, 4, 6], dtype=np.int64)
    cols = np.array([1, 2, 0, 2, 0, 1], dtype=np.int32)
    n = 3
    if mutate == "offsets":
        off = np.array([0, 4, 2, 6], dtype=np.int64)
    elif mutate == "range":
        cols[0] = 7
    elif mutate == "unsorted":
        cols[0], cols[1] = 2, 1
    elif mutate == "dup":
        cols[1] = 1
    elif mutate == "self":
        cols[0] = 0
    elif mutate == "asym":
        off = np.array([0, 1, 1, 1], np.int64)
        cols = np.array([1], np.int32)
    say(f"[validate] {mutate}")
    G = tc.from_host_csr(n, off, cols)
    assert tc.validate(G) == code
    with pytest.raises(tc.TcError) as e:
        tc.count(G, validate=True)
    assert e.value.status == code
    ok = tc.from_host_csr(3, np.array([0, 2, 4, 6], np.int64), np.array([1, 2, 0, 2, 0, 1], np.int32))
    assert tc.validate(ok) == 0
    assert tc.count(ok, validate=True).T == 1


# ------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [3, 4, 5, 17, 64, 65, 300])
def test_complete(tc, n):
    check_graph(tc, graphgen.complete(n), f"K{n}", baseline=True, per_vertex=n <= 64)


@pytest.mark.parametrize("n", [5, 6, 50, 3000])
def test_wheel(tc, n):
    check_graph(tc, graphgen.wheel(n), f"W{n}")


@pytest.mark.parametrize("g", [graphgen.cycle(3), graphgen.cycle(4), graphgen.cycle(101), graphgen.cycle(1000),
                               graphgen.path(2), graphgen.path(500), graphgen.star(20000),
                               graphgen.complete_bipartite(40, 70), graphgen.grid(30, 40),
                               graphgen.random_bipartite(50, 60, 0.2, 3)],
                         ids=lambda g: g.name)
def test_sparse_families(tc, g):
    check_graph(tc, g, g.name)


def test_complete_large_closed_form(tc):
    """K_4200: the probe set of vertex 1 (4198 forward cover edges) exceeds
    the on-chip table; closed forms C(n,3), C(n-1,2), C(n-1,2) per vertex."""
    n = 4200
    say(f"[closed form] K{n}")
    g = graphgen.complete(n)
    G = to_gpu(tc, g)
    res = tc.count(G, per_vertex=True)
    assert res.T == math.comb(n, 3)
    assert res.h == math.comb(n - 1, 2)
    pv = res.per_vertex.cpu().numpy()
    assert (pv == math.comb(n - 1, 2)).all()
    assert int(tc.count_edge_baseline(G).item()) == math.comb(n, 3)


def test_friendship_and_big_star(tc):
    """Windmill graph (k triangles through one hub) and a large wheel: long
    hub rows split into many segments, bottom-up BFS steps."""
    k = 60000
    hub = np.zeros(2 * k, np.int32)
    leaves = np.arange(1, 2 * k + 1, dtype=np.int32)
    s = np.concatenate([hub, leaves[0::2]])
    d = np.concatenate([leaves, leaves[1::2]])
    say("[closed form] windmill")
    G = tc.from_host_pairs(2 * k + 1, s, d)
    res = tc.count(G, per_vertex=True)
    assert res.T == k and res.h == k
    pv = res.per_vertex.cpu().numpy()
    assert pv[0] == k and (pv[1:] == 1).all()
    assert int(tc.count_edge_baseline(G).item()) == k
    n = 200001
    say("[closed form] W200001")
    Gw = to_gpu(tc, graphgen.wheel(n))
    res = tc.count(Gw)
    assert res.T == n - 1 and res.h == n - 1


def test_empty_and_edgeless(tc):
    import torch
    G = tc.from_host_pairs(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert tc.count(G).T == 0
    G = tc.from_host_pairs(9, np.zeros(0, np.int32), np.zeros(0, np.int32))
    res = tc.count(G, return_levels=True)
    assert res.T == 0 and res.h == 0 and (res.levels.cpu().numpy() == 0).all()
    L, nl = tc.bfs_levels(G)
    assert nl == 1 and (L.cpu().numpy() == 0).all()
    assert int(tc.count_edge_baseline(G).item()) == 0
    torch.cuda.synchronize()


# ------------------------------------------------- random graphs
@pytest.mark.parametrize("block", range(5))
def test_random_graphs(tc, block):
    rng = np.random.default_rng(1000 + block)
    for k in range(40):
        kind = rng.integers(0, 5)
        seed = int(rng.integers(0, 10**6))
        n = int(rng.integers(2, 400))
        if kind == 0:
            g = graphgen.erdos_renyi(n, float(rng.uniform(0.005, 0.3)), seed)
        elif kind == 1:
            g = graphgen.barabasi_albert(n, int(rng.integers(1, 8)), seed)
        elif kind == 2:
            g = graphgen.rmat(int(rng.integers(3, 10)), int(rng.integers(2, 20)), seed=seed)
        elif kind == 3:
            g = graphgen.chung_lu(max(n, 50), 2.1, float(rng.uniform(2, 12)), seed)
        else:
            g = graphgen.disjoint_union([graphgen.erdos_renyi(n, 0.05, seed), graphgen.complete(5),
                                         graphgen.cycle(7), graphgen.barabasi_albert(n // 2 + 2, 2, seed)])
        root = -1 if k % 3 else int(rng.integers(0, g.n))
        check_graph(tc, g, f"block{block}/{k} {g.name}", root=root)


def test_rmat_medium_full_parity(tc):
    """Scales 12-16: several tiles, hub rows over the short-row limit, heavy
    anchors with emitted tasks, bottom-up BFS."""
    for scale, seed in [(12, 1), (14, 7), (16, 1)]:
        check_graph(tc, graphgen.rmat(scale, 16, seed=seed), f"rmat{scale}", per_vertex=scale <= 14)


def test_golden_rmat_s10(tc):
    gold = json.load(open(os.path.join(GOLDEN, "rmat_s10.json")))
    G = to_gpu(tc, graphgen.rmat(10, 16, seed=1))
    res = tc.count(G, return_levels=True)
    digest = hashlib.sha256(res.levels.cpu().numpy().astype("<i4").tobytes()).hexdigest()
    assert (res.T, res.h, digest) == (gold["triangles"], gold["h"], gold["levels_sha256"])


def test_determinism(tc):
    G = to_gpu(tc, graphgen.rmat(14, 16, seed=3))
    outs = set()
    for _ in range(5):
        r = tc.count(G, return_levels=True)
        outs.add((r.T, r.h, hashlib.sha256(r.levels.cpu().numpy().tobytes()).hexdigest(),
                  int(tc.count_edge_baseline(G).item())))
    assert len(outs) == 1


def test_bfs_isolated_vertices_beside_one_component(tc):
    """The BFS from r0 reaches every vertex with an edge, so the vertices
    left are isolated and take level 0 without the component pass; from an
    isolated root the component pass levels the clique from its smallest id;
    with two cliques the pass runs with vertices of degree > 0 left."""
    g = graphgen.disjoint_union([graphgen.complete(12)] + [graphgen.path(1)] * 6)
    check_graph(tc, g, "K12 + 6 isolated")
    deg = np.diff(oracle.from_graph(g).row_offsets)
    check_graph(tc, g, "K12 + 6 isolated, isolated root", root=int(np.flatnonzero(deg == 0)[0]))
    g2 = graphgen.disjoint_union([graphgen.complete(12), graphgen.complete(7)] + [graphgen.path(1)] * 4)
    check_graph(tc, g2, "K12 + K7 + 4 isolated")


def test_small_path_stats_and_workspace(tc):
    """After the one-workgroup path the work statistics carry n, nnz and |H|
    (the rest zero); the call runs in a workspace of tc_workspace_bytes."""
    from paper_2210_00389_amd import _lib
    g = graphgen.rmat(10, 16, seed=1)
    G = to_gpu(tc, g)
    ws = tc.Workspace()
    r = tc.count(G, ws=ws, tuning=SMALL_ON)
    st = tc.read_stats(ws)
    assert (st["n"], st["nnz"], st["h"]) == (G.n, G.nnz, r.h)
    assert st["heavy_items"] == 0 and st["descriptors"] == 0
    assert ws.buf.numel() == tc.workspace_bytes(_lib.OP_COUNT, G.n, G.nnz)
    r_off = tc.count(G, tuning=SMALL_OFF)
    assert (r.T, r.h) == (r_off.T, r_off.h)


TUNINGS = [dict(light_max=1, dn_light=1), dict(light_max=8, dn_light=4, item_log2=12),
           dict(bitmap_member_words=1, bitmap_desc_words=1), dict(bitmap_member_words=1024, bitmap_desc_words=1024),
           dict(item_log2=24, bin0_mode=1, bins_mode=2), dict(item_log2=14, bin0_mode=2, bins_mode=1),
           dict(light_max=32, dn_light=1000, item_log2=16, bins_mode=2, bin0_mode=2),
           dict(twolevel_sparsity=1), dict(twolevel_sparsity=-1, bins_mode=1), dict(bin0_max_desc=1),
           dict(bin0_max_desc=-1, bitmap_member_words=64), dict(up_anchor_min=32),
           dict(up_anchor_min=32, light_max=8, dn_light=4, bitmap_member_words=1, bitmap_desc_words=1),
           dict(degree_groups=4), dict(degree_groups=4, up_anchor_min=32, bitmap_desc_words=1)]


def test_determinism_across_tunings(tc):
    """Every tuning of the intersection stage gives the oracle's T and |H|,
    for the cover count and the comparator, on graphs that exercise every
    table bin (R-MAT scales 12-16, a windmill hub, a complete graph beyond
    the on-chip tables)."""
    k = 5000
    hub = np.zeros(2 * k, np.int32)
    leaves = np.arange(1, 2 * k + 1, dtype=np.int32)
    windmill = graphgen.Graph(2 * k + 1, np.concatenate([hub, leaves[0::2]]), np.concatenate([leaves, leaves[1::2]]))
    graphs = [("rmat12", graphgen.rmat(12, 16, seed=5)), ("rmat14", graphgen.rmat(14, 16, seed=6)),
              ("rmat16", graphgen.rmat(16, 16, seed=7)), ("windmill", windmill), ("K1500", graphgen.complete(1500))]
    for name, g in graphs:
        if name == "K1500":  # closed forms: C(n,3) triangles, C(n-1,2) cover edges from any root
            T, h = math.comb(1500, 3), math.comb(1499, 2)
        else:
            c = oracle.from_graph(g)
            lv = oracle.bfs_levels(c)
            T = oracle.count(c, lv.levels).triangles
            h = len(oracle.cover_edges(c, lv.levels)[0])
        G = to_gpu(tc, g)
        for t in TUNINGS:
            say(f"[tuning] {name} {t}")
            r = tc.count(G, tuning=dict(t, small_max_n=-1))
            assert (r.T, r.h) == (T, h), (name, t)
            assert int(tc.count_edge_baseline(G, tuning=t).item()) == T, (name, t)


def test_autotune_count(tc):
    """The autotuner returns tunings whose counts equal the oracle's."""
    g = graphgen.rmat(13, 16, seed=9)
    G = to_gpu(tc, g)
    T = oracle.triangle_count(oracle.from_graph(g))
    small = {"item_log2": [17, 19], "bins_mode": [1, 2]}
    for path in ("cover", "edge"):
        say(f"[autotune] {path}")
        t = tc.autotune_count(G, path=path, reps=2, space=small, use_cache=False)
        assert set(t) <= set(small)
        got = tc.count(G, tuning=t).T if path == "cover" else int(tc.count_edge_baseline(G, tuning=t).item())
        assert got == T


def test_up_anchor_pairs(tc):
    """Down-class pairs (x, w) anchored at w (up_anchor_min): w streams
    Hfwd(x) against the Up part of its table when Up(w) is the longer list.
    T, |H| and the per-vertex counts equal the oracle's, and the statistics
    show the changed work: more task descriptors, fewer streamed elements."""
    for scale, seed in [(12, 3), (14, 7), (16, 1)]:
        g = graphgen.rmat(scale, 16, seed=seed)
        say(f"[up-anchor] rmat{scale}")
        c = oracle.from_graph(g)
        lv = oracle.bfs_levels(c)
        want = oracle.count(c, lv.levels, per_vertex=scale <= 14)
        G = to_gpu(tc, g)
        ws = tc.Workspace()
        r0 = tc.count(G, ws=ws, tuning=dict(small_max_n=-1, up_anchor_min=-1))
        st0 = tc.read_stats(ws)
        for upa in (32, 64, 256):
            r = tc.count(G, ws=ws, per_vertex=scale <= 14, tuning=dict(small_max_n=-1, up_anchor_min=upa))
            st = tc.read_stats(ws)
            assert (r.T, r.h) == (want.triangles, r0.h) == (r0.T, r0.h), (scale, upa)
            if scale <= 14:
                assert np.array_equal(r.per_vertex.cpu().numpy(), want.per_vertex), (scale, upa)
            if upa == 32:
                assert st["descriptors"] > st0["descriptors"], (scale, st, st0)
                assert sum(st["bin_elems"]) + st["light_elems"] < sum(st0["bin_elems"]) + st0["light_elems"]


def test_two_level_tables(tc):
    """Probe sets too large for an LDS bitmap or hash table take the
    two-level table (block bits in LDS, member words in global memory): a
    root adjacent to 2M vertices, two vertices B and C two levels down, B
    with 20000 up-neighbours spread over that level, C adjacent to B and to
    1000 of them (the cover edge (B, C) makes B the anchor of a two-level
    table), random edges inside the level, ids permuted (the comparator's
    root keeps a forward list over the whole id range).  T and |H| equal
    the oracle's on both paths and the statistics show two-level probes."""
    rng = np.random.default_rng(42)
    M = 2_000_000
    n = M + 3
    root, B, C = 0, M + 1, M + 2
    lvl1 = np.arange(1, M + 1)
    bn = rng.choice(lvl1, size=20_000, replace=False)
    ea = rng.choice(lvl1, size=300_000)
    eb = rng.choice(lvl1, size=300_000)
    src = np.concatenate([np.full(M, root), np.full(bn.size, B), ea, bn[:5000], [B], np.full(1000, C)])
    dst = np.concatenate([lvl1, bn, eb, bn[5000:10000], [C], bn[10000:11000]])
    perm = rng.permutation(n)
    z = int(np.flatnonzero(perm == 0)[0])
    perm[z], perm[root] = perm[root], 0  # the root takes id 0: its forward list spans every id
    g = graphgen.Graph(n, perm[src].astype(np.int32), perm[dst].astype(np.int32))
    say("[two-level] hub graph")
    c = oracle.from_graph(g)
    lv = oracle.bfs_levels(c)
    T = oracle.count(c, lv.levels).triangles
    h = len(oracle.cover_edges(c, lv.levels)[0])
    say(f"[two-level] oracle T={T} |H|={h}")
    G = to_gpu(tc, g)
    ws = tc.Workspace()
    r = tc.count(G, ws=ws)
    st = tc.read_stats(ws)
    say(f"[two-level] cover stats {st}")
    assert (r.T, r.h) == (T, h)
    # B (20000 up-neighbours, a two-level table) anchors its down-class pairs
    r2 = tc.count(G, ws=ws, tuning={"up_anchor_min": 32})
    assert (r2.T, r2.h) == (T, h)
    wb = tc.Workspace()
    Tb = int(tc.count_edge_baseline(G, ws=wb).item())
    stb = tc.read_stats(wb)
    say(f"[two-level] comparator stats {stb}")
    assert Tb == T
    assert st["twolevel_elems"] > 0 and stb["twolevel_elems"] > 0
