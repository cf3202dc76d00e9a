"""The request loop on the GPU: every request's (T, |H|) in a mix of
overlapping requests on several slots equals the same graph counted alone,
and the oracle's T."""
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _pool_graphs():
    return [graphgen.rmat(10, seed=1), graphgen.rmat(12, seed=2), graphgen.rmat(13, seed=3),
            graphgen.chung_lu(10000, 2.1, 20.0, seed=4), graphgen.chung_lu(30000, 2.1, 20.0, seed=5),
            graphgen.rmat(11, seed=6), graphgen.complete(60), graphgen.grid(40, 40)]


@pytest.mark.parametrize("tight", [False, True])
def test_serving_mix_equals_alone(tight):
    import torch
    import paper_2210_00389_amd as tc
    from paper_2210_00389_amd import serve
    graphs = _pool_graphs()
    pool, sizes = serve.build_pool(graphs)
    alone = {}
    for gid, g in enumerate(graphs):
        G = tc.from_host_pairs(g.n, g.src, g.dst)
        r = tc.count(G)
        alone[gid] = (r.T, r.h)
        assert r.T == oracle.triangle_count(oracle.from_graph(g)), gid
    total = sum(gb + serve.count_ws_bytes(n, nnz) for n, nnz, gb in sizes.values())
    biggest = max(gb + serve.count_ws_bytes(n, nnz) for n, nnz, gb in sizes.values())
    # roomy: everything fits at once; tight: the largest request alone nearly
    # fills the budget, so resident graphs must be evicted
    budget = biggest + 100_000 if tight else 4 * total
    reqs = serve.make_requests(sizes, serve.count_ws_bytes, rate=3000.0, count=80, seed=11)
    print(f"case: serving mix budget={budget}", flush=True)
    st = serve.Server(serve.GpuExecutor(pool, 3), slots=3, budget_bytes=budget).run(reqs)
    torch.cuda.synchronize()
    for r in reqs:
        assert (r.triangles, r.h) == alone[r.graph_id], (r.rid, r.graph_id)
    assert st["max_running"] > 1
    assert st["p99_ms"] >= st["p50_ms"] > 0
    if tight:
        assert st["evictions"] > 0


def test_serving_levels_digest():
    """With the levels digest on, every request also carries the digest of
    its BFS levels, equal to the digest of the oracle's levels (Alg. 1
    scan order, default root)."""
    import torch
    from paper_2210_00389_amd import serve
    graphs = _pool_graphs()[:5]
    want = {}
    for gid, g in enumerate(graphs):
        c = oracle.from_graph(g)
        want[gid] = serve.levels_digest(oracle.bfs_levels(c).levels)
    pool, sizes = serve.build_pool(graphs)
    reqs = serve.make_requests(sizes, serve.count_ws_bytes, rate=2000.0, count=30, seed=12)
    print("case: serving with levels digest", flush=True)
    budget = 4 * sum(gb + serve.count_ws_bytes(n, nnz) for n, nnz, gb in sizes.values())
    serve.Server(serve.GpuExecutor(pool, 2, levels_hash=True), slots=2, budget_bytes=budget).run(reqs)
    torch.cuda.synchronize()
    for r in reqs:
        assert r.levels_hash == want[r.graph_id], (r.rid, r.graph_id)


def test_serving_same_graph_at_once():
    """Many requests for one graph arriving together on four slots: the
    first admitted uploads it while the others start at once; every answer
    equals the graph counted alone (a slot must never count a graph whose
    upload on another slot's stream has not finished)."""
    import torch
    import paper_2210_00389_amd as tc
    from paper_2210_00389_amd import serve
    graphs = [graphgen.rmat(16, seed=21)]
    G = tc.from_host_pairs(graphs[0].n, graphs[0].src, graphs[0].dst)
    want = (tc.count(G).T, tc.count(G).h)
    pool, sizes = serve.build_pool(graphs)
    budget = 8 * sum(gb + serve.count_ws_bytes(n, nnz) for n, nnz, gb in sizes.values())
    ex = serve.GpuExecutor(pool, 4)
    for rnd in range(3):
        print(f"case: same graph at once, round {rnd}", flush=True)
        reqs = serve.make_requests(sizes, serve.count_ws_bytes, rate=1e6, count=24, seed=30 + rnd)
        serve.Server(ex, slots=4, budget_bytes=budget).run(reqs)
        torch.cuda.synchronize()
        assert all((r.triangles, r.h) == want for r in reqs)
        assert sum(r.uploaded for r in reqs) >= 1
