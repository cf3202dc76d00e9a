"""The request loop on the GPU: every request's (T, |H|) in a mix of
overlapping requests on several slots, alone or coalesced into batched
launches, equals the same graph counted alone and the oracle's values; the
serving pool's graphs (R-MAT up to scale 22, Chung-Lu up to n = 9e5) are
checked against the oracle's stored (T, |H|, levels digest)."""
import json
import os

import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _pool_graphs():
    return [graphgen.rmat(10, seed=1), graphgen.rmat(12, seed=2), graphgen.rmat(13, seed=3),
            graphgen.chung_lu(10000, 2.1, 20.0, seed=4), graphgen.chung_lu(30000, 2.1, 20.0, seed=5),
            graphgen.rmat(11, seed=6), graphgen.complete(60), graphgen.grid(40, 40)]


@pytest.mark.parametrize("tight,batching", [(False, False), (True, False), (False, True), (True, True)])
def test_serving_mix_equals_alone(tight, batching):
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
    ws_fn = (lambda n, nnz: serve.request_ws_bytes(n, nnz, batching))  # noqa: E731
    reqs = serve.make_requests(sizes, ws_fn, rate=3000.0, count=80, seed=11)
    print(f"case: serving mix budget={budget} batching={batching}", flush=True)
    st = serve.Server(serve.GpuExecutor(pool, 3), slots=3, budget_bytes=budget,
                      small=serve.small_request if batching else None).run(reqs)
    torch.cuda.synchronize()
    assert st["failed"] == 0, st["errors"]
    for r in reqs:
        assert (r.triangles, r.h) == alone[r.graph_id], (r.rid, r.graph_id, r.batched)
    if batching:
        assert st["batched"] > 0 and st["jobs"] < len(reqs)
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
    # the graph stays resident across the rounds: one upload in all, however
    # many slots asked for it at once
    assert ex.uploads == 1


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "serving_pool.json")


def _pool_subset(gold):
    """Every small graph of the serving pool (the coalesced ones), the
    largest Chung-Lu graph, one R-MAT scale 22 graph and a few in between."""
    rows = gold["graphs"]
    small = [r["i"] for r in rows if r["n"] <= 65536]
    cl = _largest(rows, "chung_lu")
    s22 = _largest(rows, "rmat")
    mid = [r["i"] for r in rows if 65536 < r["n"] <= 600000][:6]
    return sorted(set(small + mid + [cl, s22]))


def test_serving_pool_against_oracle():
    """A Poisson mix over the serving pool (batching on, levels digests on):
    every answer equals the oracle's stored T, |H| and levels digest."""
    import torch
    from paper_2210_00389_amd import serve
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/serving_pool.json not generated")
    gold = json.load(open(GOLDEN))
    ids = _pool_subset(gold)
    rows = {r["i"]: r for r in gold["graphs"]}
    print(f"case: serving pool subset of {len(ids)} graphs", flush=True)
    graphs = [graphgen.from_spec(rows[i]["spec"]) for i in ids]
    pool, sizes = serve.build_pool(graphs)
    del graphs
    for k, i in enumerate(ids):
        assert sizes[k][0] == rows[i]["n"] and sizes[k][1] == 2 * rows[i]["m"], i
    budget = 4 * sum(gb + serve.request_ws_bytes(n, nnz) for n, nnz, gb in sizes.values())
    reqs = serve.make_requests(sizes, serve.request_ws_bytes, rate=1000.0, count=160, seed=17)
    # the two largest graphs are asked for at least twice each, mid-stream
    for k in (ids.index(_largest(gold["graphs"], "chung_lu")), ids.index(_largest(gold["graphs"], "rmat"))):
        n, nnz, gb = sizes[k]
        for t in (0.03, 0.06):
            reqs.append(serve.Request(len(reqs), k, t, n, nnz, gb, serve.request_ws_bytes(n, nnz)))
    ex = serve.GpuExecutor(pool, 4, levels_hash=True)
    st = serve.Server(ex, slots=4, budget_bytes=budget, small=serve.small_request).run(reqs)
    torch.cuda.synchronize()
    assert st["failed"] == 0, st["errors"]
    assert st["batched"] > 0
    bad = []
    for r in reqs:
        g = rows[ids[r.graph_id]]
        if (r.triangles, r.h, r.levels_hash) != (g["triangles"], g["h"], g["levels_blake2b64"]):
            bad.append((r.rid, ids[r.graph_id], r.batched, r.triangles, g["triangles"]))
    assert not bad, bad[:5]
    assert len({r.graph_id for r in reqs}) > len(ids) // 2


def _largest(rows, kind):
    return max((r for r in rows if r["spec"]["kind"] == kind), key=lambda r: r["n"])["i"]
