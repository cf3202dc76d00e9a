"""Parity of tc_count_batch (many small graphs in one call) with the CPU
oracle: T, |H| and the level array of every graph, across tunings, in a
captured graph, and on the full 4096-graph workload against the stored
oracle results."""
import json
import os
from types import SimpleNamespace

import numpy as np
import pytest

import graphgen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.gpu


def _oracle(g):
    c = oracle.from_graph(g)
    lv = oracle.bfs_levels(c)
    hu, _ = oracle.cover_edges(c, lv.levels)
    return oracle.count(c, lv.levels, 0).triangles, int(hu.size), lv.levels


def _empty(n):
    z = np.zeros(0, dtype=np.int32)
    return SimpleNamespace(n=n, src=z, dst=z, name=f"empty{n}")


def _check(graphs, tuning=None, levels=True):
    import paper_2210_00389_amd as tc
    b = tc.Batch.from_graphs(graphs)
    r = tc.count_batch(b, tuning, return_levels=levels)
    T = r.triangles.cpu().numpy()
    H = r.h_count.cpu().numpy()
    L = r.levels.cpu().numpy() if levels else None
    vb = b.vbase.cpu().numpy()
    for i, g in enumerate(graphs):
        t_ref, h_ref, l_ref = _oracle(g)
        assert T[i] == t_ref, (i, getattr(g, "name", ""), T[i], t_ref)
        assert H[i] == h_ref, (i, getattr(g, "name", ""), H[i], h_ref)
        if levels:
            assert np.array_equal(L[vb[i]:vb[i + 1]], l_ref), (i, getattr(g, "name", ""))
    return b, r


def test_batch_small_mix():
    """64 graphs of the batch recipe (n up to 4096): every count, |H| and
    level array equals the oracle's."""
    print("case: batch_mix(64, n_max=4096)", flush=True)
    _check(graphgen.batch_mix(64, n_max=4096))


def test_batch_closed_forms_and_edge_cases():
    """Closed forms, several components, isolated vertices, a hub above the
    wave-expansion degree, a long path (many levels), an empty graph and a
    graph at the 65536-vertex limit."""
    graphs = [graphgen.complete(40), graphgen.wheel(100), graphgen.cycle(7), graphgen.cycle(8),
              graphgen.star(300), graphgen.path(3000), graphgen.grid(30, 30),
              graphgen.random_bipartite(50, 60, 0.2, 3),
              graphgen.disjoint_union([graphgen.complete(5), graphgen.path(10), _empty(7), graphgen.wheel(9),
                                       graphgen.cycle(5)]),
              _empty(5), _empty(0), graphgen.complete(3),
              graphgen.erdos_renyi(65536, 8.0 / 65535, 77), graphgen.barabasi_albert(20000, 16, 5)]
    print("case: closed forms / edge cases", flush=True)
    b, r = _check(graphs)
    T = r.triangles.cpu().numpy()
    assert T[0] == 40 * 39 * 38 // 6 and T[1] == 99 and T[2] == 0 and T[3] == 0
    assert T[4] == 0 and T[5] == 0 and T[6] == 0 and T[7] == 0 and T[9] == 0 and T[10] == 0 and T[11] == 1


@pytest.mark.parametrize("tuning", [dict(batch_block=256, batch_piece=1024), dict(batch_block=512, batch_piece=4096),
                                    dict(batch_block=256, batch_piece=65536, batch_blocks_per_cu=1)])
def test_batch_tunings_agree(tuning):
    print(f"case: tuning {tuning}", flush=True)
    _check(graphgen.batch_mix(48, seed_base=777, n_max=16384), tuning, levels=False)


def test_batch_invalid_tuning():
    import paper_2210_00389_amd as tc
    b = tc.Batch.from_graphs([graphgen.complete(10)])
    with pytest.raises(tc.TcError):
        tc.count_batch(b, dict(batch_block=128))
    with pytest.raises(tc.TcError):
        tc.count_batch(b, dict(batch_piece=100))


def test_batch_captured_replays():
    """The call recorded in a graph and replayed four times, with eager work
    and synchronisation between replays: every replay equals the eager run."""
    import torch
    import paper_2210_00389_amd as tc
    print("case: captured batch", flush=True)
    b = tc.Batch.from_graphs(graphgen.batch_mix(40, seed_base=99, n_max=8192))
    ref = tc.count_batch(b)
    T0, H0 = ref.triangles.cpu(), ref.h_count.cpu()
    cap = tc.CapturedBatch(b)
    for k in range(4):
        out = cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.triangles.cpu(), T0), k
        assert torch.equal(out.h_count.cpu(), H0), k
        tc.count_batch(b)  # eager work between replays
        torch.cuda.synchronize()


def test_batch_full_workload_golden():
    """The 4096-graph workload (ER half, BA half, n log-uniform in [64,
    65536]) in the launch configuration the benchmark times, against the
    oracle's stored per-graph T and |H|."""
    import paper_2210_00389_amd as tc
    path = os.path.join(HERE, "golden", "batch_mix.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/batch_mix.json not generated")
    gold = json.load(open(path))["graphs"]
    print("case: full batch 4096", flush=True)
    b = tc.Batch.from_graphs(graphgen.batch_mix(4096))
    r = tc.count_batch(b)
    T = r.triangles.cpu().numpy()
    H = r.h_count.cpu().numpy()
    assert len(gold) == 4096
    bad = [(g["i"], int(T[g["i"]]), g["triangles"]) for g in gold
           if T[g["i"]] != g["triangles"] or H[g["i"]] != g["h"]]
    assert not bad, bad[:5]
