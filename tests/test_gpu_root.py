"""Root choice by the size of the cover-edge set (tc_select_root) against
the oracle: the same candidates (largest degree first, smallest id on
ties), the same |H| for each candidate root (oracle BFS of Alg. 1 from that
root, then the horizontal edges), the same winner, and the count with the
chosen root equal to the oracle's T (Thm. 2: T does not depend on the root).
"""
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


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


def _oracle_choice(c, k):
    deg = np.diff(c.row_offsets)
    order = np.lexsort((np.arange(c.n), -deg))[:k]
    hs = [len(oracle.cover_edges(c, oracle.bfs_levels(c, int(r)).levels)[0]) for r in order.tolist()]
    return order.tolist(), hs, int(order[int(np.argmin(hs))])


GRAPHS = [
    ("ba3000", lambda: graphgen.barabasi_albert(3000, 6, 41)),
    ("rmat12", lambda: graphgen.rmat(12, 16, seed=42)),
    ("chunglu", lambda: graphgen.chung_lu(10000, seed=43)),
    ("union", lambda: graphgen.disjoint_union([graphgen.erdos_renyi(500, 0.02, 44), graphgen.wheel(30),
                                               graphgen.complete(12), graphgen.path(40)])),
    ("K5", lambda: graphgen.complete(5)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_select_root_matches_oracle(tc, name, make):
    g = make()
    say(f"[root] {name} n={g.n}")
    c = oracle.from_graph(g)
    G = tc.from_host_pairs(g.n, g.src, g.dst, device="cuda")
    k = 8
    cand, hs, best = _oracle_choice(c, k)
    got = tc.select_root(G, k)
    assert got.candidates == cand
    assert got.h == hs
    assert got.root == best
    T = oracle.count(c, oracle.bfs_levels(c).levels).triangles
    assert tc.count(G, root=got.root).T == T
    assert tc.count(G, root=got.root).h == min(hs)


def test_select_root_limits(tc):
    g = graphgen.complete(6)
    G = tc.from_host_pairs(g.n, g.src, g.dst, device="cuda")
    with pytest.raises(tc.TcError):
        tc.select_root(G, 0)
    with pytest.raises(tc.TcError):
        tc.select_root(G, 65)
    assert tc.select_root(G, 64).candidates == list(range(6))
    E = tc.from_host_pairs(0, np.zeros(0, np.int32), np.zeros(0, np.int32), device="cuda")
    assert tc.select_root(E, 4).root == -1
