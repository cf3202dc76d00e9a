"""Input generators: determinism and distribution checks (no GPU)."""
import math

import numpy as np

import graphgen
import oracle


def test_rmat_deterministic_and_seeded():
    a = graphgen.rmat(12, 16, seed=1)
    b = graphgen.rmat(12, 16, seed=1)
    c = graphgen.rmat(12, 16, seed=2)
    assert (a.src == b.src).all() and (a.dst == b.dst).all()
    assert not (a.src == c.src).all()
    assert a.num_pairs == 16 * 4096
    assert a.src.min() >= 0 and a.src.max() < 4096


def test_rmat_quadrant_frequencies():
    # before relabelling, the top bit of (row, col) picks the quadrant with
    # probabilities a, b, c, d
    g = graphgen.rmat(14, 16, seed=7, permute=False)
    top_r = g.src >> 13
    top_c = g.dst >> 13
    q = 2 * top_r + top_c
    freq = np.bincount(q, minlength=4) / q.size
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_permutation_is_bijection():
    p = graphgen.permutation(1000, 3)
    assert sorted(p.tolist()) == list(range(1000))
    assert not (p == np.arange(1000)).all()


def test_er_mean_degree():
    n, p = 4000, 0.005
    g = graphgen.erdos_renyi(n, p, 11)
    c = oracle.from_graph(g)
    assert g.num_pairs == c.m  # geometric skipping never repeats a pair
    exp = p * n * (n - 1) / 2
    assert abs(c.m - exp) < 5 * math.sqrt(exp)
    assert (g.src > g.dst).all()


def test_er_complete_when_p_is_one():
    g = graphgen.erdos_renyi(20, 1.0, 1)
    assert oracle.from_graph(g).m == 190


def test_ba_edges_and_connectivity():
    g = graphgen.barabasi_albert(3000, 4, 5)
    c = oracle.from_graph(g)
    assert 0.9 * 4 * 3000 < c.m <= 4 * 3000
    lv = oracle.bfs_levels(c)
    assert lv.num_roots == 1  # preferential attachment builds one component


def test_chung_lu_expected_degrees():
    n, d = 20000, 20.0
    w = graphgen.chung_lu_weights(n, 2.1, d)
    assert abs(w.mean() - d) < 1e-6 * d
    assert abs(w[0] - math.sqrt(n * d)) < 1e-3 * w[0]
    assert (np.diff(w) <= 0).all()
    g = graphgen.chung_lu(n, 2.1, d, 3, permute=False)
    c = oracle.from_graph(g)
    assert abs(2 * c.m / n - d) < 0.1 * d
    deg = c.degrees()
    # the heaviest vertices get degrees near their weights
    assert abs(deg[:50].mean() - w[:50].mean()) < 0.2 * w[:50].mean()


def test_batch_specs_recipe():
    specs = graphgen.batch_specs(4096)
    assert len(specs) == 4096
    er = [s for s in specs if s["kind"] == "er"]
    ba = [s for s in specs if s["kind"] == "ba"]
    assert len(er) == len(ba) == 2048
    ns = np.array([s["n"] for s in specs])
    assert ns.min() >= 64 and ns.max() <= 65536
    # log-uniform: the median sits near the geometric mean of the bounds
    assert abs(math.log(np.median(ns)) - math.log(math.sqrt(64 * 65536))) < 0.2
    assert all(8 <= s["mean_degree"] <= 64 for s in er)
    assert {s["m"] for s in ba} == set(range(2, 17))


def test_serving_specs_mix():
    specs = graphgen.serving_specs(64)
    kinds = [s["kind"] for s in specs]
    assert kinds.count("rmat") == kinds.count("chung_lu") == 32
    assert all(12 <= s["scale"] <= 22 for s in specs if s["kind"] == "rmat")
    assert all(10**4 <= s["n"] <= 10**6 for s in specs if s["kind"] == "chung_lu")
