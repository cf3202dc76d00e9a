"""Parity at the full sizes of the R-MAT workloads (scales 20, 22, 24) in the
launch configuration the benchmark times, against values the CPU oracle
stored in tests/golden/ (written by tests/golden/make_golden.py): T, |H|,
the level array and the horizontal-edge list (SHA-256), the comparator's
count, and sampled per-vertex counts that are recomputed one by one on the
CPU."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gold(scale):
    p = os.path.join(GOLDEN, f"rmat_s{scale}.json")
    if not os.path.exists(p):
        pytest.skip(f"tests/golden/rmat_s{scale}.json not generated")
    return json.load(open(p))


def _vertex_triangles(off, cols, x):
    """Triangles through x: edges among N(x), by sorted-list intersections."""
    nx = cols[off[x]:off[x + 1]]
    t = 0
    for y in nx:
        ny = cols[off[y]:off[y + 1]]
        t += np.intersect1d(nx, ny, assume_unique=True).size
    return t // 2


@pytest.mark.parametrize("scale", [20, 22, 24])
def test_rmat_full_size(scale):
    import torch
    import paper_2210_00389_amd as tc
    gold = _gold(scale)
    print(f"case: rmat{scale} full size", flush=True)
    g = graphgen.rmat(scale, 16, seed=1)
    G = tc.from_host_pairs(g.n, g.src, g.dst)
    del g
    assert (G.n, G.m) == (gold["n"], gold["m"])
    res = tc.count(G, return_levels=True, per_vertex=(scale == 20))
    assert res.T == gold["triangles"]
    assert res.h == gold["h"]
    if "levels_sha256" in gold:
        digest = hashlib.sha256(res.levels.cpu().numpy().astype("<i4").tobytes()).hexdigest()
        assert digest == gold["levels_sha256"]
    if "h_sha256" in gold:
        # the explicit cover-edge list of these levels (tc_cover_edges),
        # lexicographic, against the oracle's list: SHA-256 of h_u then h_v
        hu, hv = tc.cover_edges(G, res.levels)
        assert hu.numel() == gold["h"]
        hsh = hashlib.sha256()
        hsh.update(hu.cpu().numpy().astype("<i4").tobytes())
        hsh.update(hv.cpu().numpy().astype("<i4").tobytes())
        assert hsh.hexdigest() == gold["h_sha256"]
        del hu, hv
    if "edge_iterator_triangles" in gold:
        assert int(tc.count_edge_baseline(G).item()) == gold["edge_iterator_triangles"]
    if scale == 20:
        pv = res.per_vertex.cpu().numpy()
        assert int(pv.sum()) == 3 * gold["triangles"]
        off = G.row_offsets.cpu().numpy()
        cols = G.cols.cpu().numpy()
        deg = np.diff(off)
        rng = np.random.default_rng(20)
        cand = np.nonzero((deg > 0) & (deg <= 300))[0]
        sample = rng.choice(cand, size=150, replace=False)
        for x in sample:
            assert pv[x] == _vertex_triangles(off, cols, x), int(x)
    torch.cuda.synchronize()
