"""The oracle's pins must catch plausible mistakes.

Each case copies oracle.c, plants one mistake (a dropped term, a wrong
operand, an off-by-one in a comparison, a skipped step), compiles the copy
with gcc on the CPU and runs a battery of the pins from test_oracle.py against
it.  The battery must fail for every mutant and pass for the real oracle.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "apex_order_uses_u": ("(L[u] == L[w] && v < w)", "(L[u] == L[w] && u < w)"),
    "apex_order_flipped": ("(L[u] == L[w] && v < w)", "(L[u] == L[w] && w < v)"),
    "drop_other_level_term": ("return (L[u] != L[w]) ||", "return 0 ||"),
    "drop_same_level_term": ("|| (L[u] == L[w] && v < w)", "|| 0"),
    "both_orientations": ("if (v > u && L[u] == L[v]) {", "if (v != u && L[u] == L[v]) {"),
    "count_skips_direction": ("if (!(v > u && L[u] == L[v])) continue;",
                              "if (!(L[u] == L[v])) continue;"),
    "bfs_no_increment": ("L[y] = L[x] + 1;", "L[y] = L[x];"),
    "root_ties_largest": ("if (d > bestd) { bestd = d; best = v; }",
                          "if (d >= bestd) { bestd = d; best = v; }"),
    "no_rescan": ("    if (L[v] < 0) {\n      int32_t d = bfs_from", "    if (L[v] < -1) {\n      int32_t d = bfs_from"),
    "no_dedup": ("if (out > row_begin && cols[out - 1] == cols[i]) continue;", ""),
    "merge_wrong_pointer": ("else if (cols[a] > cols[b]) ++b;\n          else {\n            int32_t w",
                            "else if (cols[a] > cols[b]) ++a;\n          else {\n            int32_t w"),
    "stamp_wrong_owner": ("if (stamp[w] == u && counts", "if (stamp[w] == v && counts"),
    "edge_iter_wrong_bound": ("if (cols[a] > v) ++total;", "if (cols[a] > u) ++total;"),
    "loops_kept": ("    if (s == d) continue;\n    deg[s] += 1;", "    deg[s] += 1;"),
    "sort3_last_swap_missing": ("  if (t[1] > t[2]) { x = t[1]; t[1] = t[2]; t[2] = x; }\n  if (t[0] > t[1]) { x = t[0]; t[0] = t[1]; t[1] = x; }\n}",
                                "  if (t[1] > t[2]) { x = t[1]; t[1] = t[2]; t[2] = x; }\n}"),
    "list_wrong_slot": ("    c->tri[3 * c->at + 2] = t[2];", "    c->tri[3 * c->at + 2] = t[1];"),
    "support_one_orientation": ("  c->support[find_in_row(c->off, c->cols, b, a)]++;\n", ""),
    "support_skips_an_edge": ("  add_edge(c, t[1], t[2]);\n", ""),
    "list_both_orientations": ("if (v <= u || L[u] != L[v]) continue;", "if (v == u || L[u] != L[v]) continue;"),
}


def battery():
    """Subset of the pins; returns the names of those that fail."""
    bad = []

    def check(name, fn):
        try:
            if not fn():
                bad.append(name)
        except Exception:
            bad.append(name)

    for mode in (0, 1):
        check(f"K7 mode{mode}", lambda: oracle.count(oracle.from_graph(graphgen.complete(7)),
                                                     oracle.bfs_levels(oracle.from_graph(graphgen.complete(7))).levels,
                                                     mode).triangles == math.comb(7, 3))
    check("W9", lambda: oracle.triangle_count(oracle.from_graph(graphgen.wheel(9))) == 8)
    check("C7 H", lambda: len(oracle.cover_edges(oracle.from_graph(graphgen.cycle(7)),
                                                 oracle.bfs_levels(oracle.from_graph(graphgen.cycle(7))).levels)[0]) == 1)
    check("K6 edge iterator", lambda: oracle.edge_count(oracle.from_graph(graphgen.complete(6))) == 20)
    check("path levels", lambda: oracle.bfs_levels(oracle.from_graph(graphgen.path(9))).levels.tolist()
          == [1, 0, 1, 2, 3, 4, 5, 6, 7])
    check("csr literal", lambda: oracle.build_csr(5, np.array([0, 1, 1, 2, 3, 2, 0, 3], np.int32),
                                                  np.array([1, 0, 1, 0, 3, 3, 2, 0], np.int32)).cols.tolist()
          == [1, 2, 3, 0, 0, 3, 0, 2])

    def brute_case(seed):
        g = graphgen.disjoint_union([graphgen.erdos_renyi(24, 0.3, seed), graphgen.complete(4),
                                     graphgen.cycle(5)])
        c = oracle.from_graph(g)
        adj = brute.adjacency(g.n, g.src, g.dst)
        tris = brute.triangles(adj)
        L = oracle.bfs_levels(c).levels
        hops = brute.all_pairs_hops(adj)
        r0 = oracle.default_root(c)
        ok = all((L[v] == hops[r0, v]) for v in range(g.n) if hops[r0, v] >= 0)
        # other components: distance from their smallest id
        for v in range(g.n):
            if hops[r0, v] < 0:
                root = min(w for w in range(g.n) if hops[v, w] >= 0)
                ok &= L[v] == hops[root, v]
        for mode in (0, 1):
            r = oracle.count(c, L, mode, per_vertex=True)
            ok &= r.triangles == len(tris)
            ok &= (r.per_vertex == brute.per_vertex(g.n, tris)).all()
        ok &= oracle.edge_count(c) == len(tris)
        return bool(ok)

    for seed in (1, 2):
        check(f"brute {seed}", lambda: brute_case(seed))

    def listing_case(seed):
        g = graphgen.disjoint_union([graphgen.erdos_renyi(30, 0.3, seed), graphgen.wheel(7)])
        c = oracle.from_graph(g)
        L = oracle.bfs_levels(c).levels
        got = sorted(map(tuple, oracle.list_triangles(c, L).tolist()))
        ok = got == brute.triangles(brute.adjacency(g.n, g.src, g.dst))
        sup = oracle.edge_supports(c, L)
        for u in range(c.n):
            for e in range(c.row_offsets[u], c.row_offsets[u + 1]):
                v = c.cols[e]
                ok &= sup[e] == np.intersect1d(c.cols[c.row_offsets[u]:c.row_offsets[u + 1]],
                                               c.cols[c.row_offsets[v]:c.row_offsets[v + 1]]).size
        return bool(ok)

    for seed in (3, 4):
        check(f"listing {seed}", lambda: listing_case(seed))
    return bad


@pytest.fixture(scope="module")
def real_battery():
    oracle._use_library(None)
    return battery()


def test_real_oracle_passes_battery(real_battery):
    assert real_battery == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/present"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(path)])
    try:
        oracle._use_library(str(so))
        bad = battery()
    finally:
        oracle._use_library(None)
    assert bad, f"mutant {name} passed every pin"
