"""Write the stored expected values for the R-MAT configurations.

Every value here comes from the CPU oracle (``oracle/``) run on graphs from
the seeded input generator (``graphgen``); nothing is taken from the GPU
library.  Usage::

    python tests/golden/make_golden.py 10 20        # scales to (re)write
    python tests/golden/make_golden.py --batch       # per-graph batch counts
    python tests/golden/make_golden.py --serving     # the serving request pool

Output: ``tests/golden/rmat_s<scale>.json`` with n, m, |H|, T (Alg. 1 count,
direct-address mode), the edge-iterator count, level statistics and SHA-256
digests of the level array and of the horizontal-edge list, plus
``batch_mix.json`` with every graph's (n, m, |H|, T), and
``serving_pool.json`` with every pool graph's (n, m, |H|, T), the SHA-256 of
its horizontal-edge list and the 64-bit BLAKE2b digest of its levels (the
digest a served request carries: little-endian int32 levels in vertex
order).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen  # noqa: E402
import oracle  # noqa: E402


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def rmat_golden(scale: int, with_edge_count: bool = True) -> dict:
    t0 = time.time()
    g = graphgen.rmat(scale, 16, seed=1)
    c = oracle.from_graph(g)
    t1 = time.time()
    lv = oracle.bfs_levels(c)
    hu, hv = oracle.cover_edges(c, lv.levels)
    t2 = time.time()
    res = oracle.count(c, lv.levels, 0)
    t3 = time.time()
    out = dict(
        config=f"R-MAT scale {scale}, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), seed 1, "
               "relabelled; root = largest degree (smallest id on ties)",
        source="CPU oracle (oracle/oracle.c) on graphgen.rmat(scale, 16, seed=1)",
        scale=scale, n=c.n, m=c.m, nnz=c.nnz, max_degree=int(c.degrees().max()),
        root=oracle.default_root(c), num_levels=lv.num_levels, num_roots=lv.num_roots,
        h=int(hu.size), triangles=res.triangles,
        levels_sha256=digest(lv.levels.astype("<i4")),
        h_sha256=digest(hu.astype("<i4"), hv.astype("<i4")),
        csr_sha256=digest(c.row_offsets.astype("<i8"), c.cols.astype("<i4")),
        oracle_seconds=dict(build=t1 - t0, bfs_and_h=t2 - t1, count=t3 - t2),
    )
    if with_edge_count:
        t4 = time.time()
        out["edge_iterator_triangles"] = oracle.edge_count(c)
        out["oracle_seconds"]["edge_iterator"] = time.time() - t4
    return out


def _batch_row(item):
    i, s = item
    c = oracle.from_graph(graphgen.from_spec(s))
    lv = oracle.bfs_levels(c)
    hu, _ = oracle.cover_edges(c, lv.levels)
    T = oracle.count(c, lv.levels, 0).triangles
    return dict(i=i, n=c.n, m=c.m, h=int(hu.size), triangles=T,
                levels_sha256=digest(lv.levels.astype("<i4")))


def batch_golden(workers: int = 6) -> dict:
    """Per-graph oracle results of graphgen.batch_specs(4096), computed by
    `workers` processes (each graph is independent)."""
    from multiprocessing import Pool
    specs = graphgen.batch_specs(4096)
    t0 = time.time()
    with Pool(workers) as pool:
        rows = []
        for r in pool.imap(_batch_row, list(enumerate(specs)), chunksize=8):
            rows.append(r)
            if r["i"] % 256 == 0:
                print(f"batch {r['i']}/4096 {time.time() - t0:.1f}s", flush=True)
    return dict(source="CPU oracle on graphgen.batch_specs(4096)", graphs=rows,
                oracle_seconds=time.time() - t0)


def _serving_row(item):
    i, s = item
    t0 = time.time()
    c = oracle.from_graph(graphgen.from_spec(s))
    lv = oracle.bfs_levels(c)
    hu, hv = oracle.cover_edges(c, lv.levels)
    T = oracle.count(c, lv.levels, 0).triangles
    lv32 = np.ascontiguousarray(lv.levels.astype("<i4"))
    return dict(i=i, spec=s, n=c.n, m=c.m, h=int(hu.size), triangles=T, num_levels=lv.num_levels,
                levels_blake2b64=hashlib.blake2b(lv32.tobytes(), digest_size=8).hexdigest(),
                h_sha256=digest(hu.astype("<i4"), hv.astype("<i4")), oracle_seconds=time.time() - t0)


def serving_golden(workers: int = 6) -> dict:
    """Oracle results for every graph of graphgen.serving_specs(128), the
    largest first so the slowest counts start early."""
    from multiprocessing import Pool
    specs = graphgen.serving_specs(128)

    def cost(s):
        return 2.0 ** s["scale"] * 16 if s["kind"] == "rmat" else s["n"] * 10.0
    order = sorted(range(len(specs)), key=lambda i: -cost(specs[i]))
    t0 = time.time()
    rows = []
    with Pool(workers) as pool:
        for r in pool.imap_unordered(_serving_row, [(i, specs[i]) for i in order]):
            rows.append(r)
            print(f"serving graph {r['i']} ({len(rows)}/{len(specs)}) {r['oracle_seconds']:.1f}s "
                  f"T={r['triangles']}", flush=True)
    rows.sort(key=lambda r: r["i"])
    return dict(source="CPU oracle on graphgen.serving_specs(128)", graphs=rows,
                oracle_seconds=time.time() - t0)


def main(argv):
    if "--batch" in argv:
        out = batch_golden()
        with open(os.path.join(HERE, "batch_mix.json"), "w") as f:
            json.dump(out, f, indent=1)
        argv = [a for a in argv if a != "--batch"]
    if "--serving" in argv:
        out = serving_golden()
        with open(os.path.join(HERE, "serving_pool.json"), "w") as f:
            json.dump(out, f, indent=1)
        argv = [a for a in argv if a != "--serving"]
    for a in argv:
        scale = int(a)
        out = rmat_golden(scale, with_edge_count=scale <= 22)
        with open(os.path.join(HERE, f"rmat_s{scale}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
