#!/usr/bin/env python
"""Benchmark: exact cover-edge triangle counting on one MI355X.

Workload (default): R-MAT scale 20, edge factor 16, quadrant probabilities
(0.57, 0.19, 0.19, 0.05), seed 1, vertex ids relabelled, symmetrised and
deduplicated; CSR int64 offsets / int32 sorted columns resident in HBM.

One step = tc_count on the resident CSR: BFS levels from the largest-degree
vertex (plus the remaining components), level-class layout and cover-edge
list, intersections, reduction -- CSR in HBM to T in HBM.  The comparator
(plain direction-oriented edge iterator on the same kernels) is timed the same
way.  Prints one JSON line.

Roofline: the dominant stage's algorithmic bytes per launch (exact element
counts reported by the library) divided by its average duration, taken from
HIP events the library records around each stage on the call's stream during
the timed steps.

traffic: counter-measured bytes of the dominant stage from the committed
summary under profiles/ when it was taken on the current kernel source.

stream_bw: what a plain 1 GiB device copy and a float32 sum reach on the same
device, as the practical ceiling beside the 8 TB/s peak.

cpu_baseline: the CPU oracle, single-threaded, on a bounded sample (full BFS
and cover edges, then the count over a prefix of the rows -- a uniform sample
because ids are relabelled -- scaled to all rows); alg1_work holds the
oracle's work measures of Alg. 1 on the same graph.

Other workloads: --workload batch (4096 graphs per captured launch), serving
(Poisson request streams, p50/p99), list (triangle finding and supports), pmc
(the program profiled for counters).  --summarize / --summarize-kernels turn
rocprofv3 output into the summaries kept under profiles/.
"""
import argparse
import json
import math
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def stage_bytes(name, st, n, nnz, cover):
    """Algorithmic HBM bytes of one stage (what the method must move)."""
    if name == "bfs":
        # offsets + every row once + visited-bit gathers + levels + queues
        return 8 * (n + 1) + 4 * nnz + nnz / 8 + 4 * n + 8 * n
    if name == "relabel":
        # offsets + rows + new-id gathers + re-laid-out rows + offsets + vertex records
        return 8 * (n + 1) + 4 * nnz + 4 * nnz + 4 * nnz + 8 * (n + 1) + 32 * n
    if name == "forward_lists":
        return 8 * (n + 1) + 4 * nnz + 4 * nnz + 32 * n
    if name == "plan":
        # vertex records + descriptor counts + plan bytes + scan + the 16-byte
        # records the resolution reads of neighbours
        return 32 * n + 4 * n + n + 12 * n + 16 * n
    if name == "resolve":
        # per descriptor: its column entry + the other endpoint's 16-byte
        # record; light merges; records written; items written, read and regrouped
        d = st.get("descriptors", 0)
        return 20 * d + 4 * st["light_elems"] + 16 * st["heavy_desc"] + 48 * st["heavy_items"]
    if name == "heavy":
        # streamed list elements + records + probe-set inserts + items
        return 4 * st["heavy_elems"] + 16 * st["heavy_desc"] + 4 * st["heavy_builds"] + 16 * st["heavy_items"]
    return None


def run_timed(fn, steps, sync):
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    stage_ms = {}
    sync()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record()
        fn()
        ev[i][1].record()
        for name, ms in read_profile():
            stage_ms.setdefault(name, []).append(ms)
    sync()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    return wall, per, stage_ms


def read_profile():
    import paper_2210_00389_amd as tc
    return tc.profile_read()


def stream_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """What plain streaming reaches on this device: a device-to-device copy
    (reads and writes nbytes each) and a read-only float32 sum over nbytes,
    median of reps launches timed with events on the current stream.  The
    buffers are 4x the 256 MB last-level cache, so both stream from HBM."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b) / 1000.0)
        return statistics.median(ts)
    t_copy = timed(lambda: y.copy_(x))
    t_read = timed(lambda: x.sum())
    del x, y
    return {"bytes": nbytes, "copy_GBps": round(2 * nbytes / t_copy / 1e9, 1),
            "read_GBps": round(nbytes / t_read / 1e9, 1)}


def _cpu_model():
    try:
        return [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        return platform.processor()


def row_work(c, levels):
    """List elements the oracle's count touches per row u (its
    direct-address mode): N(u) is stamped once if u has a cover edge (u, v),
    v > u, and N(v) is scanned for each such edge.  A cost model for the
    sampled CPU estimate, from degrees and levels only."""
    import numpy as np
    deg = np.diff(c.row_offsets)
    rows = np.repeat(np.arange(c.n, dtype=np.int64), deg)
    cols = c.cols.astype(np.int64)
    lv = np.asarray(levels)
    hz = (rows < cols) & (lv[rows] == lv[cols])
    u, v = rows[hz], cols[hz]
    del rows, cols, hz
    w = np.bincount(u, weights=deg[v].astype(np.float64), minlength=c.n)
    w += np.where(np.bincount(u, minlength=c.n) > 0, deg, 0)
    return w


def _strided_estimate(oracle, c, levels, phase, stride, work):
    """Time the oracle count over the rows phase, phase + stride, ... and
    scale it to all rows by the elements those rows touch (a ratio
    estimate: time per element of the sample times all elements).  Times
    are the process's CPU time: the oracle is single-threaded, and the legs
    run beside the GPU benchmark, whose host work would otherwise be
    counted as the oracle's."""
    t = time.process_time()
    oracle.count_rows_strided(c, levels, phase, stride)
    dt = time.process_time() - t
    rows = len(range(phase, c.n, stride))
    w_s = float(work[phase::stride].sum())
    return dt, rows, dt * float(work.sum()) / max(w_s, 1.0)


def cpu_leg(args):
    """The CPU oracle on the benchmark graph, single-threaded, on a bounded
    sample: full BFS and cover edges, then the count over `parts` systematic
    row samples (rows phase, phase + stride, ... for different phases: ids
    are relabelled uniformly at random, so every phase is a uniform sample
    spread over the whole id range), each scaled to all rows.  Prints one
    JSON line (run as a child process of the benchmark)."""
    import numpy as np
    import graphgen
    import oracle
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    c = oracle.from_graph(g)
    del g
    log(f"[cpu] oracle CSR of R-MAT scale {args.scale} built")
    t = time.process_time()  # CPU time of this single-threaded process (see _strided_estimate)
    lv = oracle.bfs_levels(c)
    t_bfs = time.process_time() - t
    t = time.process_time()
    hu, _ = oracle.cover_edges(c, lv.levels)
    t_h = time.process_time() - t
    del hu
    work_rows = row_work(c, lv.levels)
    # pilot: about 1/1024 of the rows, to size the sample to the budget
    pilot_stride = max(1, c.n // 1024)
    dt, rows, _ = _strided_estimate(oracle, c, lv.levels, 0, pilot_stride, work_rows)
    per_row = dt / max(rows, 1)
    parts = 4
    stride = max(1, int(math.ceil(c.n * per_row * parts / max(args.cpu_budget, 1e-3))))
    ests, t_count, sampled = [], 0.0, 0
    if stride <= parts:
        # the budget covers the whole count: time it exactly
        t = time.process_time()
        oracle.count(c, lv.levels, 0)
        t_count = time.process_time() - t
        ests = [t_count]
        sampled = c.n
        stride = 1
    else:
        for k in range(parts):
            phase = (k * stride) // parts + stride // (2 * parts)
            dt, rows, est = _strided_estimate(oracle, c, lv.levels, phase, stride, work_rows)
            ests.append(est)
            t_count += dt
            sampled += rows
            log(f"[cpu] sample {k + 1}/{parts}: {rows} rows in {dt:.1f}s -> full count {est:.0f}s")
    est_count = float(np.mean(ests))
    est = t_bfs + t_h + est_count
    work = oracle.work_counters(c, lv.levels)
    m = c.m
    spread = (max(ests) - min(ests)) / est_count if len(ests) > 1 else 0.0
    out = {
        "value": m / est, "unit": "edges/s", "cores": 1, "kind": "oracle",
        "sample": (f"single-threaded CPU oracle (oracle/oracle.c, gcc -O2) on this host (1 of {os.cpu_count()} "
                   f"cores, {_cpu_model()}; process CPU time) on R-MAT scale {args.scale}: full BFS {t_bfs:.2f}s + cover edges "
                   f"{t_h:.2f}s, then the count over {len(ests)} systematic row samples (every {stride}th row, "
                   f"{sampled} rows = {100.0 * sampled / max(c.n, 1):.3f}% in {t_count:.1f}s), each scaled to "
                   f"all rows by the list elements the rows touch; estimated full run {est:.0f}s"),
        "estimated_full_seconds": est,
        "count_estimates_s": ests,
        "estimate_spread": spread,
        "stride": stride,
        "alg1_work": work,
    }
    print(json.dumps(out), flush=True)


def cpu_validate(args):
    """How good the sampled estimate is: on R-MAT scale `args.scale` the
    full oracle count is timed, then systematic row samples at two strides
    (8 phases each) are scaled to all rows as the CPU baseline does;
    prints the relative errors as one JSON line."""
    import graphgen
    import oracle
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    c = oracle.from_graph(g)
    del g
    lv = oracle.bfs_levels(c)
    work_rows = row_work(c, lv.levels)
    t = time.process_time()  # CPU time, as the estimates (see _strided_estimate)
    oracle.count(c, lv.levels, 0)
    t_full = time.process_time() - t
    log(f"[cpu-check] full oracle count at scale {args.scale}: {t_full:.1f}s")
    res = {"scale": args.scale, "full_count_s": t_full, "strides": {}}
    for stride in (32, 512):
        errs = []
        for k in range(8):
            _, _, est = _strided_estimate(oracle, c, lv.levels, (k * stride) // 8, stride, work_rows)
            errs.append((est - t_full) / t_full)
        res["strides"][str(stride)] = {"rel_errors": [round(e, 4) for e in errs],
                                       "max_abs_rel_error": round(max(abs(e) for e in errs), 4)}
    print(json.dumps(res), flush=True)


def bench_list(args):
    """Triangle finding on R-MAT: tc_list_triangles into an exact-size buffer
    (count pass recording per-unit counts, offsets, write pass), then the
    per-edge supports from the list (tc_edge_support)."""
    import torch
    import graphgen
    import paper_2210_00389_amd as tc
    dev = torch.device("cuda:0")
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    G = tc.from_host_pairs(g.n, g.src, g.dst, device=dev)
    del g
    ws = tc.Workspace(dev)
    T = tc.count(G, ws=ws).T
    res = tc.list_triangles(G, cap=T, ws=ws)
    tc.profile_enable(True)
    for _ in range(args.warmup):
        tc.list_triangles(G, cap=T, ws=ws, out=res)
    torch.cuda.synchronize()
    log(f"[bench] listing {T} triangles, {args.steps} steps")
    wall, per, stages = run_timed(lambda: tc.list_triangles(G, cap=T, ws=ws, out=res), args.steps,
                                  torch.cuda.synchronize)
    tc.profile_enable(False)
    assert res.T == T
    sup_ms = []
    for _ in range(max(3, args.steps // 4)):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        sup = tc.edge_support(G, res.tri)
        s1.record()
        torch.cuda.synchronize()
        sup_ms.append(s0.elapsed_time(s1))
    assert int(sup.to(torch.int64).sum().item()) == 6 * T
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"rmat_s{args.scale}.json")
    if args.edge_factor == 16 and args.seed == 1 and os.path.exists(gpath):
        golden = {"triangles": json.load(open(gpath))["triangles"]}
        golden["match"] = golden["triangles"] == T
    ms = 1000 * wall / args.steps
    return {
        "metric": "triangles listed/s", "value": T / (wall / args.steps), "unit": "triangles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale}, edge factor {args.edge_factor}, seed {args.seed}: "
                               "triangle finding into an exact-size buffer (12 bytes per triangle), then "
                               "per-edge supports", "n": G.n, "m": G.m, "triangles": T},
        "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99),
        "stages": {k: round(statistics.mean(v), 4) for k, v in stages.items()},
        "output_GB_per_s": 12 * T / (wall / args.steps) / 1e9,
        "support_ms": statistics.median(sup_ms),
        "golden": golden,
    }


def bench_batch(args):
    """4096 ER/BA graphs in one captured tc_count_batch replay per step."""
    import numpy as np
    import torch
    import graphgen
    import paper_2210_00389_amd as tc
    log("[bench] generating the 4096-graph batch")
    graphs = graphgen.batch_mix(4096)
    b = tc.Batch.from_graphs(graphs)
    del graphs
    torch.cuda.synchronize()
    log(f"[bench] batch: G={b.num_graphs} sum n={b.total_vertices} sum m={b.total_edges}")
    tuning = tc.autotune(b, verbose=True, use_cache=False)
    cap = tc.CapturedBatch(b, tuning)
    for _ in range(args.warmup):
        cap.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, z in ev:
        a.record()
        cap.replay()
        z.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(z) for a, z in ev]
    T = cap.out.triangles.cpu().numpy()
    H = cap.out.h_count.cpu().numpy()
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch_mix.json")
    if os.path.exists(gpath):
        gd = json.load(open(gpath))["graphs"]
        golden = {"graphs": len(gd), "all_match": all(T[g["i"]] == g["triangles"] and H[g["i"]] == g["h"]
                                                       for g in gd)}
    ms = 1000 * wall / args.steps
    return {
        "metric": "cover-edge TC edges/s (batched, 4096 graphs per launch)", "value": b.total_edges / (wall / args.steps),
        "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "4096 graphs: 2048 Erdos-Renyi (mean degree U[8,64]) + 2048 Barabasi-Albert "
                               "(m U{2..16}), n log-uniform in [64, 65536], seed base 4096; one captured "
                               "tc_count_batch per step", "num_graphs": b.num_graphs,
                   "sum_n": b.total_vertices, "sum_m": b.total_edges, "tuning": tuning},
        "triangles_per_s": float(T.sum()) / (wall / args.steps),
        "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99), "golden": golden,
    }


def bench_serving(args):
    """Poisson request stream over a pool of R-MAT and Chung-Lu graphs."""
    import numpy as np
    import torch
    import graphgen
    from paper_2210_00389_amd import serve
    specs = graphgen.serving_specs(args.pool, scale_max=args.serve_scale_max,
                                   cl_n_max=args.serve_cl_n_max)
    log(f"[bench] building the serving pool ({len(specs)} graphs)")
    graphs = []
    for i, sp in enumerate(specs):
        graphs.append(graphgen.from_spec(sp))
        log(f"[bench] pool: graph {i + 1}/{len(specs)} {sp['kind']} generated")
    pool, sizes = serve.build_pool(graphs)
    del graphs
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * args.serve_budget_frac)
    runs = []
    # one executor for every rate: its streams, per-slot workspaces and
    # resident graphs persist like a long-running server's (fresh streams per
    # rate would strand each rate's workspaces in the caching allocator,
    # which reuses a freed block only on the stream that allocated it)
    ex = serve.GpuExecutor(pool, args.slots)
    # every pool graph counted alone (median of 3 device times, the path
    # tc_count picks): the offered load of a rate is rate x the mean of these
    # over its requests, in GPU-seconds per second
    import paper_2210_00389_amd as tc
    alone_ms = {}
    wsa = tc.Workspace(torch.device("cuda"))
    for gid, (off, cols) in pool.items():
        G = tc.Graph(sizes[gid][0], off.to("cuda"), cols.to("cuda"))
        ts = []
        for _ in range(4):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            tc.count(G, ws=wsa)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        alone_ms[gid] = statistics.median(ts[1:])
        del G
    del wsa
    torch.cuda.empty_cache()
    log(f"[bench] pool counted alone: {sum(alone_ms.values()):.1f} ms in all")
    # the oracle's stored answers for the default pool (tests/golden/serving_pool.json)
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "serving_pool.json")
    if os.path.exists(gpath):
        rows = json.load(open(gpath))["graphs"]
        if len(rows) == len(specs) and all(r["spec"] == sp for r, sp in zip(rows, specs)):
            gold = {r["i"]: (r["triangles"], r["h"]) for r in rows}
    batching = not args.no_batching
    small = serve.small_request if batching else None
    ws_fn = lambda n, nnz: serve.request_ws_bytes(n, nnz, batching)  # noqa: E731
    checked, mismatched = 0, 0
    for rate in args.rates:
        reqs = serve.make_requests(sizes, ws_fn, rate=rate, count=args.requests, seed=int(rate))
        st = serve.Server(ex, slots=args.slots, budget_bytes=budget, small=small,
                          batch_max=args.batch_max).run(reqs)
        torch.cuda.synchronize()
        st["rate_req_s"] = rate
        st["offered_load"] = rate * float(np.mean([alone_ms[r.graph_id] for r in reqs])) / 1000.0
        if gold is not None:
            bad = [r.rid for r in reqs if (r.triangles, r.h) != gold[r.graph_id]]
            checked += len(reqs)
            mismatched += len(bad)
            st["golden_mismatches"] = len(bad)
        log(f"[bench] rate {rate}: offered load {st['offered_load']:.2f} p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
            f"edges/s {st['edges_per_s']:.3e} busy {st['busy_fraction']:.2f} batched {st['batched']} "
            f"jobs {st['jobs']} failed {st['failed']}")
        runs.append(st)
    top = runs[-1]
    return {
        "metric": "served cover-edge TC latency p50/p99 and edges/s", "value": top["edges_per_s"],
        "unit": "edges/s", "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": top["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals over a pool of {len(specs)} graphs (half R-MAT scale "
                               f"12-{args.serve_scale_max} ef16, half Chung-Lu gamma 2.1 mean degree 20 n "
                               f"1e4-{args.serve_cl_n_max:.0e}); {args.slots} slots; HBM budget "
                               f"{args.serve_budget_frac:.2f} of free; "
                               + (f"small graphs (n <= {serve.SMALL_N}, nnz <= {serve.SMALL_NNZ}) coalesced "
                                  f"into tc_count_batch launches of up to {args.batch_max}" if batching
                                  else "no batching"),
                   "rates": args.rates, "requests_per_rate": args.requests},
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "runs": runs,
        "golden": ({"requests_checked": checked, "mismatches": mismatched, "all_match": mismatched == 0
                    and all(r["failed"] == 0 for r in runs)} if gold is not None else None),
        "pool_alone_ms": {"sum": sum(alone_ms.values()), "mean_per_graph": float(np.mean(list(alone_ms.values()))),
                          "max": max(alone_ms.values())},
        "uploads": ex.uploads,
    }


HEAVY_SRCS = [os.path.join(ROOT, "paper_2210_00389_amd", "csrc", f) for f in ("count.hip", "tc_common.h",
                                                                              "tc_internal.h")]


def source_sha(paths=None):
    """SHA-256 over the sources the heavy kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for p in paths or HEAVY_SRCS:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def traffic_record(scale):
    """Counter-measured DRAM bytes per heavy-stage launch, from the committed
    summary of rocprofv3 --pmc runs (see summarize_counters); None when
    missing or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"counters_rmat{scale}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    heavy = rec.get("heavy")
    if not heavy or heavy.get("source_sha256") != source_sha():
        return None
    return {"traffic_bytes": heavy.get("traffic_bytes"), "summary": f"profiles/counters_rmat{scale}.md"}


def bench_pmc(args):
    """Program run under rocprofv3 --pmc: a few counts of the R-MAT graph,
    then one plain 1 GiB device copy for the counter calibration."""
    import torch
    import graphgen
    import paper_2210_00389_amd as tc
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    G = tc.from_host_pairs(g.n, g.src, g.dst)
    ws = tc.Workspace(torch.device("cuda"))
    for i in range(args.warmup + args.steps):
        if args.pmc_comparator:
            # the comparator with its table bins one after another, so that a
            # trace gives every bin's own duration
            T = int(tc.count_edge_baseline(G, ws=ws, tuning={"bins_mode": 1}).item())
        else:
            T = tc.count(G, ws=ws).T
        torch.cuda.synchronize()
        log(f"[pmc] count {i}: T={T}")
    x = torch.empty(256 * 2**20, dtype=torch.int32, device="cuda").fill_(1)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log("[pmc] copy of 1 GiB done")
    print(json.dumps({"pmc_program": "done", "scale": args.scale, "counted_steps": args.warmup + args.steps,
                      "copy_bytes": 2**30}), flush=True)


def _csv_rows(d, name):
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(d, "**", f"*{name}"), recursive=True):
        out += list(csv.DictReader(open(f)))
    return out


def _kname(name):
    import re
    m = re.match(r"[A-Za-z_0-9]+", name)  # names may be truncated (-T)
    return m.group(0) if m else name[:40]


# kernels launched with several LDS sizes (the table bins of the heavy
# kernel) get one row per size
_MULTI_LDS = ("heavy_kernel",)


def _kkey(row):
    kn = _kname(row["Kernel_Name"])
    if kn in _MULTI_LDS:
        lds = _col(row, "LDS_Block_Size")
        if lds is not None:
            return f"{kn}[lds={int(lds)}]"
    return kn


def _col(row, *keys):
    """First present (case-insensitive) column among keys, as a float."""
    low = {k.lower(): v for k, v in row.items()}
    for k in keys:
        v = low.get(k.lower())
        if v not in (None, ""):
            try:
                return float(v)
            except ValueError:
                pass
    return None


WAVES_PER_SIMD_MAX = 8     # gfx950: 32 waves per CU, 4 SIMDs
VGPRS_PER_SIMD_LANE = 512  # unified architectural + accumulation registers
LDS_PER_CU = 160 * 1024
# rocprofv3's kernel-trace VGPR_Count on gfx950 counts register pairs: for the
# same kernels the compiler's kernel-resource-usage report gives twice the
# figure (32, 80 and 128 allocated registers appear as 16, 40 and 64)
TRACE_VGPR_UNIT = 2


def theoretical_waves_per_simd(vgpr, agpr, lds, wg):
    """Waves per SIMD a kernel's resources allow on gfx950: registers
    (granule 8 of the 512 per lane), LDS (whole workgroups in 160 KB per CU)
    and the 8-wave cap.  Returns (waves, limiter)."""
    lim = [(WAVES_PER_SIMD_MAX, "cap")]
    regs = (vgpr or 0) + (agpr or 0)
    if regs > 0:
        lim.append((VGPRS_PER_SIMD_LANE // (int(math.ceil(regs / 8.0)) * 8), "vgpr"))
    waves_wg = max(1, int(math.ceil((wg or 64) / 64.0)))
    if lds and lds > 0:
        lim.append(((LDS_PER_CU // int(lds)) * waves_wg / 4.0, "lds"))
    return min(lim)


def summarize_counters(args):
    """Per-kernel figures of one count call (the last of the pmc program's
    calls: dispatches from the last --call-start kernel, root_key_kernel by
    default, to the next stats_kernel) from
    rocprofv3 --pmc runs (any of TCC_EA0_RDREQ_DRAM_32B,
    TCC_EA0_WRREQ_WRITE_DRAM_32B, TCC_HIT, TCC_MISS, FETCH_SIZE, WRITE_SIZE,
    MeanOccupancyPerCU) and a --kernel-trace run (durations, registers, LDS,
    workgroup size).  DRAM bytes are 32 x the 32-byte request counts, scaled
    by what they read for the pmc program's plain 1 GiB device copy.  Writes
    <out>.md and <out>.json; the json's "heavy" entry is the traffic per
    heavy-stage launch that bench.py reports."""
    counters = {}  # counter -> {dispatch: value}
    names, dur = {}, {}
    for d in args.pmc_dir or []:
        for r in _csv_rows(d, "counter_collection.csv"):
            k = int(r["Dispatch_Id"])
            c = r["Counter_Name"]
            counters.setdefault(c, {})
            counters[c][k] = counters[c].get(k, 0.0) + float(r["Counter_Value"])
            names.setdefault(c, {})[k] = _kkey(r)
            if "Start_Timestamp" in r and r["Start_Timestamp"]:
                dur.setdefault(c, {})[k] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6

    def last_call(nm):
        ids = sorted(nm)
        if args.whole_run:
            return ids
        starts = [k for k in ids if nm[k].startswith(args.call_start)]
        if not starts:
            return ids
        a = starts[-1]
        b = next((k for k in ids if k > a and nm[k].startswith("stats_kernel")), ids[-1])
        return [k for k in ids if a <= k <= b]

    def copy_value(c):
        v = [x for k, x in counters.get(c, {}).items() if "copy" in names[c][k].lower()]
        return max(v) if v else None

    table = {}

    def add(kn, field, v):
        t = table.setdefault(kn, {})
        t[field] = t.get(field, 0.0) + v

    calib = {}
    for c, unit, field, expect in (("TCC_EA0_RDREQ_DRAM_32B", 32.0, "dram_read", 2**30),
                                   ("TCC_EA0_WRREQ_WRITE_DRAM_32B", 32.0, "dram_write", 2**30),
                                   ("FETCH_SIZE", 1024.0, "fetch", 2**30), ("WRITE_SIZE", 1024.0, "write", 2**30),
                                   ("TCC_HIT", 1.0, "l2_hit", None), ("TCC_MISS", 1.0, "l2_miss", None)):
        if c not in counters:
            continue
        f = 1.0
        if expect:
            cv = copy_value(c)
            f = expect / (cv * unit) if cv else 1.0
            calib[c] = {"copy_reading_bytes": cv * unit if cv else None, "factor": f}
        for k in last_call(names[c]):
            add(names[c][k], field, counters[c][k] * unit * f)
            if field in ("dram_read", "fetch"):
                add(names[c][k], "n_" + field, 1)
                add(names[c][k], "ms_" + field, dur.get(c, {}).get(k, 0.0))
    if "MeanOccupancyPerCU" in counters:
        c = "MeanOccupancyPerCU"
        for k in last_call(names[c]):
            w = dur.get(c, {}).get(k, 1.0)
            add(names[c][k], "occ_w", counters[c][k] * w)
            add(names[c][k], "occ_t", w)
    # durations and resources from the kernel trace (last call)
    trace = sorted(_csv_rows(args.trace_dir, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"])) \
        if args.trace_dir else []
    tnames = {i: _kkey(r) for i, r in enumerate(trace)}
    res = {}
    for i in last_call(tnames) if trace else []:
        r = trace[i]
        kn = tnames[i]
        add(kn, "ms", (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
        add(kn, "n", 1)
        vg_trace = _col(r, "VGPR_Count", "Arch_VGPR_Count", "vgpr_count")
        ag_trace = _col(r, "Accum_VGPR_Count", "agpr_count")
        res[kn] = (vg_trace * TRACE_VGPR_UNIT if vg_trace is not None else None,
                   ag_trace * TRACE_VGPR_UNIT if ag_trace is not None else None,
                   _col(r, "LDS_Block_Size", "LDS_Size", "Group_Segment_Size", "lds_size"),
                   _col(r, "Workgroup_Size_X", "Workgroup_Size", "workgroup_size"))
    for kn, t in table.items():
        if "ms" not in t:  # no trace: the counter run's own durations
            t["ms"] = t.get("ms_dram_read", t.get("ms_fetch", 0.0))
            t["n"] = t.get("n_dram_read", t.get("n_fetch", 0))
        if kn in res:
            vg, ag, lds, wg = res[kn]
            w, why = theoretical_waves_per_simd(vg, ag, lds, wg)
            t.update(vgpr=vg, agpr=ag, lds=lds, wg=wg, theo_waves_simd=w, theo_limit=why)
        if t.get("occ_t"):
            t["achieved_waves_simd"] = t["occ_w"] / t["occ_t"] / 4.0
        hm = t.get("l2_hit", 0.0) + t.get("l2_miss", 0.0)
        if hm > 0:
            t["l2_hit_frac"] = t.get("l2_hit", 0.0) / hm
    tot_ms = sum(t.get("ms", 0.0) for t in table.values())
    tot_b = sum(t.get("dram_read", 0.0) + t.get("dram_write", 0.0) for t in table.values())
    heavy = {}
    for kn, t in table.items():
        if kn.startswith("heavy_kernel"):
            for f in ("n", "ms", "dram_read", "dram_write", "fetch", "write"):
                heavy[f] = heavy.get(f, 0.0) + t.get(f, 0.0)
    rec = {"calibration": calib, "kernel_ms": tot_ms, "dram_bytes": tot_b, "kernels": table,
           "heavy": {"source_sha256": source_sha(), "dispatches": heavy.get("n"), "ms": heavy.get("ms"),
                     "traffic_bytes": (heavy.get("dram_read", 0.0) + heavy.get("dram_write", 0.0)) or None,
                     "fetch_write_bytes": (heavy.get("fetch", 0.0) + heavy.get("write", 0.0)) or None}}

    def fmt(v, f):
        return "" if v is None else f.format(v)
    out_md = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
              ("Every kernel of the traced run (all its calls), one row per kernel name. " if args.whole_run else
               "Every kernel of one count call (the last of the program's calls), one row per kernel name. ") +
              "DRAM bytes: 32 x TCC_EA0_RDREQ_DRAM_32B (reads) and 32 x TCC_EA0_WRREQ_WRITE_DRAM_32B (writes), "
              "each scaled by its reading for a plain 1 GiB device copy "
              + ", ".join(f"{c}: factor {v['factor']:.3f}" for c, v in calib.items()) + ". "
              "Requests leaving the L2 for memory include those the 256 MB Infinity Cache serves: "
              "no counter here separates them. L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS). "
              "Theoretical waves per SIMD from the kernel's registers (the trace's VGPR_Count, which "
              "counts register pairs on gfx950, times 2), LDS and workgroup size "
              "(8 at most); achieved = MeanOccupancyPerCU / 4 (time-weighted over dispatches).", "",
              "| kernel | dispatches | ms | DRAM read GB | DRAM write GB | GB/s | L2 hit | VGPR | LDS B | WG | "
              "theo. waves/SIMD | achieved waves/SIMD |",
              "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    has_dram = "TCC_EA0_RDREQ_DRAM_32B" in counters
    for kn, t in sorted(table.items(), key=lambda kv: -kv[1].get("ms", 0.0)):
        if tot_ms and t.get("ms", 0.0) < 0.003 * tot_ms:
            continue
        b = t.get("dram_read", 0.0) + t.get("dram_write", 0.0)
        rd = t.get("dram_read", 0.0) / 1e9 if has_dram else None
        wr = t.get("dram_write", 0.0) / 1e9 if has_dram else None
        out_md.append(
            f"| {kn} | {int(t.get('n', 0))} | {t.get('ms', 0.0):.3f} | {fmt(rd, '{:.3f}')} | "
            f"{fmt(wr, '{:.3f}')} | {fmt(b / (t['ms'] / 1e3) / 1e9 if t.get('ms') and has_dram else None, '{:.0f}')} | "
            f"{fmt(t.get('l2_hit_frac'), '{:.2f}')} | {fmt(t.get('vgpr'), '{:.0f}')} | {fmt(t.get('lds'), '{:.0f}')} | "
            f"{fmt(t.get('wg'), '{:.0f}')} | {fmt(t.get('theo_waves_simd'), '{:.2f}')}"
            f"{' (' + t['theo_limit'] + ')' if t.get('theo_limit') else ''} | "
            f"{fmt(t.get('achieved_waves_simd'), '{:.2f}')} |")
    if tot_ms and not has_dram:
        out_md += ["", f"All kernels {'of the run' if args.whole_run else 'of the call'}: {tot_ms:.2f} ms of "
                       f"kernel time (no counters taken).", ""]
    if tot_ms and has_dram:
        out_md += ["", f"All kernels of the call: {tot_ms:.2f} ms of kernel time, {tot_b/1e9:.1f} GB of DRAM "
                       f"requests: {tot_b / (tot_ms / 1e3) / 1e9:.0f} GB/s time-weighted "
                       f"({tot_b / (tot_ms / 1e3) / 1e9 / HBM_PEAK_GBS:.2f} of 8 TB/s).", ""]
    stats = _csv_rows(args.trace_dir, "kernel_stats.csv") if args.trace_dir else []
    if stats:
        stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
        out_md += ["Top kernels of the whole traced run (rocprofv3 --kernel-trace --stats; every call of the "
                   "program, warm-up included):", "",
                   "| kernel | calls | total ms | average us | share |", "|---|---|---|---|---|"]
        for r in stats[:14]:
            out_md.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.3f} | "
                          f"{float(r['AverageNs'])/1e3:.1f} | {float(r['Percentage']):.1f}% |")
        out_md.append("")
    if heavy.get("ms") and has_dram:
        out_md += [f"Heavy stage (heavy_kernel, {int(heavy.get('n', 0))} dispatches): {heavy['ms']:.3f} ms, "
                   f"DRAM traffic {rec['heavy']['traffic_bytes'] / 1e9 if rec['heavy']['traffic_bytes'] else 0:.2f} GB "
                   f"per call (source sha256 {rec['heavy']['source_sha256'][:16]}).", ""]
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(out_md) + "\n")
    with open(args.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"summary": args.out}), flush=True)


def rmat_line(args, scale, steps, warmup, comparator=True, stream=True, root_candidates=0, profile=True):
    """One single-graph line: tc_count on R-MAT `scale` resident in HBM,
    timed over `steps` calls after `warmup`, beside the comparator, with
    the dominant stage's roofline and per-stage rates."""
    import numpy as np
    import torch
    import graphgen
    import paper_2210_00389_amd as tc
    from paper_2210_00389_amd import comm_model
    dev = torch.device("cuda:0")
    log(f"[bench] generating R-MAT scale {scale} ef {args.edge_factor} seed {args.seed}")
    t = time.perf_counter()
    g = graphgen.rmat(scale, args.edge_factor, seed=args.seed)
    t_gen = time.perf_counter() - t
    t = time.perf_counter()
    G = tc.from_host_pairs(g.n, g.src, g.dst, device=dev)
    del g
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    n, m, nnz = G.n, G.m, G.nnz
    log(f"[bench] n={n} m={m} nnz={nnz} gen {t_gen:.1f}s upload+build {t_build:.2f}s")

    ws = tc.Workspace(dev)
    res = tc.CountResult(torch.zeros(1, dtype=torch.int64, device=dev), torch.zeros(1, dtype=torch.int64, device=dev),
                         None, None)
    tb = torch.zeros(1, dtype=torch.int64, device=dev)
    tun_c = tun_b = None
    tune_info = None
    if args.autotune:
        # both paths tuned by the library's autotuner before timing (outside
        # the timed region); the comparator over a shorter search when its
        # calls are long
        from paper_2210_00389_amd import tune
        t0 = time.perf_counter()
        tun_c = tc.autotune_count(G, "cover", reps=3, ws=ws, use_cache=False)
        t1 = time.perf_counter()
        tun_b = (tc.autotune_count(G, "edge", reps=2 if nnz > 2**26 else 3, ws=ws, use_cache=False,
                                   space=tune.EDGE_SPACE_SHORT if nnz > 2**26 else None) if comparator else None)
        t2 = time.perf_counter()
        tune_info = {"cover": tun_c, "comparator": tun_b, "cover_search_s": round(t1 - t0, 1),
                     "comparator_search_s": round(t2 - t1, 1)}
        log(f"[bench] autotuned: cover {tun_c} comparator {tun_b}")
    step = lambda: tc.count(G, ws=ws, out=res, tuning=tun_c)  # noqa: E731
    base = lambda: tc.count_edge_baseline(G, ws=ws, out=tb, tuning=tun_b)  # noqa: E731

    # per-stage HIP events (for the stage rates and the roofline); the
    # latency line times both paths without them
    tc.profile_enable(profile)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done; timing {steps} cover-edge steps")
    wall, per, stages = run_timed(step, steps, torch.cuda.synchronize)
    T, h = res.T, res.h
    st = tc.read_stats(ws)
    comp = None
    if comparator:
        for _ in range(warmup):
            base()
        torch.cuda.synchronize()
        log(f"[bench] timing {steps} comparator steps")
        wall_b, per_b, stages_b = run_timed(base, steps, torch.cuda.synchronize)
        Tb = int(tb.item())
        st_b = tc.read_stats(ws)
        comp = {
            "name": "plain direction-oriented edge iterator (same kernels, forward lists N+(x))",
            "ms_per_step": 1000 * wall_b / steps,
            "p50_ms": percentile(per_b, 50), "p99_ms": percentile(per_b, 99),
            "edges_per_s": m / (wall_b / steps), "triangles": Tb, "exact_match": Tb == T,
            "stream_elems": st_b["stream_elems"], "bin_elems": st_b["bin_elems"],
            "stages_ms": {k: statistics.mean(v) for k, v in stages_b.items()},
        }
        hb = comp["stages_ms"].get("heavy")
        if hb:
            comp["heavy_GBps"] = round(stage_bytes("heavy", st_b, n, nnz, False) / (hb / 1e3) / 1e9, 1)
        comp["element_ratio_vs_cover"] = round(st_b["stream_elems"] / max(st["stream_elems"], 1), 4)
    tc.profile_enable(False)

    ms = 1000 * wall / steps
    stage_avg = {k: statistics.mean(v) for k, v in stages.items()}
    dom = max(stage_avg, key=stage_avg.get) if stage_avg else None
    dom_bytes = stage_bytes(dom, st, n, nnz, True) if dom else None
    roof = None
    if dom_bytes is not None:
        ach = dom_bytes / (stage_avg[dom] / 1000.0) / 1e9
        tr = traffic_record(scale) if dom == "heavy" else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": int(tr["traffic_bytes"]) if tr and tr.get("traffic_bytes") else None,
                "traffic_source": tr.get("summary") if tr else None,
                "algorithmic_bytes_per_launch": int(dom_bytes), "avg_launch_ms": round(stage_avg[dom], 4)}
    stage_roofs = {}
    for k, v in stage_avg.items():
        b = stage_bytes(k, st, n, nnz, True)
        if b is not None and v > 0:
            stage_roofs[k] = {"ms": round(v, 4), "GB/s": round(b / (v / 1000.0) / 1e9, 1)}
        else:
            stage_roofs[k] = {"ms": round(v, 4)}

    # the whole path: every stage's algorithmic bytes over the time per count
    path_bytes = sum(b for b in (stage_bytes(k, st, n, nnz, True) for k in stage_avg) if b is not None)
    path_gbs = path_bytes / (ms / 1000.0) / 1e9
    end_to_end = ({"algorithmic_bytes": int(path_bytes), "ms": round(ms, 4), "GB/s": round(path_gbs, 1),
                   "frac": round(path_gbs / HBM_PEAK_GBS, 4)} if path_bytes else None)

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"rmat_s{scale}.json")
    if args.edge_factor == 16 and args.seed == 1 and os.path.exists(gpath):
        gd = json.load(open(gpath))
        golden = {"triangles": gd["triangles"], "h": gd["h"], "match": gd["triangles"] == T and gd["h"] == h}
        if comp is not None:
            golden["comparator_match"] = comp["triangles"] == gd["triangles"]

    # Distributed-variant context: the communication model of the parallel
    # algorithm for this graph's measured k, on one node of 8 GPUs
    comm = None
    if st["num_levels"] > 0 and m > 0:  # the one-workgroup path reports no level count
        deg = np.diff(G.row_offsets.cpu().numpy())
        wedges = int((deg * (deg - 1) // 2).sum())
        cmr = comm_model.volume_for_count(n, m, h, st["num_levels"], p=8, wedges=wedges)
        comm = {"p": 8, "k": round(cmr.k, 4), "level_bits": cmr.level_bits, "wedges": wedges,
                "cover_bytes": int(cmr.cover_bytes), "wedge_check_bytes": int(cmr.previous_bytes),
                "reduction": round(cmr.reduction, 2)}

    sbw = None
    if stream:
        log("[bench] copy/read bandwidth reference")
        sbw = stream_bandwidth(torch, dev)
        if roof is not None:
            sbw["dominant_vs_copy"] = round(roof["achieved"] / sbw["copy_GBps"], 4)

    root_choice = None
    if root_candidates > 0:
        # the paper's goal of the smallest k: choose the root among the
        # highest-degree vertices by |H|, then time the count from it
        log(f"[bench] root choice over {root_candidates} candidates")
        t0 = time.perf_counter()
        rc = tc.select_root(G, root_candidates, ws=ws)
        t_sel = time.perf_counter() - t0
        res_r = tc.count(G, root=rc.root, ws=ws)
        wall_r, per_r, _ = run_timed(lambda: tc.count(G, root=rc.root, ws=ws, out=res_r), steps,
                                     torch.cuda.synchronize)
        assert res_r.T == T
        root_choice = {"candidates": rc.candidates, "h": rc.h, "root": rc.root, "k": min(rc.h) / m,
                       "k_default_root": h / m, "select_ms": 1000 * t_sel,
                       "count_ms_chosen_root": 1000 * wall_r / steps}
    del G, ws
    torch.cuda.empty_cache()
    return {
        "metric": "cover-edge TC edges/s", "value": m / (wall / steps), "unit": "edges/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {scale}, edge factor {args.edge_factor}, "
                               f"(0.57,0.19,0.19,0.05), seed {args.seed}, relabelled, symmetrised, deduplicated; "
                               f"root = largest degree; single-graph cover-edge count",
                   "n": n, "m": m, "nnz": nnz, "h": h, "k": h / max(m, 1), "triangles": T,
                   "num_levels": st["num_levels"]},
        "triangles_per_s": T / (wall / steps),
        "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99),
        "comparator": comp,
        "speedup_vs_comparator": (comp["ms_per_step"] / ms) if comp else None,
        "roofline": roof,
        "end_to_end": end_to_end,
        "stream_bw": sbw,
        "stages": stage_roofs,
        "work": st,
        "golden": golden,
        "comm_model": comm,
        "root_choice": root_choice,
        "tuning": tune_info,
    }


def _child(args, mode, scale, budget=None):
    """Start a CPU-oracle leg (cpu_leg / cpu_validate) of this benchmark as
    a child process on the host cores; its JSON line comes back on stdout."""
    cmd = [sys.executable, os.path.abspath(__file__), mode, "--scale", str(scale),
           "--edge-factor", str(args.edge_factor), "--seed", str(args.seed)]
    if budget is not None:
        cmd += ["--cpu-budget", str(budget)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env)


def _collect(proc):
    out, _ = proc.communicate()
    lines = [l for l in out.splitlines() if l.startswith("{")]
    if proc.returncode != 0 or not lines:
        log(f"[bench] CPU leg failed with status {proc.returncode}")
        return None
    return json.loads(lines[-1])


def start_cpu_legs(args):
    """Start the CPU oracle legs; call before anything touches the GPU, so
    that no child is started from a process that has initialised it."""
    kids = {}
    if not args.no_cpu_baseline:
        kids["cpu"] = _child(args, "--cpu-leg", args.scale, args.cpu_budget)
        if args.cpu_check_scale > 0:
            kids["check"] = _child(args, "--cpu-validate", args.cpu_check_scale)
    return kids


def bench_rmat(args, kids):
    """The headline line (R-MAT at --scale, default 24) with the R-MAT scale
    20 line nested, and the CPU oracle legs (already started) beside them."""
    out = rmat_line(args, args.scale, args.steps, args.warmup, comparator=not args.no_comparator,
                    stream=not args.no_stream, root_candidates=args.root_candidates)
    if args.latency_scale > 0:
        # the small-graph latency floor (1000 counts of R-MAT scale 10)
        lat = rmat_line(args, args.latency_scale, args.latency_steps, max(args.warmup, 20),
                        comparator=not args.no_comparator, stream=False, profile=False)
        out[f"rmat{args.latency_scale}_latency"] = {k: lat[k] for k in (
            "ms_per_step", "p50_ms", "p99_ms", "config", "golden")}
        if lat["comparator"]:
            out[f"rmat{args.latency_scale}_latency"]["comparator"] = {
                k: lat["comparator"][k] for k in ("ms_per_step", "p50_ms", "p99_ms", "exact_match")}
            out[f"rmat{args.latency_scale}_latency"]["p50_speedup_vs_comparator"] = (
                lat["comparator"]["p50_ms"] / lat["p50_ms"])
    if args.nested_scale > 0 and args.nested_scale != args.scale:
        nest = rmat_line(args, args.nested_scale, args.steps, args.warmup, comparator=not args.no_comparator,
                         stream=False)
        out[f"rmat{args.nested_scale}"] = {k: nest[k] for k in (
            "value", "unit", "ms_per_step", "p50_ms", "p99_ms", "triangles_per_s", "config", "comparator",
            "speedup_vs_comparator", "roofline", "end_to_end", "stages", "golden", "tuning")}
    cpu = None
    if "cpu" in kids:
        log("[bench] waiting for the CPU oracle legs")
        cpu = _collect(kids["cpu"])
        if cpu is not None and "check" in kids:
            cpu["estimator_check"] = _collect(kids["check"])
    out["cpu_baseline"] = cpu
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--nested-scale", type=int, default=20, help="a second R-MAT line nested in the first (0: none)")
    ap.add_argument("--latency-scale", type=int, default=10,
                    help="an R-MAT latency line (small-graph floor) nested in the first (0: none)")
    ap.add_argument("--latency-steps", type=int, default=1000)
    ap.add_argument("--cpu-check-scale", type=int, default=20,
                    help="scale of the full oracle run that checks the sampled CPU estimate (0: none)")
    ap.add_argument("--cpu-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-validate", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle count in the CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="time both single-graph paths with their compiled defaults")
    ap.add_argument("--no-stream", action="store_true", help="skip the copy/read bandwidth reference")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--workload", choices=("rmat", "batch", "serving", "pmc", "list"), default="rmat")
    ap.add_argument("--root-candidates", type=int, default=0,
                    help="also choose the root by |H| among this many highest-degree vertices and time it")
    ap.add_argument("--summarize-counters", action="store_true",
                    help="per-kernel DRAM traffic, L2 hits and occupancy of one count call from rocprofv3 runs")
    ap.add_argument("--trace-dir", default=None)
    ap.add_argument("--pmc-dir", action="append", default=None, help="a rocprofv3 --pmc output folder (repeatable)")
    ap.add_argument("--whole-run", action="store_true", help="summaries: every dispatch of the run, not one call")
    ap.add_argument("--call-start", default="root_key_kernel",
                    help="summaries: the first kernel of a call (forward_meta_kernel for the comparator)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--pool", type=int, default=128, help="serving: graphs in the request pool")
    ap.add_argument("--rates", type=float, nargs="+", default=[50, 100, 200, 500, 1000, 2000])
    ap.add_argument("--requests", type=int, default=2000, help="serving: requests per rate")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--serve-scale-max", type=int, default=22)
    ap.add_argument("--serve-cl-n-max", type=int, default=10**6)
    ap.add_argument("--serve-budget-frac", type=float, default=0.5)
    ap.add_argument("--no-batching", action="store_true", help="serving: one tc_count per request")
    ap.add_argument("--pmc-comparator", action="store_true",
                    help="pmc program: count with the comparator (table bins in sequence)")
    ap.add_argument("--batch-max", type=int, default=64, help="serving: graphs per coalesced launch")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.cpu_leg:
        cpu_leg(args)
        return
    if args.cpu_validate:
        cpu_validate(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("bench.py: only --gpus 1 is supported (the library runs on one GPU)")
        sys.exit(2)

    kids = start_cpu_legs(args) if args.workload == "rmat" else {}
    import torch

    torch.cuda.set_device(0)
    if args.workload == "pmc":
        bench_pmc(args)
        return
    if args.workload != "rmat":
        out = {"batch": bench_batch, "serving": bench_serving, "list": bench_list}[args.workload](args)
        line = json.dumps(out)
        print(line, flush=True)
        if args.json_out:
            with open(args.json_out, "w") as f:
                f.write(line + "\n")
        return
    out = bench_rmat(args, kids)
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
