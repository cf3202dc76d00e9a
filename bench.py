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
        # vertex records + descriptor counts + plan bytes + scan
        return 32 * n + 4 * n + n + 12 * n
    if name == "resolve":
        # per descriptor: its column entry + the other endpoint's record;
        # light merges; records written; items written, read and regrouped
        d = st.get("descriptors", 0)
        return 36 * d + 4 * st["light_elems"] + 16 * st["heavy_desc"] + 48 * st["heavy_items"]
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


def cpu_baseline(g, n, m, budget_s):
    """Oracle on the host: full BFS + cover edges, count over a row prefix."""
    import numpy as np
    import oracle
    c = oracle.from_graph(g)
    t = time.perf_counter()
    lv = oracle.bfs_levels(c)
    t_bfs = time.perf_counter() - t
    t = time.perf_counter()
    hu, _ = oracle.cover_edges(c, lv.levels)
    t_h = time.perf_counter() - t
    rows_done, t_count, chunk = 0, 0.0, max(1, c.n // 4096)
    while rows_done < c.n and t_count < budget_s:
        hi = min(c.n, rows_done + chunk)
        t = time.perf_counter()
        oracle.count_rows(c, lv.levels, rows_done, hi)
        t_count += time.perf_counter() - t
        rows_done = hi
        chunk = min(chunk * 2, max(1, c.n // 64))
    frac = rows_done / max(c.n, 1)
    est = t_bfs + t_h + t_count / max(frac, 1e-12)
    # the cost measures of Alg. 1 on this graph (not timed): the list
    # elements its intersections would scan, beside the GPU path's own count
    work = oracle.work_counters(c, lv.levels)
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = platform.processor()
    return {
        "value": m / est, "unit": "edges/s", "cores": 1, "kind": "oracle",
        "sample": (f"single-threaded CPU oracle (oracle/oracle.c, gcc -O2) on this host "
                   f"(1 of {os.cpu_count()} cores, {model}): full BFS {t_bfs:.2f}s + cover edges "
                   f"{t_h:.2f}s, count over rows [0, {rows_done}) = {100 * frac:.1f}% of the rows "
                   f"(uniform sample, ids relabelled) in {t_count:.1f}s, scaled to all rows; "
                   f"estimated full run {est:.1f}s"),
        "estimated_full_seconds": est,
        "alg1_work": work,
    }


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
    for rate in args.rates:
        reqs = serve.make_requests(sizes, serve.count_ws_bytes, rate=rate, count=args.requests, seed=int(rate))
        st = serve.Server(ex, slots=args.slots, budget_bytes=budget).run(reqs)
        torch.cuda.synchronize()
        st["rate_req_s"] = rate
        log(f"[bench] rate {rate}: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
            f"edges/s {st['edges_per_s']:.3e} busy {st['busy_fraction']:.2f}")
        runs.append(st)
    top = runs[-1]
    return {
        "metric": "served cover-edge TC latency p50/p99 and edges/s", "value": top["edges_per_s"],
        "unit": "edges/s", "n_gpus": 1, "steps": args.requests, "warmup": 0, "ms_per_step": top["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals over a pool of {len(specs)} graphs (half R-MAT scale "
                               f"12-{args.serve_scale_max} ef16, half Chung-Lu gamma 2.1 mean degree 20 n "
                               f"1e4-{args.serve_cl_n_max:.0e}); {args.slots} slots; HBM budget "
                               f"{args.serve_budget_frac:.2f} of free", "rates": args.rates,
                   "requests_per_rate": args.requests},
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"], "runs": runs,
    }


COUNT_SRC = os.path.join(ROOT, "paper_2210_00389_amd", "csrc", "count.hip")


def source_sha(path=COUNT_SRC):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def traffic_record(scale):
    """Counter-measured HBM bytes per heavy-stage launch, from the committed
    summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a
    1 GiB copy; None when missing or taken on another kernel source."""
    path = os.path.join(ROOT, "profiles", f"heavy_rmat{scale}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_sha():
        return None
    return rec


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
        r = tc.count(G, ws=ws)
        torch.cuda.synchronize()
        log(f"[pmc] count {i}: T={r.T}")
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


def summarize(args):
    """Turn rocprofv3 CSV output into the short text summaries kept under
    profiles/ (kernel statistics, heavy-stage spans, counter traffic)."""
    out_md = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", ""]
    rec = {}
    if args.trace_dir:
        stats = _csv_rows(args.trace_dir, "kernel_stats.csv")
        stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
        out_md += ["Top kernels (rocprofv3 --kernel-trace --stats):", "",
                   "| kernel | calls | total ms | average us | share |", "|---|---|---|---|---|"]
        for r in stats[:16]:
            out_md.append(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs'])/1e6:.3f} | "
                          f"{float(r['AverageNs'])/1e3:.1f} | {float(r['Percentage']):.1f}% |")
        trace = sorted(_csv_rows(args.trace_dir, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"]))
        heavy = [r for r in trace if "heavy_kernel" in r["Kernel_Name"]]
        spans = []
        for i in range(0, len(heavy) - 3, 4):  # the four bins of one call run side by side
            grp = heavy[i:i + 4]
            spans.append((max(int(r["End_Timestamp"]) for r in grp) - min(int(r["Start_Timestamp"]) for r in grp)) / 1e6)
        if spans:
            out_md += ["", f"Heavy stage (the four bin kernels: in sequence for the cover count, side by side for the comparator) span per call, ms: "
                           f"{', '.join(f'{x:.3f}' for x in spans)}; mean {statistics.mean(spans):.3f}", ""]
            rec["heavy_span_ms"] = spans
    if args.fetch_dir and args.write_dir:
        def per_dispatch(d, counter):
            rows = _csv_rows(d, "counter_collection.csv")
            acc = {}
            for r in rows:
                if r["Counter_Name"] != counter:
                    continue
                k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
            return sorted(acc.items())
        fetch = per_dispatch(args.fetch_dir, "FETCH_SIZE")
        write = per_dispatch(args.write_dir, "WRITE_SIZE")
        copy_f = [v for (d, k), v in fetch if "copy" in k.lower()]
        copy_w = [v for (d, k), v in write if "copy" in k.lower()]
        hf = [v for (d, k), v in fetch if "heavy_kernel" in k]
        hw = [v for (d, k), v in write if "heavy_kernel" in k]
        gib_kib = 2**30 / 1024
        ff = gib_kib / max(copy_f) if copy_f else None
        wf = gib_kib / max(copy_w) if copy_w else None
        steps = len(hf) // 4
        fetch_launch = [sum(hf[4 * i:4 * i + 4]) * 1024 * ff for i in range(steps)] if ff else []
        write_launch = [sum(hw[4 * i:4 * i + 4]) * 1024 * wf for i in range(len(hw) // 4)] if wf else []
        rec.update({"source_sha256": source_sha(), "fetch_factor": ff, "write_factor": wf,
                    "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
                    "fetch_bytes_per_launch": fetch_launch, "write_bytes_per_launch": write_launch,
                    "traffic_bytes": (statistics.mean(fetch_launch[1:] or fetch_launch) +
                                      statistics.mean(write_launch[1:] or write_launch))
                    if fetch_launch and write_launch else None})
        out_md += ["Counter traffic of the heavy stage (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, "
                   "KiB per dispatch summed over the four bin kernels of a call):", "",
                   f"- calibration: a 1 GiB device copy reads FETCH_SIZE {copy_f} KiB, WRITE_SIZE {copy_w} KiB "
                   f"-> factors {ff:.3f} (fetch), {wf:.3f} (write)" if ff and wf else "- calibration missing",
                   f"- fetch per call (scaled), GB: {', '.join(f'{x/1e9:.3f}' for x in fetch_launch)}",
                   f"- write per call (scaled), GB: {', '.join(f'{x/1e9:.4f}' for x in write_launch)}",
                   f"- traffic per call (mean after the first): {rec['traffic_bytes']/1e9:.3f} GB"
                   if rec.get("traffic_bytes") else "", ""]
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(out_md) + "\n")
    if args.fetch_dir:
        with open(args.out + ".json", "w") as f:
            json.dump(rec, f, indent=1)
    print(json.dumps({"summary": args.out}), flush=True)


def summarize_kernels(args):
    """Per-kernel HBM traffic of one count call from two unfiltered
    rocprofv3 --pmc runs of the pmc program (FETCH_SIZE, then WRITE_SIZE),
    scaled by the 1 GiB copy like the heavy-stage record.  A count call is
    the dispatches from a root_key_kernel to the next stats_kernel; the
    table covers the last call, and the totals give the time-weighted rate
    over all of its kernels."""
    import re

    def rows(d, counter):
        acc, dur, name = {}, {}, {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            k = int(r["Dispatch_Id"])
            acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
            dur[k] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            m = re.match(r"[A-Za-z_0-9]+", r["Kernel_Name"])  # names are truncated (-T)
            name[k] = m.group(0) if m else r["Kernel_Name"][:40]
        return acc, dur, name

    fa, fdur, fname = rows(args.fetch_dir, "FETCH_SIZE")
    wa, _, wname = rows(args.write_dir, "WRITE_SIZE")
    gib_kib = 2**30 / 1024
    cf = [v for k, v in fa.items() if "copy" in fname[k].lower()]
    cw = [v for k, v in wa.items() if "copy" in wname[k].lower()]
    ff, wf = gib_kib / max(cf), gib_kib / max(cw)

    def last_call(names):
        ids = sorted(names)
        starts = [k for k in ids if names[k].startswith("root_key_kernel")]
        a = starts[-1]
        b = next(k for k in ids if k > a and names[k].startswith("stats_kernel"))
        return [k for k in ids if a <= k <= b]

    fc, wc = last_call(fname), last_call(wname)
    table = {}
    for k in fc:
        t = table.setdefault(fname[k], [0, 0.0, 0.0, 0.0])
        t[0] += 1
        t[1] += fdur[k]
        t[2] += fa[k] * 1024 * ff
    for k in wc:
        if wname[k] in table:
            table[wname[k]][3] += wa[k] * 1024 * wf
    tot_ms = sum(t[1] for t in table.values())
    tot_b = sum(t[2] + t[3] for t in table.values())
    out_md = [f"# {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
              f"Counter traffic of every kernel of one count call (the last of the program's calls), "
              f"FETCH_SIZE x {ff:.3f} and WRITE_SIZE x {wf:.3f} (factors from a 1 GiB device copy); "
              f"kernel times are those of the counter runs.", "",
              "| kernel | dispatches | kernel ms | fetch GB | write GB | GB/s |", "|---|---|---|---|---|---|"]
    for nm, t in sorted(table.items(), key=lambda kv: -kv[1][1]):
        if t[1] < 0.005 * tot_ms:
            continue
        out_md.append(f"| {nm} | {t[0]} | {t[1]:.3f} | {t[2]/1e9:.3f} | {t[3]/1e9:.3f} | "
                      f"{(t[2] + t[3]) / (t[1] / 1e3) / 1e9:.0f} |")
    out_md += ["", f"All kernels of the call: {len(fc)} dispatches, {tot_ms:.2f} ms of kernel time, "
                   f"{tot_b/1e9:.1f} GB moved: {tot_b / (tot_ms / 1e3) / 1e9:.0f} GB/s time-weighted "
                   f"({tot_b / (tot_ms / 1e3) / 1e9 / HBM_PEAK_GBS:.2f} of 8 TB/s).", ""]
    rec = {"fetch_factor": ff, "write_factor": wf, "kernel_ms": tot_ms, "bytes": tot_b,
           "kernels": {nm: {"dispatches": t[0], "ms": t[1], "fetch_bytes": t[2], "write_bytes": t[3]}
                       for nm, t in table.items()}}
    with open(args.out + ".md", "w") as f:
        f.write("\n".join(out_md) + "\n")
    with open(args.out + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"summary": args.out}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edge-factor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle count in the CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-stream", action="store_true", help="skip the copy/read bandwidth reference")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--workload", choices=("rmat", "batch", "serving", "pmc", "list"), default="rmat")
    ap.add_argument("--root-candidates", type=int, default=0,
                    help="also choose the root by |H| among this many highest-degree vertices and time it")
    ap.add_argument("--summarize", action="store_true", help="summarise rocprofv3 output into --out(.md/.json)")
    ap.add_argument("--summarize-kernels", action="store_true",
                    help="per-kernel counter traffic of one count call from unfiltered --pmc runs")
    ap.add_argument("--trace-dir", default=None)
    ap.add_argument("--fetch-dir", default=None)
    ap.add_argument("--write-dir", default=None)
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
    args = ap.parse_args()

    if args.summarize:
        summarize(args)
        return
    if args.summarize_kernels:
        summarize_kernels(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("bench.py: only --gpus 1 is supported (the library runs on one GPU)")
        sys.exit(2)

    import torch
    import graphgen
    import paper_2210_00389_amd as tc

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
    dev = torch.device("cuda:0")
    log(f"[bench] generating R-MAT scale {args.scale} ef {args.edge_factor} seed {args.seed}")
    t = time.perf_counter()
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    t_gen = time.perf_counter() - t
    t = time.perf_counter()
    G = tc.from_host_pairs(g.n, g.src, g.dst, device=dev)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    n, m, nnz = G.n, G.m, G.nnz
    log(f"[bench] n={n} m={m} nnz={nnz} gen {t_gen:.1f}s upload+build {t_build:.2f}s")

    ws = tc.Workspace(dev)
    ws_b = tc.Workspace(dev)
    res = tc.CountResult(torch.zeros(1, dtype=torch.int64, device=dev), torch.zeros(1, dtype=torch.int64, device=dev),
                         None, None)
    tb = torch.zeros(1, dtype=torch.int64, device=dev)
    step = lambda: tc.count(G, ws=ws, out=res)  # noqa: E731
    base = lambda: tc.count_edge_baseline(G, ws=ws_b, out=tb)  # noqa: E731

    tc.profile_enable(True)
    for _ in range(args.warmup):
        step()
        if not args.no_comparator:
            base()
    torch.cuda.synchronize()
    log(f"[bench] warmup done; timing {args.steps} cover-edge steps")
    wall, per, stages = run_timed(step, args.steps, torch.cuda.synchronize)
    T, h = res.T, res.h
    st = tc.read_stats(ws)
    comp = None
    if not args.no_comparator:
        log(f"[bench] timing {args.steps} comparator steps")
        wall_b, per_b, stages_b = run_timed(base, args.steps, torch.cuda.synchronize)
        Tb = int(tb.item())
        st_b = tc.read_stats(ws_b)
        comp = {
            "name": "plain direction-oriented edge iterator (same kernels, forward lists N+(x))",
            "ms_per_step": 1000 * wall_b / args.steps,
            "p50_ms": percentile(per_b, 50), "p99_ms": percentile(per_b, 99),
            "edges_per_s": m / (wall_b / args.steps), "triangles": Tb, "exact_match": Tb == T,
            "stream_elems": st_b["stream_elems"],
            "stages_ms": {k: statistics.mean(v) for k, v in stages_b.items()},
        }
    tc.profile_enable(False)

    ms = 1000 * wall / args.steps
    stage_avg = {k: statistics.mean(v) for k, v in stages.items()}
    dom = max(stage_avg, key=stage_avg.get)
    dom_bytes = stage_bytes(dom, st, n, nnz, True)
    roof = None
    if dom_bytes is not None:
        ach = dom_bytes / (stage_avg[dom] / 1000.0) / 1e9
        tr = traffic_record(args.scale) if dom == "heavy" else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": int(tr["traffic_bytes"]) if tr and tr.get("traffic_bytes") else None,
                "algorithmic_bytes_per_launch": int(dom_bytes), "avg_launch_ms": round(stage_avg[dom], 4)}
    stage_roofs = {}
    for k, v in stage_avg.items():
        b = stage_bytes(k, st, n, nnz, True)
        if b is not None and v > 0:
            stage_roofs[k] = {"ms": round(v, 4), "GB/s": round(b / (v / 1000.0) / 1e9, 1)}
        else:
            stage_roofs[k] = {"ms": round(v, 4)}

    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", f"rmat_s{args.scale}.json")
    if args.edge_factor == 16 and args.seed == 1 and os.path.exists(gpath):
        gd = json.load(open(gpath))
        golden = {"triangles": gd["triangles"], "h": gd["h"], "match": gd["triangles"] == T and gd["h"] == h}

    # Distributed-variant context: the communication model of the parallel
    # algorithm for this graph's measured k, on one node of 8 GPUs
    import numpy as np
    from paper_2210_00389_amd import comm_model
    deg = np.diff(G.row_offsets.cpu().numpy())
    wedges = int((deg * (deg - 1) // 2).sum())
    cmr = comm_model.volume_for_count(n, m, h, st["num_levels"], p=8, wedges=wedges)
    comm = {"p": 8, "k": round(cmr.k, 4), "level_bits": cmr.level_bits, "wedges": wedges,
            "cover_bytes": int(cmr.cover_bytes), "wedge_check_bytes": int(cmr.previous_bytes),
            "reduction": round(cmr.reduction, 2)}

    stream = None
    if not args.no_stream:
        log("[bench] copy/read bandwidth reference")
        stream = stream_bandwidth(torch, dev)
        if roof is not None:
            stream["dominant_vs_copy"] = round(roof["achieved"] / stream["copy_GBps"], 4)

    root_choice = None
    if args.root_candidates > 0:
        # the paper's goal of the smallest k: choose the root among the
        # highest-degree vertices by |H|, then time the count from it
        log(f"[bench] root choice over {args.root_candidates} candidates")
        t0 = time.perf_counter()
        rc = tc.select_root(G, args.root_candidates, ws=ws)
        t_sel = time.perf_counter() - t0
        res_r = tc.count(G, root=rc.root, ws=ws)
        wall_r, per_r, _ = run_timed(lambda: tc.count(G, root=rc.root, ws=ws, out=res_r), args.steps,
                                     torch.cuda.synchronize)
        assert res_r.T == T
        root_choice = {"candidates": rc.candidates, "h": rc.h, "root": rc.root, "k": min(rc.h) / m,
                       "k_default_root": h / m, "select_ms": 1000 * t_sel,
                       "count_ms_chosen_root": 1000 * wall_r / args.steps}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline(g, n, m, args.cpu_budget)

    out = {
        "metric": "cover-edge TC edges/s", "value": m / (wall / args.steps), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale}, edge factor {args.edge_factor}, "
                               f"(0.57,0.19,0.19,0.05), seed {args.seed}, relabelled, symmetrised, deduplicated; "
                               f"root = largest degree; single-graph cover-edge count",
                   "n": n, "m": m, "nnz": nnz, "h": h, "k": h / max(m, 1), "triangles": T,
                   "num_levels": st["num_levels"]},
        "triangles_per_s": T / (wall / args.steps),
        "p50_ms": percentile(per, 50), "p99_ms": percentile(per, 99),
        "comparator": comp,
        "speedup_vs_comparator": (comp["ms_per_step"] / ms) if comp else None,
        "roofline": roof,
        "stream_bw": stream,
        "stages": stage_roofs,
        "work": st,
        "golden": golden,
        "comm_model": comm,
        "root_choice": root_choice,
        "cpu_baseline": cpu,
    }
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
