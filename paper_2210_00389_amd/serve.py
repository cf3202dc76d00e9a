"""Request loop: continuous admission of counting requests on one GPU.

Requests (a graph id plus its host CSR) arrive over time.  The dispatcher
admits the oldest waiting request as soon as an execution slot is free and
the device memory it needs fits the budget: the graph's CSR (unless it is
already resident) plus the counting workspace.  Idle resident graphs are
evicted least-recently-used first to make room.  Each slot owns a host
thread, a HIP stream (default priority) and a workspace, so requests on
different slots overlap on the device while one slot's host thread waits on
its own stream.  Finished requests leave their CSR resident for later
requests on the same graph.

A request's answer is (T, |H|) and, when the executor is asked for it, a
64-bit digest of the BFS levels (:func:`levels_digest`), so a client can
check the levels without receiving n integers.

The scheduling state (:class:`Scheduler`) is plain Python and is exercised
with a fake executor on the CPU; :class:`GpuExecutor` runs tc_count.
"""
from __future__ import annotations

import hashlib
import math
import queue
import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    graph_id: int
    arrival: float            # seconds from the start of the run
    n: int
    nnz: int
    graph_bytes: int
    ws_bytes: int
    # filled in by the server
    t_admit: float = math.nan
    t_done: float = math.nan
    slot: int = -1
    uploaded: bool = False
    triangles: int = -1
    h: int = -1
    levels_hash: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival

    @property
    def queueing(self) -> float:
        return self.t_admit - self.arrival


class ResidentCache:
    """Device-resident graphs, least recently used first; entries in use by a
    running request are pinned."""

    def __init__(self):
        self.entries: OrderedDict[int, dict] = OrderedDict()

    @property
    def bytes(self) -> int:
        return sum(e["bytes"] for e in self.entries.values())

    def has(self, gid: int) -> bool:
        return gid in self.entries

    def touch(self, gid: int):
        self.entries.move_to_end(gid)

    def pin(self, gid: int):
        self.entries[gid]["pins"] += 1
        self.touch(gid)

    def unpin(self, gid: int):
        self.entries[gid]["pins"] -= 1

    def put(self, gid: int, nbytes: int, handle=None, pinned: bool = True):
        self.entries[gid] = dict(bytes=nbytes, handle=handle, pins=1 if pinned else 0)
        self.touch(gid)

    def evictable_bytes(self) -> int:
        return sum(e["bytes"] for e in self.entries.values() if e["pins"] == 0)

    def evict(self, need: int) -> list:
        """Evict unpinned entries, oldest first, until `need` bytes are freed
        (or nothing is left to evict).  Returns the evicted graph ids."""
        out, freed = [], 0
        for gid in list(self.entries):
            if freed >= need:
                break
            e = self.entries[gid]
            if e["pins"] == 0:
                freed += e["bytes"]
                out.append(gid)
                del self.entries[gid]
        return out


class Scheduler:
    """Admission control: FIFO, a request starts when a slot is free and its
    bytes fit next to the resident graphs and the running requests."""

    def __init__(self, slots: int, budget_bytes: int):
        self.slots = slots
        self.budget = budget_bytes
        self.free_slots = deque(range(slots))
        self.cache = ResidentCache()
        self.running: dict[int, Request] = {}
        self.reserved = 0        # workspaces (and uploads) of running requests
        self.waiting: deque[Request] = deque()
        self.evictions = 0

    def used(self) -> int:
        return self.cache.bytes + self.reserved

    def need(self, r: Request) -> int:
        return r.ws_bytes + (0 if self.cache.has(r.graph_id) else r.graph_bytes)

    def submit(self, r: Request):
        if r.ws_bytes + r.graph_bytes > self.budget:
            raise ValueError(f"request {r.rid} needs {r.ws_bytes + r.graph_bytes} B, budget {self.budget} B")
        self.waiting.append(r)

    def admit(self, now: float):
        """Start waiting requests in arrival order while a slot is free and
        they fit (evicting idle resident graphs, oldest first).  Returns
        (started requests, evicted graph ids)."""
        started, evicted = [], []
        while self.waiting and self.free_slots:
            r = self.waiting[0]
            over = self.used() + self.need(r) - self.budget
            if over > 0:
                own = self.cache.entries.get(r.graph_id)
                keep = own["bytes"] if own is not None and own["pins"] == 0 else 0
                if self.cache.evictable_bytes() - keep < over:
                    break  # wait for running requests to finish
                if own is not None:
                    own["pins"] += 1  # never evict the graph this request needs
                ev = self.cache.evict(over)
                if own is not None:
                    own["pins"] -= 1
                self.evictions += len(ev)
                evicted += ev
            self.waiting.popleft()
            r.slot = self.free_slots.popleft()
            r.t_admit = now
            if self.cache.has(r.graph_id):
                self.cache.pin(r.graph_id)
                r.uploaded = False
            else:
                self.cache.put(r.graph_id, r.graph_bytes, pinned=True)
                r.uploaded = True
            self.reserved += r.ws_bytes
            self.running[r.rid] = r
            started.append(r)
        return started, evicted

    def complete(self, r: Request, now: float):
        r.t_done = now
        self.reserved -= r.ws_bytes
        self.cache.unpin(r.graph_id)
        self.free_slots.append(r.slot)
        del self.running[r.rid]


def levels_digest(levels) -> str:
    """Hex BLAKE2b-64 of the levels as little-endian int32 (one per vertex,
    in vertex order)."""
    a = np.ascontiguousarray(np.asarray(levels, dtype="<i4"))
    return hashlib.blake2b(a.tobytes(), digest_size=8).hexdigest()


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


class Server:
    """Runs a list of requests against an executor with `slots` worker
    threads.  The executor provides run(slot, request, upload: bool) ->
    (triangles, h) or (triangles, h, levels digest) (blocking, called on the
    slot's thread) and evict(gid)."""

    def __init__(self, executor, slots: int, budget_bytes: int):
        self.ex = executor
        self.sched = Scheduler(slots, budget_bytes)
        self.slots = slots

    def run(self, requests) -> dict:
        """Replay the requests in real time (arrival offsets from now) and
        return latency and throughput figures."""
        done_q: queue.Queue = queue.Queue()
        work_q = [queue.Queue() for _ in range(self.slots)]
        errors = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731

        def worker(s):
            while True:
                r = work_q[s].get()
                if r is None:
                    return
                try:
                    ans = self.ex.run(s, r, r.uploaded)
                    r.triangles, r.h = ans[0], ans[1]
                    if len(ans) > 2:
                        r.levels_hash = ans[2]
                except Exception as e:  # reported after the run
                    errors.append((r.rid, repr(e)))
                done_q.put((r, clock()))

        threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(self.slots)]
        for th in threads:
            th.start()
        pending = sorted(requests, key=lambda r: r.arrival)
        arrivals = deque(pending)
        finished, max_running = 0, 0
        busy, busy_since = 0.0, None
        try:
            while finished < len(pending):
                now = clock()
                while arrivals and arrivals[0].arrival <= now:
                    self.sched.submit(arrivals.popleft())
                started, evicted = self.sched.admit(now)
                for gid in evicted:
                    self.ex.evict(gid)
                for r in started:
                    if busy_since is None:
                        busy_since = now
                    work_q[r.slot].put(r)
                max_running = max(max_running, len(self.sched.running))
                timeout = max(0.0, arrivals[0].arrival - clock()) if arrivals else None
                if timeout is None and not self.sched.running:
                    raise RuntimeError("requests left that can never be admitted")
                try:
                    r, t = done_q.get(timeout=timeout)
                except queue.Empty:
                    continue
                batch = [(r, t)]
                while True:
                    try:
                        batch.append(done_q.get_nowait())
                    except queue.Empty:
                        break
                for r, t in batch:
                    self.sched.complete(r, t)
                    finished += 1
                if not self.sched.running and busy_since is not None:
                    busy += max(t for _, t in batch) - busy_since
                    busy_since = None
        finally:
            for q in work_q:
                q.put(None)
            for th in threads:
                th.join()
        if errors:
            raise RuntimeError(f"requests failed: {errors[:3]}")
        lat = [r.latency for r in pending]
        qd = [r.queueing for r in pending]
        span = max(r.t_done for r in pending) - min(r.arrival for r in pending) if pending else 0.0
        tri = sum(r.triangles for r in pending)
        edges = sum(r.nnz // 2 for r in pending)
        return dict(requests=len(pending), slots=self.slots, budget_bytes=self.sched.budget,
                    p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                    mean_ms=1e3 * float(np.mean(lat)) if lat else math.nan,
                    queue_p50_ms=1e3 * percentile(qd, 50), queue_p99_ms=1e3 * percentile(qd, 99),
                    triangles_per_s=tri / span if span > 0 else math.nan,
                    edges_per_s=edges / span if span > 0 else math.nan,
                    busy_fraction=busy / span if span > 0 else math.nan,
                    max_running=max_running, uploads=sum(r.uploaded for r in pending),
                    evictions=self.sched.evictions, span_s=span)


class GpuExecutor:
    """Runs tc_count for requests on per-slot streams.  `pool` maps graph id
    to host CSR (row_offsets int64, cols int32) in pinned memory.  With
    levels_hash, tc_count also writes the levels and the answer carries
    their digest (the levels are copied to the host for it)."""

    def __init__(self, pool: dict, slots: int, device="cuda", levels_hash: bool = False):
        import torch
        from . import api
        self.torch, self.api = torch, api
        self.pool = pool
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.dev = dev
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.ws = [api.Workspace(self.dev) for _ in range(slots)]
        self.resident: dict[int, object] = {}
        self.lock = threading.Lock()
        self.levels_hash = levels_hash

    def graph_bytes(self, gid: int) -> int:
        off, cols = self.pool[gid]
        return off.numel() * 8 + cols.numel() * 4

    def run(self, slot: int, r: Request, upload: bool):
        torch, api = self.torch, self.api
        s = self.streams[slot]
        torch.cuda.set_device(self.dev)
        with torch.cuda.stream(s):
            if upload or r.graph_id not in self.resident:
                off, cols = self.pool[r.graph_id]
                g = api.Graph(r.n, off.to(self.dev, non_blocking=True), cols.to(self.dev, non_blocking=True))
                # the copies run on this slot's stream: finish them before the
                # graph is published, since other slots count it on their own
                # streams with no wait on this one
                s.synchronize()
                with self.lock:
                    self.resident[r.graph_id] = g
            else:
                with self.lock:
                    g = self.resident[r.graph_id]
            res = api.count(g, ws=self.ws[slot], stream=s, return_levels=self.levels_hash)
            out = torch.stack([res.triangles[0], res.h_count[0]]).cpu()
            if self.levels_hash:
                return int(out[0]), int(out[1]), levels_digest(res.levels.cpu().numpy())
        return int(out[0]), int(out[1])

    def evict(self, gid: int):
        with self.lock:
            self.resident.pop(gid, None)


def make_requests(pool_sizes: dict, ws_bytes, rate: float, count: int, seed: int) -> list:
    """`count` Poisson arrivals at `rate` req/s over graph ids drawn uniformly
    from the pool; pool_sizes maps id -> (n, nnz, graph_bytes)."""
    ids = sorted(pool_sizes)
    rng = np.random.default_rng(seed + 1)
    arr = poisson_arrivals(rate, count, seed)
    pick = rng.integers(0, len(ids), size=count)
    out = []
    for i, (t, k) in enumerate(zip(arr, pick)):
        gid = ids[int(k)]
        n, nnz, gb = pool_sizes[gid]
        out.append(Request(i, gid, float(t), n, nnz, gb, int(ws_bytes(n, nnz))))
    return out


def build_pool(graphs, device="cuda"):
    """Host CSR of every raw graph (built on the device by tc_build_csr, then
    copied to pinned host memory): returns (pool, sizes) for GpuExecutor and
    make_requests."""
    import torch
    from . import api
    pool, sizes = {}, {}
    for gid, g in enumerate(graphs):
        G = api.from_host_pairs(g.n, g.src, g.dst, device=device)
        off = torch.empty(G.row_offsets.shape, dtype=torch.int64, pin_memory=True)
        cols = torch.empty(G.cols.shape, dtype=torch.int32, pin_memory=True)
        off.copy_(G.row_offsets)
        cols.copy_(G.cols)
        pool[gid] = (off, cols)
        sizes[gid] = (g.n, int(cols.numel()), off.numel() * 8 + cols.numel() * 4)
    torch.cuda.synchronize()
    return pool, sizes


def count_ws_bytes(n: int, nnz: int) -> int:
    from . import _lib as L
    from .api import workspace_bytes
    return workspace_bytes(L.OP_COUNT, n, nnz)
