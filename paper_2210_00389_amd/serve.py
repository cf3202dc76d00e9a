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

Continuous batching: small graphs (at most 65536 vertices and a bounded
number of entries, the ``small`` predicate) are coalesced.  When a slot
starts a small request it also takes every other waiting small request
that fits the budget (up to ``batch_max``), and the slot counts them all in
one tc_count_batch launch; large graphs keep a slot each.  A request that
fails is answered with its error and does not stop the others; its slot
and reserved bytes are released like those of a finished request.

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
    job: int = -1             # requests of one job share a slot (and a batched launch)
    batched: bool = False
    uploaded: bool = False
    triangles: int = -1
    h: int = -1
    levels_hash: str = ""
    error: str = ""

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
    bytes fit next to the resident graphs and the running requests.  With a
    `small` predicate, a slot that starts a small request also takes the
    other waiting small requests that fit (at most batch_max per job)."""

    def __init__(self, slots: int, budget_bytes: int, small=None, batch_max: int = 64):
        self.slots = slots
        self.budget = budget_bytes
        self.free_slots = deque(range(slots))
        self.cache = ResidentCache()
        self.running: dict[int, Request] = {}
        self.reserved = 0        # workspaces (and uploads) of running requests
        self.waiting: deque[Request] = deque()
        self.evictions = 0
        self.small = small
        self.batch_max = batch_max
        self.slot_users = [0] * slots
        self.jobs = 0

    def used(self) -> int:
        return self.cache.bytes + self.reserved

    def need(self, r: Request) -> int:
        return r.ws_bytes + (0 if self.cache.has(r.graph_id) else r.graph_bytes)

    def submit(self, r: Request):
        if r.ws_bytes + r.graph_bytes > self.budget:
            raise ValueError(f"request {r.rid} needs {r.ws_bytes + r.graph_bytes} B, budget {self.budget} B")
        self.waiting.append(r)

    def _make_room(self, r: Request, evicted: list) -> bool:
        """Evict idle resident graphs (oldest first, never r's own) until r
        fits; False if it cannot fit while the running requests hold their
        memory."""
        over = self.used() + self.need(r) - self.budget
        if over <= 0:
            return True
        own = self.cache.entries.get(r.graph_id)
        keep = own["bytes"] if own is not None and own["pins"] == 0 else 0
        if self.cache.evictable_bytes() - keep < over:
            return False
        if own is not None:
            own["pins"] += 1  # never evict the graph this request needs
        ev = self.cache.evict(over)
        if own is not None:
            own["pins"] -= 1
        self.evictions += len(ev)
        evicted += ev
        return True

    def _start(self, r: Request, slot: int, job: int, now: float):
        r.slot, r.job, r.t_admit = slot, job, now
        if self.cache.has(r.graph_id):
            self.cache.pin(r.graph_id)
            r.uploaded = False
        else:
            self.cache.put(r.graph_id, r.graph_bytes, pinned=True)
            r.uploaded = True
        self.reserved += r.ws_bytes
        self.running[r.rid] = r
        self.slot_users[slot] += 1

    def admit(self, now: float):
        """Start waiting requests in arrival order while a slot is free and
        they fit (evicting idle resident graphs, oldest first); a small
        request's slot also takes the other waiting small requests that fit.
        Returns (started requests, evicted graph ids)."""
        started, evicted = [], []
        while self.waiting and self.free_slots:
            r = self.waiting[0]
            if not self._make_room(r, evicted):
                break  # wait for running requests to finish
            self.waiting.popleft()
            slot = self.free_slots.popleft()
            job = self.jobs
            self.jobs += 1
            self._start(r, slot, job, now)
            started.append(r)
            if self.small is not None and self.small(r):
                r.batched = True
                i = 0
                members = 1
                while i < len(self.waiting) and members < self.batch_max:
                    q = self.waiting[i]
                    if self.small(q) and self._make_room(q, evicted):
                        del self.waiting[i]
                        q.batched = True
                        self._start(q, slot, job, now)
                        started.append(q)
                        members += 1
                    else:
                        i += 1
        return started, evicted

    def complete(self, r: Request, now: float):
        r.t_done = now
        self.reserved -= r.ws_bytes
        self.cache.unpin(r.graph_id)
        self.slot_users[r.slot] -= 1
        if self.slot_users[r.slot] == 0:
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
    (triangles, h) or (triangles, h, levels digest), run_batch(slot,
    requests) -> one such answer per request (both blocking, called on the
    slot's thread) and evict(gid).  `small` (a predicate on requests)
    switches continuous batching on."""

    def __init__(self, executor, slots: int, budget_bytes: int, small=None, batch_max: int = 64):
        self.ex = executor
        self.sched = Scheduler(slots, budget_bytes, small=small, batch_max=batch_max)
        self.slots = slots

    def run(self, requests) -> dict:
        """Replay the requests in real time (arrival offsets from now) and
        return latency and throughput figures."""
        done_q: queue.Queue = queue.Queue()
        work_q = [queue.Queue() for _ in range(self.slots)]
        errors = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731

        def answer(r, ans):
            r.triangles, r.h = ans[0], ans[1]
            if len(ans) > 2:
                r.levels_hash = ans[2]

        def worker(s):
            while True:
                job = work_q[s].get()
                if job is None:
                    return
                try:
                    if len(job) == 1 and not job[0].batched:
                        answer(job[0], self.ex.run(s, job[0], job[0].uploaded))
                    else:
                        answers = self.ex.run_batch(s, job)
                        for r, ans in zip(job, answers):
                            answer(r, ans)
                except Exception as e:  # answered per request; the others go on
                    for r in job:
                        r.error = repr(e)
                        errors.append((r.rid, r.error))
                t = clock()
                for r in job:
                    done_q.put((r, t))

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
                jobs: dict[int, list] = {}
                for r in started:
                    if busy_since is None:
                        busy_since = now
                    jobs.setdefault(r.job, []).append(r)
                for job in jobs.values():
                    work_q[job[0].slot].put(job)
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
        ok = [r for r in pending if not r.error]
        lat = [r.latency for r in ok]
        qd = [r.queueing for r in ok]
        span = max(r.t_done for r in pending) - min(r.arrival for r in pending) if pending else 0.0
        tri = sum(r.triangles for r in ok)
        edges = sum(r.nnz // 2 for r in ok)
        return dict(requests=len(pending), failed=len(pending) - len(ok), errors=errors[:5],
                    batched=sum(r.batched for r in pending), jobs=len({r.job for r in pending}),
                    slots=self.slots, budget_bytes=self.sched.budget,
                    p50_ms=1e3 * percentile(lat, 50), p99_ms=1e3 * percentile(lat, 99),
                    mean_ms=1e3 * float(np.mean(lat)) if lat else math.nan,
                    queue_p50_ms=1e3 * percentile(qd, 50), queue_p99_ms=1e3 * percentile(qd, 99),
                    triangles_per_s=tri / span if span > 0 else math.nan,
                    edges_per_s=edges / span if span > 0 else math.nan,
                    busy_fraction=busy / span if span > 0 else math.nan,
                    max_running=max_running, uploads=sum(r.uploaded for r in pending),
                    evictions=self.sched.evictions, span_s=span)


class GpuExecutor:
    """Runs tc_count for requests on per-slot streams, and tc_count_batch
    for a job of coalesced small requests.  `pool` maps graph id to host CSR
    (row_offsets int64, cols int32) in pinned memory.  Each graph is
    uploaded once: a request whose graph is being uploaded by another slot
    waits for that upload.  With levels_hash the levels are written too and
    the answer carries their digest (the levels are copied to the host for
    it)."""

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
        self.pending: dict[int, threading.Event] = {}
        self.uploads = 0
        self.lock = threading.Lock()
        self.levels_hash = levels_hash

    def graph_bytes(self, gid: int) -> int:
        off, cols = self.pool[gid]
        return off.numel() * 8 + cols.numel() * 4

    def _graph(self, gid: int, n: int, s):
        """The resident device CSR of graph gid, uploading it on stream s if
        no other slot has (or is) uploading it.  The copies are finished
        before the graph is published: other slots count it on their own
        streams with no wait on this one."""
        torch, api = self.torch, self.api
        with self.lock:
            g = self.resident.get(gid)
            if g is not None:
                return g
            ev = self.pending.get(gid)
            mine = ev is None
            if mine:
                ev = self.pending[gid] = threading.Event()
        if not mine:
            ev.wait()
            with self.lock:
                g = self.resident.get(gid)
            if g is None:
                raise RuntimeError(f"the upload of graph {gid} failed on another slot")
            return g
        try:
            off, cols = self.pool[gid]
            with torch.cuda.stream(s):
                g = api.Graph(n, off.to(self.dev, non_blocking=True), cols.to(self.dev, non_blocking=True))
            s.synchronize()
            with self.lock:
                self.resident[gid] = g
                self.uploads += 1
        finally:
            with self.lock:
                del self.pending[gid]
            ev.set()
        return g

    def run(self, slot: int, r: Request, upload: bool):
        torch, api = self.torch, self.api
        s = self.streams[slot]
        torch.cuda.set_device(self.dev)
        g = self._graph(r.graph_id, r.n, s)
        with torch.cuda.stream(s):
            res = api.count(g, ws=self.ws[slot], stream=s, return_levels=self.levels_hash)
            out = torch.stack([res.triangles[0], res.h_count[0]]).cpu()
            if self.levels_hash:
                return int(out[0]), int(out[1]), levels_digest(res.levels.cpu().numpy())
        return int(out[0]), int(out[1])

    def run_batch(self, slot: int, reqs: list) -> list:
        """One tc_count_batch over the graphs of `reqs` (concatenated on the
        slot's stream: vertex bases, row offsets shifted by each graph's
        first entry, local columns as they are)."""
        torch = self.torch
        from . import batch as B
        s = self.streams[slot]
        torch.cuda.set_device(self.dev)
        graphs = [self._graph(r.graph_id, r.n, s) for r in reqs]
        ns = [g.n for g in graphs]
        zs = [g.nnz for g in graphs]
        vb = np.zeros(len(graphs) + 1, dtype=np.int64)
        np.cumsum(ns, out=vb[1:])
        eb = np.zeros(len(graphs) + 1, dtype=np.int64)
        np.cumsum(zs, out=eb[1:])
        with torch.cuda.stream(s):
            vbase = torch.from_numpy(vb).to(self.dev, non_blocking=False)
            offs = [g.row_offsets[:-1] + int(e) for g, e in zip(graphs, eb[:-1])]
            offs.append(torch.tensor([int(eb[-1])], dtype=torch.int64, device=self.dev))
            row_offsets = torch.cat(offs)
            cols = torch.cat([g.cols for g in graphs]) if eb[-1] > 0 else torch.zeros(1, dtype=torch.int32,
                                                                                        device=self.dev)
            b = B.Batch(vbase, row_offsets, cols[: int(eb[-1])], list(zip(ns, zs)))
            # one-wave counting blocks over pieces of 1024 entries: a handful of
            # small graphs then spreads over many waves instead of one block
            # per graph
            res = B.count_batch(b, BATCH_TUNING, ws=self.ws[slot], stream=s, return_levels=self.levels_hash)
            T = res.triangles[: len(reqs)].cpu().tolist()
            H = res.h_count[: len(reqs)].cpu().tolist()
            if self.levels_hash:
                L = res.levels.cpu().numpy()
                return [(t, h, levels_digest(L[vb[i]:vb[i + 1]])) for i, (t, h) in enumerate(zip(T, H))]
        return list(zip(T, H))

    def evict(self, gid: int):
        with self.lock:
            self.resident.pop(gid, None)


SMALL_N = 65536        # the batched kernels' per-graph vertex limit
BATCH_TUNING = {"batch_block": 64, "batch_piece": 1024}  # coalesced launches of a few graphs
SMALL_NNZ = 1 << 18    # entries up to which a graph is coalesced into a batch


def small_request(r: Request, max_n: int = SMALL_N, max_nnz: int = SMALL_NNZ) -> bool:
    """Requests the server coalesces into tc_count_batch launches."""
    return 0 < r.n <= max_n and r.nnz <= max_nnz


def batch_ws_bytes(n: int, nnz: int) -> int:
    """Device bytes one graph adds to a coalesced batch: its share of the
    tc_count_batch workspace plus the concatenated copy of its CSR."""
    from . import _lib as L
    from .api import workspace_bytes
    return workspace_bytes(L.OP_COUNT_BATCH, n, nnz, 1) + 8 * (n + 1) + 4 * nnz


def request_ws_bytes(n: int, nnz: int, batching: bool = True) -> int:
    """Bytes a request reserves while it runs: a coalesced batch's share for
    small graphs (when batching), else the tc_count workspace."""
    if batching and 0 < n <= SMALL_N and nnz <= SMALL_NNZ:
        return batch_ws_bytes(n, nnz)
    return count_ws_bytes(n, nnz)


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
