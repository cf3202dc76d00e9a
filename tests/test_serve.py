"""Host logic of the request loop (admission, residency, LRU eviction,
arrivals, statistics) with a fake executor; no GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2210_00389_amd.serve import (Request, ResidentCache, Scheduler, Server, make_requests, percentile,
                                        poisson_arrivals)


def req(rid, gid, t=0.0, gb=100, ws=10):
    return Request(rid, gid, t, n=10, nnz=20, graph_bytes=gb, ws_bytes=ws)


def test_resident_cache_lru_and_pins():
    c = ResidentCache()
    c.put(1, 50, pinned=False)
    c.put(2, 50, pinned=True)
    c.put(3, 50, pinned=False)
    c.touch(1)  # order now 2, 3, 1
    assert c.evictable_bytes() == 100
    assert c.evict(60) == [3, 1]  # oldest unpinned first; 2 is pinned
    assert c.has(2) and not c.has(1) and not c.has(3)
    c.unpin(2)
    assert c.evict(1) == [2]


def test_scheduler_fifo_slots_and_budget():
    s = Scheduler(slots=2, budget_bytes=300)
    for i in range(4):
        s.submit(req(i, gid=i, gb=100, ws=20))
    started, ev = s.admit(0.0)
    assert [r.rid for r in started] == [0, 1] and ev == []  # two slots
    assert s.used() == 2 * 120
    s.complete(started[0], 1.0)
    started2, ev2 = s.admit(1.0)
    # request 2 needs 120 B; 240 - 20 + 120 = 340 > 300 -> graph 0 (idle) is evicted
    assert [r.rid for r in started2] == [2] and ev2 == [0]
    assert started2[0].uploaded and s.evictions == 1


def test_scheduler_reuses_resident_graph():
    s = Scheduler(slots=1, budget_bytes=1000)
    s.submit(req(0, gid=7))
    (r0,), _ = s.admit(0.0)
    s.complete(r0, 0.5)
    s.submit(req(1, gid=7))
    (r1,), _ = s.admit(0.6)
    assert r0.uploaded and not r1.uploaded


def test_scheduler_waits_when_memory_is_pinned():
    s = Scheduler(slots=3, budget_bytes=200)
    s.submit(req(0, gid=0, gb=100, ws=20))
    s.submit(req(1, gid=1, gb=100, ws=20))
    started, _ = s.admit(0.0)
    assert [r.rid for r in started] == [0]  # 1 does not fit while 0 runs (its graph is pinned)
    s.complete(started[0], 1.0)
    started, ev = s.admit(1.0)
    assert [r.rid for r in started] == [1] and ev == [0]


def test_scheduler_rejects_oversized_request():
    s = Scheduler(slots=1, budget_bytes=50)
    with pytest.raises(ValueError):
        s.submit(req(0, gid=0, gb=100))


def test_poisson_rate_and_percentile():
    a = poisson_arrivals(1000.0, 20000, seed=3)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 1000.0) < 30.0
    assert percentile([1, 2, 3, 4], 50) == 2.5 and percentile([5], 99) == 5


class FakeExecutor:
    """Sleeps a size-dependent time and answers a deterministic function of
    the graph id; records the peak number of concurrent runs."""

    def __init__(self):
        self.active = 0
        self.peak = 0
        self.lock = threading.Lock()
        self.evicted = []

    def run(self, slot, r, upload):
        with self.lock:
            self.active += 1
            self.peak = max(self.peak, self.active)
        time.sleep(0.002 + 0.0005 * (r.graph_id % 4))
        with self.lock:
            self.active -= 1
        return r.graph_id * 7 + 1, r.graph_id + 3

    def evict(self, gid):
        self.evicted.append(gid)


def test_server_overlaps_and_answers_every_request():
    sizes = {g: (100 + g, 400 + 2 * g, 5000 + 10 * g) for g in range(12)}
    reqs = make_requests(sizes, lambda n, nnz: 1000, rate=2000.0, count=120, seed=5)
    ex = FakeExecutor()
    st = Server(ex, slots=4, budget_bytes=40000).run(reqs)
    assert st["requests"] == 120
    assert all(r.triangles == r.graph_id * 7 + 1 and r.h == r.graph_id + 3 for r in reqs)
    assert ex.peak > 1 and st["max_running"] > 1
    assert st["p99_ms"] >= st["p50_ms"] > 0
    assert all(r.t_admit >= r.arrival and r.t_done >= r.t_admit for r in reqs)


def test_server_evicts_under_a_small_budget():
    sizes = {g: (100, 400, 5000) for g in range(10)}
    reqs = make_requests(sizes, lambda n, nnz: 1000, rate=500.0, count=60, seed=9)
    ex = FakeExecutor()
    st = Server(ex, slots=2, budget_bytes=15000).run(reqs)
    assert st["evictions"] > 0 and set(ex.evicted) <= set(sizes)
    assert all(r.triangles == r.graph_id * 7 + 1 for r in reqs)


def test_levels_digest():
    """BLAKE2b-64 of the little-endian int32 levels: the empty array gives
    the digest of no bytes, and the value depends on dtype only through the
    int32 cast, and on the order of the vertices."""
    import hashlib

    from paper_2210_00389_amd.serve import levels_digest
    assert levels_digest(np.zeros(0, np.int32)) == hashlib.blake2b(b"", digest_size=8).hexdigest()
    a = np.array([0, 1, 1, 2, 0], np.int32)
    assert levels_digest(a) == hashlib.blake2b(bytes([0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 2, 0, 0, 0, 0, 0, 0, 0]),
                                              digest_size=8).hexdigest()
    assert levels_digest(a.astype(np.int64)) == levels_digest(a)
    assert levels_digest(a[::-1]) != levels_digest(a)


class DigestExecutor(FakeExecutor):
    def run(self, slot, r, upload):
        t, h = super().run(slot, r, upload)
        return t, h, f"g{r.graph_id}"


def test_server_carries_levels_digest():
    sizes = {g: (100, 400, 5000) for g in range(6)}
    reqs = make_requests(sizes, lambda n, nnz: 1000, rate=2000.0, count=30, seed=3)
    Server(DigestExecutor(), slots=2, budget_bytes=40000).run(reqs)
    assert all(r.levels_hash == f"g{r.graph_id}" for r in reqs)


class BatchingExecutor(FakeExecutor):
    """FakeExecutor with run_batch; records the size of every batched job."""

    def __init__(self):
        super().__init__()
        self.jobs = []

    def run_batch(self, slot, reqs):
        self.jobs.append(len(reqs))
        time.sleep(0.002)
        return [(r.graph_id * 7 + 1, r.graph_id + 3) for r in reqs]


def test_scheduler_coalesces_small_requests():
    """A slot that starts a small request takes the other waiting small
    requests that fit; large requests keep a slot each; the slot is free
    again only when every request of its job is complete."""
    small = lambda r: r.n <= 100  # noqa: E731
    s = Scheduler(slots=2, budget_bytes=10_000, small=small, batch_max=3)
    big = Request(0, 0, 0.0, n=1000, nnz=10, graph_bytes=100, ws_bytes=10)
    s.submit(big)
    for i in range(1, 6):
        s.submit(Request(i, i, 0.0, n=50, nnz=10, graph_bytes=100, ws_bytes=10))
    started, _ = s.admit(0.0)
    jobs = {}
    for r in started:
        jobs.setdefault(r.job, []).append(r.rid)
    assert sorted(jobs.values()) == [[0], [1, 2, 3]]  # batch_max 3; two slots
    assert [r.batched for r in started] == [False, True, True, True]
    assert len(s.waiting) == 2 and not s.free_slots
    for r in [x for x in started if x.rid in (1, 2)]:
        s.complete(r, 1.0)
    assert not s.free_slots  # request 3 still holds the batch's slot
    s.complete(next(x for x in started if x.rid == 3), 1.0)
    (r4, r5), _ = s.admit(1.0)
    assert r4.job == r5.job and r4.batched and r5.batched


def test_server_batches_and_answers_every_request():
    sizes = {g: ((50 if g % 2 else 5000), 400, 5000) for g in range(12)}
    reqs = make_requests(sizes, lambda n, nnz: 1000, rate=5000.0, count=150, seed=8)
    ex = BatchingExecutor()
    st = Server(ex, slots=3, budget_bytes=200_000, small=lambda r: r.n <= 100, batch_max=16).run(reqs)
    assert st["failed"] == 0 and st["requests"] == 150
    assert all(r.triangles == r.graph_id * 7 + 1 and r.h == r.graph_id + 3 for r in reqs)
    assert st["batched"] == sum(r.n <= 100 for r in reqs) and max(ex.jobs) > 1
    assert all(r.batched == (r.n <= 100) for r in reqs)


class FailingExecutor(BatchingExecutor):
    """Raises on one graph (alone) and on every batch holding another."""

    def run(self, slot, r, upload):
        if r.graph_id == 4:
            raise RuntimeError("device error on graph 4")
        return super().run(slot, r, upload)

    def run_batch(self, slot, reqs):
        if any(r.graph_id == 5 for r in reqs):
            raise RuntimeError("device error in a batch with graph 5")
        return super().run_batch(slot, reqs)


def test_server_isolates_failed_requests():
    """A failing request is answered with its error, the others complete,
    and every slot and reserved byte is released; the run does not raise."""
    sizes = {g: ((50 if g % 2 else 5000), 400, 5000) for g in range(10)}
    reqs = make_requests(sizes, lambda n, nnz: 1000, rate=3000.0, count=100, seed=4)
    srv = Server(FailingExecutor(), slots=2, budget_bytes=100_000, small=lambda r: r.n <= 100, batch_max=8)
    st = srv.run(reqs)
    failed = [r for r in reqs if r.error]
    assert st["failed"] == len(failed) > 0 and st["requests"] == 100
    assert all(r.graph_id == 4 or any(q.graph_id == 5 and q.job == r.job for q in reqs) for r in failed)
    assert all("device error" in r.error and r.triangles == -1 for r in failed)
    assert all(r.triangles == r.graph_id * 7 + 1 for r in reqs if not r.error)
    assert sorted(srv.sched.free_slots) == [0, 1] and srv.sched.reserved == 0 and not srv.sched.running
    assert all(e["pins"] == 0 for e in srv.sched.cache.entries.values())
    assert st["p99_ms"] >= st["p50_ms"] > 0
