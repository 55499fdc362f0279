"""The TF-update server's scheduling on the CPU, with an executor that
computes through the oracle: admission by memory budget and slot cap, LRU
eviction of idle volumes, rejection of bad requests, continuous batching of
requests that arrive while launches are in flight, and exact results."""
import collections

import numpy as np
import pytest

import workloads as W
from paper_2407_21552_amd.serve import Executor, Request, Server, VolumeSpec, requests_from


class OracleExecutor(Executor):
    """Synchronous CPU executor; a launch 'finishes' after `delay` ticks."""

    def __init__(self, orc, delay=0):
        self.orc = orc
        self.delay = delay
        self.events = []
        self.launches = []

    def footprint(self, spec):
        return spec.n * spec.bricks + 2 * spec.bricks

    def admit(self, spec):
        vol = spec.load()
        h = dict(spec=spec, pdms=self.orc.pdms(vol, spec.bounds, spec.levels), alive=True)
        self.events.append(("admit", spec.vol_id))
        return h

    def ready(self, h):
        return True

    def evict(self, h):
        h["alive"] = False
        self.events.append(("evict", h["spec"].vol_id))

    def launch(self, batch):
        for h, alpha, req in batch:
            assert h["alive"]
            req.result = self.orc.tf_update(h["pdms"], h["spec"].bounds, alpha, h["spec"].levels)[0]
        self.launches.append([req.req_id for _, _, req in batch])
        return [self.delay]

    def finished(self, ticket):
        if ticket[0] <= 0:
            return True
        ticket[0] -= 1
        return False


def catalog(k=5, seed=0):
    rng = np.random.default_rng(seed)
    out = {}
    for v in range(k):
        shape = tuple(int(s) for s in rng.integers(8, 24, size=3))
        vol = rng.integers(0, 256, size=shape).astype(np.uint8)
        vol[rng.random(shape) < 0.8] = 0
        out[v] = VolumeSpec(v, shape, np.uint8, 256, W.uniform_bounds(256, 8), lambda vol=vol: vol)
    return out


def tfs(rng, k):
    return [W.trapezoid_tf(256, int(rng.integers(1, 4)), rng) for _ in range(k)]


def test_results_are_exact(orc):
    cat = catalog()
    ex = OracleExecutor(orc)
    srv = Server(ex, cat, budget_bytes=10**9)
    rng = np.random.default_rng(1)
    reqs = [Request(i, int(rng.integers(0, 5)), a, 0.0) for i, a in enumerate(tfs(rng, 30))]
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert len(srv.completed) == 30 and not srv.rejected
    for r in reqs:
        spec = cat[r.vol_id]
        want = orc.tf_update(orc.pdms(spec.load(), spec.bounds, 256), spec.bounds, r.alpha, 256)[0]
        np.testing.assert_array_equal(r.result, want)


def test_slot_cap_and_lru_eviction(orc):
    cat = catalog(6)
    ex = OracleExecutor(orc)
    srv = Server(ex, cat, budget_bytes=10**9, max_slots=3)
    rng = np.random.default_rng(2)
    order = [0, 1, 2, 0, 3, 4, 0, 5]
    for i, v in enumerate(order):
        srv.submit(Request(i, v, tfs(rng, 1)[0], 0.0))
        srv.drain()
    assert len(srv.resident) <= 3
    # 0 is used again before 3 arrives, so 1 (least recently used) goes first
    evicted = [v for kind, v in ex.events if kind == "evict"]
    assert evicted[0] == 1
    assert 0 in srv.resident
    assert len(srv.completed) == len(order)


def test_memory_budget_forces_eviction(orc):
    cat = catalog(4)
    ex = OracleExecutor(orc)
    largest = max(ex.footprint(s) for s in cat.values())
    srv = Server(ex, cat, budget_bytes=largest + 1, max_slots=24)
    rng = np.random.default_rng(3)
    for i, v in enumerate([0, 1, 2, 3, 0]):
        srv.submit(Request(i, v, tfs(rng, 1)[0], 0.0))
        srv.drain()
        assert srv.used <= srv.budget
    assert srv.stats["evictions"] >= 3
    assert len(srv.completed) == 5


def test_bad_requests_are_rejected(orc):
    cat = catalog(2)
    ex = OracleExecutor(orc)
    srv = Server(ex, cat, budget_bytes=10**9)
    srv.submit(Request(0, 99, np.zeros(256, np.float32), 0.0))       # unknown volume
    srv.submit(Request(1, 0, np.zeros(100, np.float32), 0.0))        # wrong table length
    tiny = Server(ex, cat, budget_bytes=10)
    tiny.submit(Request(2, 1, np.zeros(256, np.float32), 0.0))        # larger than the budget
    srv.drain()
    tiny.drain()
    assert [r.req_id for r in srv.rejected] == [0, 1]
    assert [r.req_id for r in tiny.rejected] == [2]
    assert all(r.error for r in srv.rejected + tiny.rejected)


def test_requests_arriving_during_a_launch_join_the_next_one(orc):
    cat = catalog(3)
    ex = OracleExecutor(orc, delay=3)
    srv = Server(ex, cat, budget_bytes=10**9)
    rng = np.random.default_rng(4)
    a = tfs(rng, 6)
    for i in range(2):
        srv.submit(Request(i, i % 3, a[i], 0.0))
    assert srv.tick() == 2                       # first launch, still in flight
    for i in range(2, 6):
        srv.submit(Request(i, i % 3, a[i], 0.0))
    assert srv.tick() == 4                       # admitted while the first runs
    assert len(srv.inflight) == 2
    srv.drain()
    assert ex.launches == [[0, 1], [2, 3, 4, 5]]
    assert len(srv.completed) == 6


def test_max_batch_and_poisson_schedule(orc):
    cat = catalog(3)
    ex = OracleExecutor(orc)
    srv = Server(ex, cat, budget_bytes=10**9, max_batch=4)
    sched = requests_from(W.poisson_requests(2000.0, 0.01, list(cat), {v: 256 for v in cat}, seed=9))
    assert 5 <= len(sched) <= 60
    assert all(b.arrival >= a.arrival for a, b in zip(sched, sched[1:]))
    for r in sched:
        srv.submit(r)
    srv.drain()
    assert all(len(b) <= 4 for b in ex.launches)
    assert len(srv.completed) == len(sched)
    rep = srv.report()
    assert rep["completed"] == len(sched) and rep["p99_ms"] >= rep["p50_ms"]


class LimitedExecutor(OracleExecutor):
    """An executor with at most `limit` requests of a volume in flight (as
    the GPU executor's pool of output maps), whose launches stay in flight
    for `delay` ticks.  It records the most requests of one volume ever in
    flight, counted as the GPU pool would see them: launched and not yet
    retired by the server."""

    def __init__(self, orc, limit, delay=0):
        super().__init__(orc, delay)
        self.limit = limit
        self.server = None
        self.peak = 0

    def per_volume_limit(self):
        return self.limit

    def launch(self, batch):
        ticket = super().launch(batch)
        unretired = collections.Counter(r.vol_id for _, reqs in self.server.inflight for r in reqs)
        unretired.update(req.vol_id for _, _, req in batch)
        self.peak = max(self.peak, max(unretired.values()))
        return ticket


def test_per_volume_limit_keeps_arrival_order(orc):
    cat = catalog(3)
    ex = LimitedExecutor(orc, limit=2)
    srv = Server(ex, cat, budget_bytes=10**9, max_batch=8)
    ex.server = srv
    rng = np.random.default_rng(6)
    vols = [0, 0, 0, 1, 0, 2, 1, 1, 1, 0]
    for i, (v, a) in enumerate(zip(vols, tfs(rng, len(vols)))):
        srv.submit(Request(i, v, a, 0.0))
    srv.drain()
    assert len(srv.completed) == len(vols)
    for launch in ex.launches:
        per = collections.Counter(vols[i] for i in launch)
        assert max(per.values()) <= 2
    # each launch takes the earliest requests its limits allow, in order
    assert ex.launches[0] == [0, 1, 3, 5, 6]
    assert sorted(i for b in ex.launches for i in b) == list(range(len(vols)))
    for b in ex.launches:
        assert b == sorted(b)
    for r in srv.completed:
        spec = cat[r.vol_id]
        want = orc.tf_update(orc.pdms(spec.load(), spec.bounds, 256), spec.bounds, r.alpha, 256)[0]
        np.testing.assert_array_equal(r.result, want)


def test_long_queue_drains_in_arrival_order(orc):
    cat = catalog(2)
    ex = OracleExecutor(orc)
    srv = Server(ex, cat, budget_bytes=10**9, max_batch=16)
    rng = np.random.default_rng(8)
    a = tfs(rng, 4)
    n = 2000
    for i in range(n):
        srv.submit(Request(i, i % 2, a[i % 4], 0.0))
    srv.drain()
    assert len(srv.completed) == n and len(ex.launches) == n // 16
    assert [i for b in ex.launches for i in b] == list(range(n))


def test_pooled_poisson_tfs_are_shared():
    sched = W.poisson_requests(5000.0, 0.2, [0, 1], {0: 256, 1: 4096}, seed=3, tf_pool=4)
    assert len(sched) > 500
    ids = collections.defaultdict(set)
    for _, v, alpha in sched:
        assert alpha.shape == ({0: 256, 1: 4096}[v],)
        ids[v].add(id(alpha))
    assert all(len(s) <= 4 for s in ids.values())


def test_per_volume_limit_counts_requests_in_flight(orc):
    """The limit covers every launch still in flight, not only the one being
    formed: a pool of `limit` output maps per volume is never handed to a
    request while an earlier request holding the same map is unretired."""
    cat = catalog(2)
    ex = LimitedExecutor(orc, limit=2, delay=4)
    done_at_retire = {}
    srv = Server(ex, cat, budget_bytes=10**9, max_batch=8,
                 on_complete=lambda r: done_at_retire.setdefault(r.req_id, r.done))
    ex.server = srv
    rng = np.random.default_rng(10)
    a = tfs(rng, 24)
    for i in range(24):
        srv.submit(Request(i, 0 if i % 3 else 1, a[i], 0.0))
        srv.tick()                        # launches overlap: each stays in flight 4 ticks
    srv.drain()
    assert len(srv.completed) == 24
    assert ex.peak == 2
    assert sorted(done_at_retire) == list(range(24))
    for r in srv.completed:
        spec = cat[r.vol_id]
        want = orc.tf_update(orc.pdms(spec.load(), spec.bounds, 256), spec.bounds, r.alpha, 256)[0]
        np.testing.assert_array_equal(r.result, want)
