"""Serving loop: scheduler logic on a virtual clock with a fake engine (CPU)."""
import numpy as np
import pytest

from paper_1804_09996_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeEngine:
    """Each launch takes `a + b * queries` seconds of virtual time; results are
    a pure function of each query (its row sum), so they cannot depend on the
    batch."""

    def __init__(self, clock, a=1e-3, b=1e-5):
        self.clock, self.a, self.b = clock, a, b
        self.done_at = {}
        self.launches = []
        self.concurrent_max = 0

    def launch(self, slot, batch):
        n = sum(r.size for r in batch)
        self.done_at[slot] = self.clock() + self.a + self.b * n
        self.launches.append((slot, [r.rid for r in batch], self.clock()))
        self.concurrent_max = max(self.concurrent_max, len(self.done_at))

    def ready(self, slot):
        return self.clock() >= self.done_at[slot] - 1e-15

    def deliver(self, slot, batch):
        del self.done_at[slot]
        for r in batch:
            r.ids = np.rint(r.queries.sum(1, keepdims=True) * 1000).astype(np.int32)
            r.dist = r.queries.sum(1, keepdims=True)

    def next_event(self):
        return min(self.done_at.values()) if self.done_at else None


def run(reqs, n_slots=3, cap=256, budget=10_000, bpq=10, a=1e-3, b=1e-5):
    clock = Clock()
    eng = FakeEngine(clock, a, b)
    sch = serve.Scheduler(n_slots, cap, budget, bpq)

    def idle(next_arrival):
        cands = [t for t in (eng.next_event(), next_arrival) if t is not None and t > clock.t]
        clock.t = min(cands) if cands else clock.t + 1e-6

    stats = serve.serve(eng, sch, reqs, clock=clock, idle=idle)
    return stats, eng, sch


def _reqs(n, rate, seed=3, max_batch=64, d=4):
    q = np.random.default_rng(seed).standard_normal((500, d)).astype(np.float32)
    return serve.poisson_requests(d, q, rate, n, seed, efs=(16, 32), max_batch=max_batch)


def test_every_request_completes_once_with_its_own_results():
    reqs = _reqs(80, 2000.0)
    stats, eng, sch = run(reqs)
    assert stats["requests"] == 80
    for r in reqs:
        assert r.done >= r.start >= r.arrival
        np.testing.assert_array_equal(r.ids, np.rint(r.queries.sum(1, keepdims=True) * 1000).astype(np.int32))
    launched = [rid for _, rids, _ in eng.launches for rid in rids]
    assert sorted(launched) == list(range(80))  # never split, never duplicated


def test_fifo_order_and_memory_budget():
    reqs = _reqs(120, 20000.0)
    stats, eng, sch = run(reqs, n_slots=4, cap=128, budget=1500, bpq=10)
    assert sch.max_mem_used <= 1500
    starts = [(r.start, r.arrival, r.rid) for r in reqs]
    order = [rid for _, _, rid in sorted(starts)]
    assert order == sorted(order, key=lambda k: (reqs[k].arrival, k))  # started in arrival order
    assert sch.mem_used == 0 and sorted(sch.free_slots) == [0, 1, 2, 3]


def test_slots_overlap_and_are_reused():
    reqs = _reqs(60, 50000.0)
    stats, eng, sch = run(reqs, n_slots=3, cap=64)
    assert eng.concurrent_max == 3
    assert {s for s, _, _ in eng.launches} == {0, 1, 2}
    assert len(eng.launches) > 3


def test_latency_of_a_lone_request_is_its_service_time():
    q = np.ones((5, 4), np.float32)
    reqs = [serve.Request(rid=0, queries=q, ef=16, arrival=0.25)]
    stats, eng, sch = run(reqs, a=2e-3, b=1e-4)
    assert reqs[0].latency == pytest.approx(2e-3 + 5e-4)
    assert stats["latency_ms_p50"] == pytest.approx(2.5)


def test_backpressure_grows_latency_not_memory():
    light, _, _ = run(_reqs(100, 500.0), budget=4000)
    heavy, _, sch = run(_reqs(100, 200000.0), budget=4000)
    assert heavy["latency_ms_p99"] > light["latency_ms_p99"]
    assert sch.max_mem_used <= 4000


def test_oversized_request_is_rejected():
    sch = serve.Scheduler(2, 16, 10_000, 10)
    with pytest.raises(ValueError):
        sch.arrive(serve.Request(rid=0, queries=np.zeros((17, 4), np.float32), ef=8, arrival=0.0))


def test_request_stream_is_seeded():
    a = _reqs(20, 100.0, seed=9)
    b = _reqs(20, 100.0, seed=9)
    assert [(r.size, r.ef, r.arrival) for r in a] == [(r.size, r.ef, r.arrival) for r in b]
    assert all(1 <= r.size <= 64 for r in a)
