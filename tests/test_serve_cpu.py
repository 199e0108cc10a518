"""Scheduling of the continuous-batching server, with a timing-only executor.

The test double below never computes: it reports a fixed workspace per
request, completes a batch after a simulated duration and returns the
request ids as "energies", so the tests check admission, batching, FIFO
order, memory caps and concurrency, not numerics (the GPU tests do that).
"""
import collections

import numpy as np
import pytest

import synth

serve = pytest.importorskip("paper_2601_09951_amd.serve")


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4  # every look at the clock advances time
        return self.t


class TimingExecutor:
    def __init__(self, clock, per_req_bytes=100, duration=0.01):
        self.clock = clock
        self.per = per_req_bytes
        self.duration = duration
        self.launched = []
        self.live_bytes = 0
        self.peak = 0

    def hamiltonian(self, req):
        return ("ham", req.rid)

    def release(self, h):
        pass

    def request_bytes(self, key, req):
        return self.per

    def batch_bytes(self, key, reqs, hams):
        return self.per * len(reqs)

    def launch(self, key, reqs, hams, nbytes):
        self.launched.append((key, [r.rid for r in reqs], self.clock.t))
        self.live_bytes += nbytes
        self.peak = max(self.peak, self.live_bytes)
        return {"end": self.clock.t + self.duration, "ids": [r.rid for r in reqs], "bytes": nbytes}

    def done(self, h):
        return self.clock.t >= h["end"]

    def collect(self, h):
        self.live_bytes -= h["bytes"]
        return np.array(h["ids"], dtype=float), None

    def drain(self):
        pass


def _requests(count=300, rate=2000.0):
    return synth.served_requests(count, rate, seed=5)


def test_every_request_answered_once_with_its_own_result():
    clock = FakeClock()
    ex = TimingExecutor(clock)
    srv = serve.Server(ex, mem_budget=10 ** 9, max_batch=16)
    reqs = _requests()
    res = srv.run(reqs, clock=clock)
    assert [r.rid for r in res] == sorted(q.rid for q in reqs)
    assert all(r.energy == r.rid for r in res)
    assert all(r.done >= r.arrival for r in res)


def test_batches_are_single_class_fifo_and_bounded():
    clock = FakeClock()
    ex = TimingExecutor(clock)
    srv = serve.Server(ex, mem_budget=10 ** 9, max_batch=8)
    reqs = _requests()
    by_id = {r.rid: r for r in reqs}
    srv.run(reqs, clock=clock)
    assert any(len(ids) > 1 for _, ids, _ in ex.launched), "requests must be batched"
    order = collections.defaultdict(list)
    for key, ids, _ in ex.launched:
        assert len(ids) <= 8
        assert len({(by_id[i].n, by_id[i].circuit.shape_key(), by_id[i].want_grad) for i in ids}) == 1
        order[key].extend(ids)
    for key, ids in order.items():
        arr = [by_id[i].arrival for i in ids]
        assert arr == sorted(arr), "FIFO inside a class"


def test_memory_cap_limits_concurrency_and_still_finishes():
    clock = FakeClock()
    ex = TimingExecutor(clock, per_req_bytes=100)
    srv = serve.Server(ex, mem_budget=250, max_batch=64)
    reqs = _requests(120)
    res = srv.run(reqs, clock=clock)
    assert len(res) == 120
    assert ex.peak <= 250
    assert max(len(ids) for _, ids, _ in ex.launched) <= 2
    assert srv.stats["memory_waits"] > 0


def test_request_larger_than_budget_is_rejected():
    clock = FakeClock()
    ex = TimingExecutor(clock, per_req_bytes=1000)
    srv = serve.Server(ex, mem_budget=500)
    with pytest.raises(MemoryError):
        srv.run(_requests(3), clock=clock)


def test_classes_overlap_in_flight():
    clock = FakeClock()
    ex = TimingExecutor(clock, duration=0.05)
    srv = serve.Server(ex, mem_budget=10 ** 9, max_batch=4, max_inflight_per_class=2)
    srv.run(_requests(200, rate=5000.0), clock=clock)
    assert srv.stats["peak_inflight"] >= 3


def test_latency_summary():
    res = [serve.Result(i, 4, False, 0.0, None, 0.0, 0.001 * (i + 1), 1) for i in range(100)]
    s = serve.latency_summary(res)
    assert s["requests"] == 100 and s["p50_ms"] <= s["p99_ms"]
