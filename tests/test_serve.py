"""Shot scheduler on the host: admission, ordering, overlap and failures.

A fake backend on a virtual clock stands in for the GPU: each shot costs
npts * nt * cost seconds of device time, shots run concurrently, and time
only moves when the scheduler sleeps, so every run is deterministic.
"""
import numpy as np
import pytest

from paper_2404_04441_amd.serve import ShotRequest, ShotServer, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    def __init__(self, clock, cost=1e-9, bytes_per_pt=12):
        self.clock = clock
        self.cost = cost
        self.bpp = bytes_per_pt
        self.live = {}
        self.peak_bytes = 0
        self.started = []
        self.released = []

    def footprint(self, req):
        if req.nt <= 0:
            raise ValueError("nt must be positive")
        return req.npts * self.bpp

    def start(self, req):
        if req.storage == "bad":
            raise RuntimeError("wave_create: invalid argument")
        h = {"req": req, "busy_until": self.clock(), "steps": 0}
        self.live[req.id] = req.npts * self.bpp
        self.peak_bytes = max(self.peak_bytes, sum(self.live.values()))
        self.started.append((req.id, self.clock()))
        return h

    def advance(self, h, n):
        start = max(self.clock(), h["busy_until"])
        h["busy_until"] = start + n * h["req"].npts * self.cost
        h["steps"] += n
        return h["busy_until"]

    def chunk_done(self, h, token):
        return self.clock() >= token

    def result(self, h):
        req = h["req"]
        return np.full((h["steps"], 1), float(req.id))

    def release(self, h):
        self.released.append(h["req"].id)
        del self.live[h["req"].id]


def req(i, arrival, n=32, nt=100, storage="f32"):
    return ShotRequest(id=i, arrival=arrival, shape=(n, n, n), nt=nt, storage=storage, h=10.0, dt=1e-3,
                       src=(n // 2, n // 2, 4), rec=np.zeros((1, 3), np.int32))


def run(server, reqs, clock, cancel=None):
    res = server.run(reqs, clock=clock, sleep=clock.sleep, cancel=cancel)
    return res


def test_all_shots_complete_and_results_are_their_own():
    clock = Clock()
    be = FakeBackend(clock)
    reqs = [req(i, 0.001 * i, n=16 + 8 * (i % 3), nt=50 + 10 * i) for i in range(12)]
    res = run(ShotServer(be, budget_bytes=1 << 40, max_slots=4, chunk_steps=30), reqs, clock)
    assert sorted(res) == list(range(12))
    for r in reqs:
        out = res[r.id]
        assert out.status == "done" and out.traces.shape == (r.nt, 1) and np.all(out.traces == r.id)
        assert out.finished >= out.admitted >= out.arrival
    assert sorted(be.released) == list(range(12)) and not be.live


def test_memory_budget_bounds_concurrency_and_keeps_fifo():
    clock = Clock()
    be = FakeBackend(clock)
    reqs = [req(i, 0.0, n=32) for i in range(6)]
    one = 32 ** 3 * 12
    server = ShotServer(be, budget_bytes=2 * one + 10, max_slots=8, chunk_steps=25)
    res = run(server, reqs, clock)
    assert be.peak_bytes <= 2 * one + 10
    assert server.max_concurrent == 2
    order = [i for i, _ in be.started]
    assert order == sorted(order)  # admitted in arrival order
    assert all(r.status == "done" for r in res.values())


def test_slot_limit():
    clock = Clock()
    be = FakeBackend(clock)
    server = ShotServer(be, budget_bytes=1 << 40, max_slots=3, chunk_steps=10)
    run(server, [req(i, 0.0) for i in range(9)], clock)
    assert server.max_concurrent == 3


def test_continuous_batching_admits_late_arrivals_while_others_run():
    """A shot that arrives while a long shot runs starts before that shot ends."""
    clock = Clock()
    be = FakeBackend(clock, cost=1e-8)
    long = req(0, 0.0, n=64, nt=400)
    late = req(1, 0.05, n=16, nt=20)
    res = run(ShotServer(be, budget_bytes=1 << 40, max_slots=4, chunk_steps=50), [long, late], clock)
    assert res[1].admitted < res[0].finished
    assert res[1].finished < res[0].finished  # the small late shot overtakes


def test_oversized_and_invalid_requests_do_not_block_the_queue():
    clock = Clock()
    be = FakeBackend(clock)
    reqs = [req(0, 0.0, n=16), req(1, 0.0, n=128), req(2, 0.0, n=16, nt=0), req(3, 0.0, n=16, storage="bad"),
            req(4, 0.0, n=16)]
    res = run(ShotServer(be, budget_bytes=64 ** 3 * 12, max_slots=4, chunk_steps=20), reqs, clock)
    assert res[0].status == "done" and res[4].status == "done"
    assert res[1].status == "rejected" and "budget" in res[1].error
    assert res[2].status == "rejected"
    assert res[3].status == "failed" and "invalid" in res[3].error
    assert not be.live


def test_cancellation_mid_run_frees_the_slot():
    clock = Clock()
    be = FakeBackend(clock, cost=1e-8)
    one = 32 ** 3 * 12
    reqs = [req(0, 0.0, nt=2000), req(1, 0.0, nt=50), req(2, 0.0, nt=50)]
    cancel = set()
    base_sleep = clock.sleep

    def sleep(dt):  # the client cancels shot 0 once it has run for 5 ms
        base_sleep(dt)
        if clock.t > 0.005:
            cancel.add(0)

    server = ShotServer(be, budget_bytes=one + 1, max_slots=4, chunk_steps=100)
    res = server.run(reqs, clock=clock, sleep=sleep, cancel=cancel)
    assert res[0].status == "failed" and res[0].error == "cancelled"
    assert res[0].admitted == 0.0
    # retired once its queued chunks drained, long before 2000 steps of work
    assert res[0].finished < 0.2 * 2000 * 32 ** 3 * 1e-8
    assert res[1].status == "done" and res[2].status == "done"
    assert res[1].admitted >= res[0].finished  # the memory it held went to the next shot
    assert not be.live


def test_cancellation_before_admission():
    clock = Clock()
    be = FakeBackend(clock)
    res = run(ShotServer(be, budget_bytes=1 << 40, max_slots=1, chunk_steps=10),
              [req(0, 0.0), req(1, 0.0)], clock, cancel={1})
    assert res[0].status == "done" and res[1].status == "failed" and res[1].error == "cancelled"
    assert [i for i, _ in be.started] == [0]


def test_summary_percentiles():
    clock = Clock()
    be = FakeBackend(clock)
    reqs = [req(i, 0.002 * i) for i in range(20)]
    server = ShotServer(be, budget_bytes=1 << 40, max_slots=2, chunk_steps=40)
    res = run(server, reqs, clock)
    s = summarize(res, reqs, server.elapsed)
    lat = sorted(r.latency for r in res.values())
    assert s["done"] == 20 and s["failed"] == 0 and s["rejected"] == 0
    assert s["p50_latency_s"] == pytest.approx(np.percentile(lat, 50), abs=1e-4)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert s["shots_per_s"] == pytest.approx(20 / server.elapsed, rel=1e-3)


def test_burst_of_arrivals():
    clock = Clock()
    be = FakeBackend(clock)
    reqs = [req(i, 0.0, n=16 + (i % 5) * 4, nt=20 + i) for i in range(200)]
    server = ShotServer(be, budget_bytes=40 * 32 ** 3 * 12, max_slots=16, chunk_steps=16)
    res = run(server, reqs, clock)
    assert all(r.status == "done" for r in res.values()) and len(res) == 200
    assert server.max_concurrent == 16
