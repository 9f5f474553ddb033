"""Serving scheduler on the CPU with a fake backend: simulated clock, memory budget,
launch durations and injected launch errors."""
import time

import pytest

from paper_2604_21984_amd.serve import QUERY, RENDER, Request, Server, run_open_loop


class Clock:
    def __init__(self):
        self.t = 0.0


class FakeSet:
    def __init__(self, set_id, H=8, W=8, K=8):
        self.set_id, self.H, self.W, self.K, self.n_slots = set_id, H, W, K, 4


class FakeBackend:
    def __init__(self, clock, free=1 << 30, per_launch=1e-3, per_point=1e-6, per_px=1e-7,
                 fail_sets=()):
        self.clock, self.free = clock, free
        self.per_launch, self.per_point, self.per_px = per_launch, per_point, per_px
        self.fail_sets = set(fail_sets)
        self.launched = []

    def now(self):
        return self.clock.t

    def free_bytes(self):
        return self.free

    def launch_queries(self, reqs, sets):
        if any(r.set_id in self.fail_sets for r in reqs):
            raise RuntimeError("injected kernel error")
        dur = self.per_launch + self.per_point * sum(r.M for r in reqs)
        self.launched.append([r.rid for r in reqs])
        return {"t_end": self.clock.t + dur, "reqs": reqs,
                "outs": [("q", r.set_id, r.rid) for r in reqs]}

    def launch_render(self, req, rset):
        if req.set_id in self.fail_sets:
            raise RuntimeError("injected kernel error")
        self.launched.append([req.rid])
        return {"t_end": self.clock.t + self.per_launch + self.per_px * rset.H * rset.W,
                "reqs": [req], "outs": [("r", req.set_id, req.rid)]}

    def done(self, h):
        return self.clock.t >= h["t_end"]

    def results(self, h):
        return list(zip(h["reqs"], h["outs"]))


def _run(server, clock, dt=1e-4, limit=100000):
    n = 0
    while server.step():
        clock.t += dt
        n += 1
        assert n < limit


def _q(rid, set_id, M, t=0.0):
    return Request(rid, set_id, QUERY, xy=None, M=M, t_arrival=t)


def test_admission_never_exceeds_budget_and_all_complete():
    clock = Clock()
    be = FakeBackend(clock)
    sets = [FakeSet(0), FakeSet(1)]
    srv = Server(be, sets, mem_budget=1000, max_inflight=8)
    for i in range(20):
        srv.submit(_q(i, i % 2, 20))      # 400 bytes each: at most two admitted at a time
    _run(srv, clock)
    assert srv.peak_reserved <= 1000
    assert len(srv.completed) == 20 and all(r.error is None for r in srv.completed)
    assert srv.reserved == 0
    assert max(len(b) for b in be.launched) == 2


def test_oversized_and_unknown_requests_are_rejected():
    clock = Clock()
    srv = Server(FakeBackend(clock), [FakeSet(0)], mem_budget=500)
    srv.submit(_q(0, 0, 100))              # 2000 bytes > budget
    srv.submit(_q(1, 7, 1))                # unknown set
    srv.submit(_q(2, 0, 5))
    _run(srv, clock)
    err = {r.rid: r.error for r in srv.completed}
    assert "budget" in err[0] and "unknown set" in err[1] and err[2] is None


def test_continuous_batching_across_sets_and_overlap():
    clock = Clock()
    be = FakeBackend(clock, per_launch=5e-3)
    srv = Server(be, [FakeSet(i) for i in range(3)], mem_budget=1 << 20)
    for i in range(5):
        srv.submit(_q(i, i % 3, 10))
    srv.step()                             # one launch: five requests over three sets
    assert be.launched == [[0, 1, 2, 3, 4]]
    assert srv.launches[0][1:] == (5, 3)
    clock.t += 1e-3
    for i in range(5, 8):                  # arrive while the first launch runs
        srv.submit(_q(i, i % 3, 10, t=clock.t))
    srv.step()
    assert be.launched[1] == [5, 6, 7]      # admitted and launched before the first ends
    assert len(srv.inflight) == 2
    _run(srv, clock)
    assert len(srv.completed) == 8


def test_failing_set_fails_only_its_requests():
    clock = Clock()
    be = FakeBackend(clock, fail_sets={1})
    srv = Server(be, [FakeSet(i) for i in range(3)], mem_budget=1 << 20)
    for i in range(9):
        srv.submit(_q(i, i % 3, 4))
    srv.submit(Request(9, 1, RENDER))
    srv.submit(Request(10, 2, RENDER))
    _run(srv, clock)
    bad = sorted(r.rid for r in srv.completed if r.error)
    good = sorted(r.rid for r in srv.completed if r.error is None)
    assert bad == [1, 4, 7, 9]
    assert good == [0, 2, 3, 5, 6, 8, 10]
    assert srv.reserved == 0


def test_max_inflight_and_renders_launch_alone():
    clock = Clock()
    be = FakeBackend(clock, per_launch=1.0)
    srv = Server(be, [FakeSet(0, 16, 16)], mem_budget=1 << 20, max_inflight=2)
    for i in range(4):
        srv.submit(Request(i, 0, RENDER))
    srv.step()
    assert len(srv.inflight) == 2 and len(be.launched) == 2
    _run(srv, clock, dt=0.25)
    assert len(srv.completed) == 4


def test_latency_percentiles():
    clock = Clock()
    srv = Server(FakeBackend(clock), [FakeSet(0)], mem_budget=1 << 20)
    for i in range(100):
        r = _q(i, 0, 1)
        r.t_arrival, r.t_done = 0.0, (i + 1) * 1e-3
        srv.completed.append(r)
    st = srv.stats()
    assert st["p50_ms"] == pytest.approx(50.0) and st["p99_ms"] == pytest.approx(99.0)


def test_result_callback_replaces_retention():
    """With on_result the outputs go to the callback and are not kept on the requests
    (a load generator keeps its requests for the statistics, not their outputs)."""
    clock = Clock()
    got = []
    srv = Server(FakeBackend(clock), [FakeSet(0)], mem_budget=1 << 20,
                 on_result=lambda r, out: got.append((r.rid, out)))
    for i in range(4):
        srv.submit(_q(i, 0, 10))
    srv.submit(Request(4, 0, RENDER, t_arrival=0.0))
    _run(srv, clock)
    assert sorted(rid for rid, _ in got) == [0, 1, 2, 3, 4]
    assert all(r.result is None and r.error is None for r in srv.completed)
    assert dict(got)[4] == ("r", 0, 4)


class WallBackend(FakeBackend):
    """The fake backend on the wall clock: every launch takes `per_launch` seconds."""

    def __init__(self, per_launch=2e-4):
        super().__init__(None, per_launch=per_launch)

    def now(self):
        return time.perf_counter()

    def launch_queries(self, reqs, sets):
        self.launched.append([r.rid for r in reqs])
        return {"t_end": time.perf_counter() + self.per_launch, "reqs": reqs,
                "outs": [None] * len(reqs)}

    def launch_render(self, req, rset):
        return self.launch_queries([req], None)

    def done(self, h):
        return time.perf_counter() >= h["t_end"]


def test_open_loop_arrivals_are_scheduled_times():
    """The open-loop driver stamps each request with its scheduled arrival (start +
    times[i], in any submission order) and counts latency from there."""
    be = WallBackend()
    srv = Server(be, [FakeSet(0)], mem_budget=1 << 20, on_result=lambda r, out: None)
    times = [0.004, 0.0, 0.002, 0.006]
    reqs = [_q(i, 0, 10) for i in range(4)]
    t0 = time.perf_counter()
    run_open_loop(srv, reqs, times, timeout=10.0)
    starts = [r.t_arrival - times[i] for i, r in enumerate(reqs)]
    assert max(starts) - min(starts) < 1e-9 and starts[0] >= t0
    assert all(r.t_done >= r.t_arrival + be.per_launch for r in reqs)
    assert all(r.latency < 1.0 and r.error is None for r in reqs)
    assert sorted(sum(be.launched, [])) == [0, 1, 2, 3]
