"""Request-loop logic on the CPU: a fake executor on a simulated clock
(admission by budget and slots, FIFO with bounded bypass, slot recycling,
latency bookkeeping), and an oracle-backed executor showing that every
request's result is the one it gets alone."""
import dataclasses
import math

import numpy as np
import pytest

from paper_1506_07207_amd import inputs as I
from paper_1506_07207_amd import serve as S


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor(S.Executor):
    """Budget- and slot-limited executor; a step costs a fixed overhead plus a
    cost per resident tracer (processor sharing on a simulated clock)."""

    def __init__(self, clock, budget, slots, per_tracer=1e-9, overhead=1e-4, run=None):
        self.clock, self.budget, self.slots = clock, budget, slots
        self.per_tracer, self.overhead = per_tracer, overhead
        self.live = {}
        self.next = 0
        self.admit_order = []
        self.max_used = 0
        self.run = run

    def used(self):
        return sum(r.spec.tracers for r, _ in self.live.values())

    def admit(self, req):
        if len(self.live) >= self.slots or self.used() + req.spec.tracers > self.budget:
            return None
        h = self.next
        self.next += 1
        self.live[h] = (req, req.spec.n_steps)
        self.admit_order.append(req.rid)
        self.max_used = max(self.max_used, self.used())
        return h

    def active(self):
        return len(self.live)

    def step(self, n):
        self.clock.t += n * (self.overhead + self.per_tracer * self.used())
        for h, (r, left) in list(self.live.items()):
            self.live[h] = (r, left - n)

    def poll(self):
        return [h for h, (r, left) in self.live.items() if left <= 0]

    def finish(self, h):
        r, _ = self.live.pop(h)
        return self.run(r) if self.run else {"W_E": 0.0, "flags": 0}


def _req(rid, t, tracers, steps, cells=64):
    spec = I.BatchSpec("landau", 0.5, 0.01, 1, tracers, cells, 0.1, steps)
    return I.Request(rid, t, spec, False)


def test_all_requests_complete_and_latency_is_bookkept():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=10_000, slots=4)
    reqs = [_req(i, 0.01 * i, 1000 + 100 * (i % 5), 50 + 10 * (i % 7)) for i in range(40)]
    rep = S.Server(ex, chunk_steps=8, clock=clk, sleep=clk.sleep).run(reqs)
    assert len(rep.completed()) == 40
    for r in rep.records:
        assert r.arrival <= r.admitted <= r.completed
        # a request needs at least its own steps (rounded up to whole chunks)
        assert r.latency >= math.ceil(r.steps / 8) * 8 * ex.overhead
    assert ex.max_used <= 10_000
    s = rep.summary()
    assert s["p50_s"] <= s["p99_s"] and s["tracer_updates_per_s"] > 0


def test_fifo_when_everything_fits():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=10 ** 9, slots=1000)
    reqs = [_req(i, 0.0, 100, 10) for i in range(20)]
    S.Server(ex, clock=clk, sleep=clk.sleep).run(reqs)
    assert ex.admit_order == list(range(20))


def test_small_requests_bypass_a_blocked_large_one_but_it_is_not_starved():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=1000, slots=100)
    reqs = [_req(0, 0.0, 600, 100)] + [_req(1, 0.0, 900, 10)] + [_req(i, 0.0, 50, 10) for i in range(2, 12)]
    rep = S.Server(ex, chunk_steps=5, bypass=8, max_passed=3, clock=clk, sleep=clk.sleep).run(reqs)
    order = ex.admit_order
    assert order[0] == 0
    assert order.index(1) > order.index(2)  # smaller ones went ahead of the blocked one
    passed_over_1 = [rid for rid in order[: order.index(1)] if rid > 1]
    assert len(passed_over_1) <= 3  # but only a bounded number of times
    assert len(rep.completed()) == len(reqs)


def test_request_larger_than_executor_is_reported():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=100, slots=4)
    with pytest.raises(RuntimeError):
        S.Server(ex, clock=clk, sleep=clk.sleep).run([_req(0, 0.0, 1000, 10)])


def test_idle_server_sleeps_until_next_arrival():
    clk = FakeClock()
    ex = FakeExecutor(clk, budget=10_000, slots=4)
    rep = S.Server(ex, chunk_steps=10, clock=clk, sleep=clk.sleep).run([_req(0, 5.0, 100, 10)])
    r = rep.records[0]
    assert r.admitted >= 5.0 and r.completed > r.admitted


def test_results_survive_scheduling_with_oracle_executor():
    """Tiny simulations advanced by the FP64 oracle behind the scheduler give
    exactly their stand-alone results, whatever the admission interleaving."""
    from oracle import oracle as O

    specs = [I.BatchSpec("landau" if i % 2 else "two_stream", 0.3 + 0.05 * i, 0.05, 4, 64 + 8 * i, 32, 0.1,
                         5 + 3 * i) for i in range(6)]

    def alone(spec):
        p = spec.build()
        return O.run_problem(p)["hist"][-1, 2]

    def run(req):
        return {"W_E": alone(req.spec), "flags": 0}

    clk = FakeClock()
    ex = FakeExecutor(clk, budget=1500, slots=3, run=run)
    reqs = [I.Request(i, 0.001 * i, s, False) for i, s in enumerate(specs)]
    rep = S.Server(ex, chunk_steps=4, clock=clk, sleep=clk.sleep).run(reqs)
    for r, s in zip(rep.records, specs):
        assert r.final_W_E == alone(s)


def test_poisson_stream_statistics():
    reqs = S.poisson_stream(4000, rate=100.0, seed=3, p_large=0.01)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(np.mean(gaps) - 0.01) < 0.001
    large = sum(r.large for r in reqs)
    assert 20 < large < 70
    assert all(r.spec.n_cells == 4096 for r in reqs if r.large)
