"""The serving scheduler (host logic) with a stand-in engine and a virtual clock.

Checks admission by footprint and slots (first come first served), closed-loop
iterations, and the latency/throughput bookkeeping.  The GPU engine is tested
in test_gpu_serving.py.
"""
import math

import numpy as np
import pytest

from paper_2008_13490_amd import serving as SV


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeEngine:
    """An evaluation round costs a fixed time plus time per sequence."""

    def __init__(self, clock, per_round=1e-3, per_seq=1e-7):
        self.clock, self.per_round, self.per_seq = clock, per_round, per_seq
        self.loaded = set()
        self.max_loaded = 0
        self.order = []

    def estimate(self, j):
        return j.S * 100

    def load(self, j):
        assert j.rid not in self.loaded
        self.loaded.add(j.rid)
        self.order.append(j.rid)
        self.max_loaded = max(self.max_loaded, len(self.loaded))

    def footprint(self, j):
        return j.S * 100

    def work(self, j):
        return float(j.S)

    def unload(self, j):
        self.loaded.remove(j.rid)

    def evaluate(self, active, keep=False):
        for j in active:
            assert j.rid in self.loaded
        self.clock.t += self.per_round + self.per_seq * sum(j.S for j in active)
        return [(j.rid, j.k) for j in active]


def _jobs(n, rate, seed=1, n_iter=5):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    S = rng.integers(1000, 100000, size=n)
    return [SV.Job(rid=x, arrival=float(t[x]), kind="2q", S=int(S[x]), data=None, n_iter=n_iter) for x in range(n)]


@pytest.mark.parametrize("max_active,budget", [(1, 10 ** 12), (8, 10 ** 12), (64, 3 * 10 ** 7)])
def test_scheduler_admission_and_iterations(max_active, budget):
    clk = Clock()
    eng = FakeEngine(clk)
    jobs = _jobs(60, rate=200.0)
    sch = SV.Scheduler(eng, budget, max_active, keep_results=True, clock=clk, sleep=clk.sleep)
    out = sch.run(jobs)
    assert out["requests"] == 60 and out["iterations"] == 60 * 5
    assert eng.max_loaded <= max_active
    assert sch.max_used <= budget
    assert not eng.loaded                                   # everything unloaded
    assert eng.order == sorted(eng.order)                   # first come first served
    for j in jobs:
        assert [r for r in j.results] == [(j.rid, k) for k in range(5)]   # closed loop, in order
        assert j.arrival <= j.t_admit <= j.t_iter[0] <= j.t_done
        assert all(b > a for a, b in zip(j.t_iter, j.t_iter[1:]))
    assert out["request_latency_ms"]["p99"] >= out["request_latency_ms"]["p50"] > 0


def test_batching_beats_a_queue_under_load():
    """At a rate where one-at-a-time service queues up, rounds over all admitted
    requests give lower latency and higher throughput (fixed cost per round)."""
    res = {}
    for name, slots in (("queue", 1), ("batched", 64)):
        clk = Clock()
        eng = FakeEngine(clk, per_round=2e-3, per_seq=2e-8)
        jobs = _jobs(200, rate=500.0, seed=3)
        res[name] = SV.Scheduler(eng, 10 ** 13, slots, clock=clk, sleep=clk.sleep).run(jobs)
    assert res["batched"]["request_latency_ms"]["p99"] < res["queue"]["request_latency_ms"]["p99"]
    assert res["batched"]["seq_evals_per_s"] > res["queue"]["seq_evals_per_s"]


def test_oversized_request_is_refused():
    clk = Clock()
    eng = FakeEngine(clk)
    jobs = _jobs(3, rate=10.0)
    with pytest.raises(RuntimeError):
        SV.Scheduler(eng, 1000, 4, clock=clk, sleep=clk.sleep).run(jobs)


def test_footprint_estimate_grows_with_size():
    a = SV.footprint_estimate(2, 6, 4, 1000, 100000)
    b = SV.footprint_estimate(2, 6, 4, 2000, 200000)
    c = SV.footprint_estimate(3, 5, 8, 1000, 100000)
    assert 0 < a < b and c > 100000 * 1024


def test_round_work_bound_keeps_small_requests_moving():
    """With a bound on the work of a round, a small request admitted next to
    large ones is served in short rounds and finishes first."""
    clk = Clock()
    eng = FakeEngine(clk, per_round=1e-4, per_seq=1e-7)
    big = [SV.Job(rid=x, arrival=0.0, kind="2q", S=100000, data=None, n_iter=5) for x in range(3)]
    small = SV.Job(rid=3, arrival=0.0, kind="1q", S=1000, data=None, n_iter=5)
    sch = SV.Scheduler(eng, 10 ** 13, 8, clock=clk, sleep=clk.sleep, round_work=100000)
    sch.run(big + [small])
    assert small.t_done <= min(j.t_done for j in big)      # rides along with the first large one
    assert small.t_done < sorted(j.t_done for j in big)[1]
    assert sch.round_sizes[:5] == [2] * 5 and max(sch.round_sizes) <= 2


class FakeAsyncEngine(FakeEngine):
    """A device timeline behind submit/finish: a round costs the host
    `host_round` when it is submitted and the device `per_round + per_seq * S`
    once the device is free; finish waits until the round has ended."""

    def __init__(self, clock, host_round=1e-3, **kw):
        super().__init__(clock, **kw)
        self.host_round = host_round
        self.free_at = 0.0
        self.inflight = set()

    def submit(self, active, keep=False):
        for j in active:
            assert j.rid in self.loaded and j.rid not in self.inflight   # one round at a time per request
            self.inflight.add(j.rid)
        self.clock.t += self.host_round
        start = max(self.clock.t, self.free_at)
        self.free_at = start + self.per_round + self.per_seq * sum(j.S for j in active)
        return (self.free_at, [(j.rid, j.k) for j in active], [j.rid for j in active])

    def finish(self, token):
        end, res, rids = token
        self.clock.t = max(self.clock.t, end)
        for r in rids:
            self.inflight.remove(r)
        return res

    def evaluate(self, active, keep=False):
        return self.finish(self.submit(active, keep))


@pytest.mark.parametrize("prefetch", [False, True])
def test_pipelined_rounds_keep_the_loop_closed_and_hide_host_time(prefetch):
    """Two rounds in flight: every request still sees its iterations in order,
    one round at a time, and the device no longer waits for the host between
    rounds, so the same trace finishes sooner than with one round in flight."""
    res = {}
    for depth in (1, 2):
        clk = Clock()
        eng = FakeAsyncEngine(clk, host_round=2e-3, per_round=2e-4, per_seq=1e-8)
        jobs = _jobs(80, rate=2000.0, seed=5)
        sch = SV.Scheduler(eng, 10 ** 13, 16, keep_results=True, clock=clk, sleep=clk.sleep, depth=depth,
                           prefetch=prefetch)
        out = sch.run(jobs)
        assert out["iterations"] == 80 * 5 and not eng.loaded and not eng.inflight
        for j in jobs:
            assert j.results == [(j.rid, k) for k in range(5)]
            assert j.arrival <= j.t_admit <= j.t_iter[0] <= j.t_done
        res[depth] = out
    if not prefetch:   # (with loads on a thread the virtual timeline depends on thread timing)
        assert res[2]["wall_s"] < res[1]["wall_s"]
        assert res[2]["seq_evals_per_s"] > res[1]["seq_evals_per_s"]


def test_prefetch_respects_budget_and_order():
    clk = Clock()
    eng = FakeAsyncEngine(clk)
    jobs = _jobs(50, rate=300.0, seed=6)
    budget = 3 * 10 ** 7
    sch = SV.Scheduler(eng, budget, 64, clock=clk, sleep=clk.sleep, depth=2, prefetch=True)
    out = sch.run(jobs)
    assert out["requests"] == 50 and sch.max_used <= budget
    assert eng.order == sorted(eng.order)


def test_depth_needs_submit():
    clk = Clock()
    with pytest.raises(ValueError):
        SV.Scheduler(FakeEngine(clk), 10 ** 9, 4, depth=2)
