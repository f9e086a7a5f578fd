"""Continuous-batching service for fit evaluations on one GPU.

A fit request brings its sequence list, its counts and the gate sets of its
optimizer iterations; each iteration is one evaluation of the negative
log-likelihood and its gradient (the thesis fits gate sets to counts by
maximum likelihood, Sec. 6.3.2).  The service keeps every admitted request
resident on the device (sequences, counts, sharing plan, partial-sum
buffers) and evaluates all admitted requests together, one iteration each,
in one batched round.  Requests that arrive while a round runs join the next
round once the HBM budget and the slots allow it (admission by footprint,
first come first served, no overtaking); a request leaves after its last
iteration.  Iterations are closed loop: iteration k + 1 of a request is
evaluated only after result k is back.

Engines
  GPUEngine    the library's batches (gst_batch): per round one persistent
               launch for the plain one- and two-qubit lists, one launch per
               kernel and level for all shared-prefix plans, and the
               three-qubit launch sequences; a round replays a HIP graph
               while its composition does not change; rounds can be enqueued
               while the previous one runs.
  PlainEngine  the plain per-request path: one request at a time, each
               iteration its own evaluation (gst_req_eval), a queue alone.

The scheduler itself is host logic and does not depend on the engine.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from types import SimpleNamespace
from typing import Any, Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    rid: int
    arrival: float              # seconds after the start of the trace
    kind: str                   # "1q", "2q", "3q"
    S: int
    data: Any                   # workloads.FitRequestData
    n_iter: int
    footprint: int = 0
    k: int = 0                  # iterations done
    t_admit: float = math.nan
    t_done: float = math.nan
    t_iter: List[float] = dataclasses.field(default_factory=list)
    results: List[Any] = dataclasses.field(default_factory=list)
    handle: Any = None          # engine state while admitted


def tile_seqs(S: int) -> int:
    """Sequences per tile of the one- and two-qubit tile kernel (as the library cuts them)."""
    per = (S + 16 * 1024 - 1) // (16 * 1024)
    return 16 * min(max(per, 1), 8)


def footprint_estimate(n_qubits: int, K: int, M: int, S: int, sum_len: int) -> int:
    """Device bytes a request will hold (inputs, tile partials, three-qubit
    step records and positions); used to admit before allocating."""
    D = 4 ** n_qubits
    b = 8 * (S + 1) + sum_len + 4 * S * M + 8 * (S + 1) + 4096
    if D == 64:
        n_tiles = (S + 15) // 16
        b += n_tiles * (1 + 64 + 64 * M) * 8 + 8 * sum_len + (sum_len // 8192 + K + 1) * 4096 * 8
        b += sum_len * 64 * 8 * 2           # per-step records of one evaluation
    else:
        n_tiles = (S + tile_seqs(S) - 1) // tile_seqs(S)
        b += n_tiles * (1 + D + M * D + K * D * D) * 8 + n_tiles * 24
    return int(b)


def step_cost(n_qubits: int) -> float:
    """Relative device time of one step of one sequence (with gradient), two
    qubits = 1: the one- and two-qubit tile kernel runs both at the same
    rate; a three-qubit step (64x64 products, per-step records and the MFMA
    gate gradient) costs about 14 two-qubit steps."""
    return 14.0 if n_qubits == 3 else 1.0


class Scheduler:
    """Admission and rounds.  ``clock`` returns seconds; ``sleep`` waits.

    Admission is first come first served by footprint and slots.  A round
    takes the admitted requests that are loaded and not in a round already,
    oldest first, while the round stays within ``round_work`` (two-qubit
    sequence steps; the oldest is always taken), so a round of many small
    requests is not held up by a large one beyond that bound.

    ``depth`` rounds may be in flight at once (engines with submit/finish):
    the ready requests are split over the free round slots (a round takes
    about its share of their work), and while the device runs one round the
    host gathers the results of the previous one and enqueues the next, so
    the device does not wait on the host between rounds.  A request is in at most one round at a time
    (iteration k + 1 starts after result k is back).  With ``prefetch`` the
    admitted requests are loaded (host plan, uploads) and unloaded on a
    background thread while rounds run."""

    def __init__(self, engine, budget_bytes: int, max_active: int, keep_results: bool = False,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 round_work: float = math.inf, depth: int = 1, prefetch: bool = False):
        self.engine = engine
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.round_work = float(round_work)
        self.depth = max(1, int(depth))
        if self.depth > 1 and not hasattr(engine, "submit"):
            raise ValueError("depth > 1 needs an engine with submit/finish")
        self.prefetch = prefetch
        self.keep = keep_results
        self.clock = clock
        self.sleep = sleep
        self.max_used = 0
        self.rounds = 0
        self.round_sizes: List[int] = []
        self.host_s = collections.Counter()   # host time by phase: load, submit, wait

    def _choose(self, ready: List[Job], free_slots: int = 1) -> List[Job]:
        order = sorted(ready, key=lambda x: x.rid)
        head = order[0]
        work = self.engine.work(head)
        cap = max(self.round_work, work + 0.25 * self.round_work)
        if free_slots > 1:   # leave work for the other rounds that can be in flight
            cap = min(cap, max(work, sum(self.engine.work(j) for j in order) / free_slots))
        chosen = [head]
        for j in sorted(order[1:], key=lambda x: (self.engine.work(x), x.rid)):
            w = self.engine.work(j)
            if work + w > cap:
                break
            chosen.append(j)
            work += w
        return sorted(chosen, key=lambda x: x.rid)

    def run(self, jobs: Sequence[Job]) -> dict:
        import concurrent.futures as cf
        jobs = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        pool = cf.ThreadPoolExecutor(max_workers=1) if self.prefetch else None
        pending: collections.deque = collections.deque()
        loading: List[Any] = []           # (job, future)
        unloading: List[Any] = []         # (job, future)
        ready: List[Job] = []             # loaded, not in a round
        inflight: collections.deque = collections.deque()   # (token, chosen)
        n_admitted = 0
        used = 0
        t0 = self.clock()
        i = 0
        n_done = 0
        try:
            while n_done < len(jobs):
                now = self.clock() - t0
                while i < len(jobs) and jobs[i].arrival <= now:
                    pending.append(jobs[i])
                    i += 1
                # requests that left: their memory is free once the unload ended
                for ent in [e for e in unloading if e[1].done()]:
                    ent[1].result()
                    used -= ent[0].footprint
                    unloading.remove(ent)
                # admission: first come first served, stop at the first that does not fit
                while pending and n_admitted < self.max_active:
                    j = pending[0]
                    est = self.engine.estimate(j)
                    if used + est > self.budget and (n_admitted or unloading or est > self.budget):
                        if not n_admitted and not unloading:
                            raise RuntimeError(f"request {j.rid} needs {est} bytes, over the budget {self.budget}")
                        break
                    pending.popleft()
                    j.footprint = est
                    used += est
                    n_admitted += 1
                    j.t_admit = self.clock() - t0
                    if pool is not None:
                        loading.append((j, pool.submit(self.engine.load, j)))
                    else:
                        h0 = self.clock()
                        self.engine.load(j)
                        self.host_s["load"] += self.clock() - h0
                        self._loaded(j)
                        used += j.footprint - est
                        ready.append(j)
                    self.max_used = max(self.max_used, used)
                for ent in [e for e in loading if e[1].done()]:
                    ent[1].result()
                    j = ent[0]
                    est = j.footprint
                    self._loaded(j)
                    used += j.footprint - est
                    self.max_used = max(self.max_used, used)
                    loading.remove(ent)
                    ready.append(j)
                if ready and len(inflight) < self.depth:
                    chosen = self._choose(ready, self.depth - len(inflight))
                    ready = [j for j in ready if j not in chosen]
                    h0 = self.clock()
                    if self.depth > 1:
                        inflight.append((self.engine.submit(chosen, self.keep), chosen))
                    else:
                        inflight.append((None, chosen, self.engine.evaluate(chosen, self.keep)))
                    self.host_s["submit"] += self.clock() - h0
                    self.rounds += 1
                    self.round_sizes.append(len(chosen))
                    continue
                if inflight:
                    ent = inflight.popleft()
                    h0 = self.clock()
                    res = ent[2] if len(ent) == 3 else self.engine.finish(ent[0])
                    self.host_s["wait"] += self.clock() - h0
                    chosen = ent[1]
                    tnow = self.clock() - t0
                    for j, r in zip(chosen, res):
                        j.t_iter.append(tnow)
                        j.k += 1
                        if self.keep:
                            j.results.append(r)
                    for j in chosen:
                        if j.k >= j.n_iter:
                            j.t_done = tnow
                            n_done += 1
                            n_admitted -= 1
                            if pool is not None:
                                unloading.append((j, pool.submit(self.engine.unload, j)))
                            else:
                                self.engine.unload(j)
                                used -= j.footprint
                        else:
                            ready.append(j)
                    continue
                # nothing to run: wait for a load, or for the next arrival
                if loading:
                    cf.wait([f for _, f in loading] + [f for _, f in unloading], timeout=1e-3,
                            return_when=cf.FIRST_COMPLETED)
                elif unloading and pending:
                    cf.wait([f for _, f in unloading], timeout=1e-3, return_when=cf.FIRST_COMPLETED)
                elif i < len(jobs):
                    wait = jobs[i].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
            for ent in unloading:
                ent[1].result()
                used -= ent[0].footprint
        finally:
            if pool is not None:
                pool.shutdown(wait=True)
        return summarize(jobs, self)

    def _loaded(self, j: Job):
        j.footprint = max(j.footprint, self.engine.footprint(j))


def _pct(x, q):
    return float(np.percentile(np.asarray(x, dtype=np.float64), q)) if len(x) else math.nan


def summarize(jobs: Sequence[Job], sched: Optional[Scheduler] = None) -> dict:
    lat = [j.t_done - j.arrival for j in jobs]
    wait = [j.t_admit - j.arrival for j in jobs]
    it = []
    for j in jobs:
        prev = j.t_admit
        for t in j.t_iter:
            it.append(t - prev)
            prev = t
    t_end = max(j.t_done for j in jobs)
    t_first = min(j.arrival for j in jobs)
    seq_evals = sum(j.S * j.n_iter for j in jobs)
    out = {
        "requests": len(jobs),
        "iterations": int(sum(len(j.t_iter) for j in jobs)),
        "wall_s": t_end - t_first,
        "seq_evals_per_s": seq_evals / max(t_end - t_first, 1e-12),
        "request_latency_ms": {"p50": _pct(lat, 50) * 1e3, "p99": _pct(lat, 99) * 1e3},
        "iteration_latency_ms": {"p50": _pct(it, 50) * 1e3, "p99": _pct(it, 99) * 1e3},
        "admission_wait_ms": {"p50": _pct(wait, 50) * 1e3, "p99": _pct(wait, 99) * 1e3},
    }
    if sched is not None:
        out["host_s"] = {k: round(v, 4) for k, v in sorted(sched.host_s.items())}
        out["rounds"] = sched.rounds
        out["mean_round_size"] = float(np.mean(sched.round_sizes)) if sched.round_sizes else 0.0
        out["max_bytes_admitted"] = sched.max_used
    return out


# ---------------------------------------------------------------------------
# engines on the library
# ---------------------------------------------------------------------------
class _LibEngine:
    def __init__(self, ctx):
        import torch
        from . import api
        self.api = api
        self.torch = torch
        self.ctx = ctx

    def estimate(self, j: Job) -> int:
        d = j.data
        g = d.iterates[0]
        return footprint_estimate(g.n_qubits, g.K, g.M, d.seqs.S, int(d.seqs.offsets[-1]))

    def work(self, j: Job) -> float:
        return step_cost(j.data.iterates[0].n_qubits) * float(j.data.seqs.offsets[-1])

    def load(self, j: Job):
        """Resident copies of a request (may run on another host thread: the
        uploads go through that thread's default stream, which is drained
        before the request is handed over)."""
        api, torch = self.api, self.torch
        d = j.data
        g0 = d.iterates[0]
        req = api.Request(self.ctx, g0.n_qubits, g0.K, g0.M, d.seqs.offsets, d.seqs.gates, d.counts)
        theta = api.DeviceGateSet.from_numpy(g0.n_qubits, g0.rho, g0.effects, g0.gates)
        its = torch.as_tensor(np.stack([g.gates for g in d.iterates]), device=theta.gates.device)
        torch.cuda.current_stream().synchronize()
        j.handle = SimpleNamespace(req=req, theta=theta, its=its)

    def footprint(self, j: Job) -> int:
        return j.handle.req.footprint()

    def unload(self, j: Job):
        j.handle.req.close()
        j.handle = None

    def _set_iterates(self, active):
        """Gate sets of the next iteration, copied on the context's stream."""
        dst = [j.handle.theta.gates for j in active]
        src = [j.handle.its[j.k] for j in active]
        with self.torch.cuda.stream(self.ctx.stream):
            if hasattr(self.torch, "_foreach_copy_"):
                self.torch._foreach_copy_(dst, src)
            else:
                for a, b in zip(dst, src):
                    a.copy_(b)


class GPUEngine(_LibEngine):
    """The chosen requests of a round in one batch (gst_batch): one persistent
    launch for the plain one- and two-qubit lists, one launch per kernel and
    level for the shared-prefix plans (one, two and three qubits), and the
    launch sequences of three-qubit lists without sharing, all on the
    context's stream.  Batches are kept per
    composition; a composition is captured into a HIP graph the second time
    it is used (a first use runs eagerly: capturing costs more than one eager
    round).

    submit() enqueues a round and returns at once; finish() waits for that
    round only (an event after it), so the next round can be enqueued while
    this one runs.  Run the context on a non-default stream so that uploads of
    requests loaded meanwhile do not wait for the rounds in flight; with loads
    on another thread, pass capture_graph=False: their uploads through the
    default stream invalidate a capture taken at the same time."""

    def __init__(self, ctx, capture_graph: bool = True, cache: int = 64):
        import threading
        super().__init__(ctx)
        self.capture = capture_graph
        self.cache_size = cache
        self.batches = collections.OrderedDict()   # composition -> [Batch, uses]
        self.builds = 0
        self.lock = threading.Lock()

    def unload(self, j: Job):
        with self.lock:
            drop = [self.batches.pop(k)[0] for k in [k for k in self.batches if j.rid in k]]
        for b in drop:
            b.close()
        super().unload(j)

    def _batch(self, active):
        key = tuple(j.rid for j in active)
        old = []
        with self.lock:
            ent = self.batches.get(key)
            if ent is not None:
                self.batches.move_to_end(key)
                ent[1] += 1
        if ent is None or (ent[1] == 2 and self.capture):
            if ent is not None:
                old.append(ent[0])
            b = self.api.Batch(self.ctx, [j.handle.req for j in active], [j.handle.theta for j in active],
                               want_probs=False, want_grad=True, capture_graph=ent is not None and self.capture)
            self.builds += 1
            ent = [b, 1 if ent is None else ent[1]]
            with self.lock:
                self.batches[key] = ent
                while len(self.batches) > self.cache_size:
                    old.append(self.batches.pop(next(iter(self.batches)))[0])
        for b in old:
            b.close()
        return ent[0]

    def submit(self, active, keep=False):
        batch = self._batch(active)
        self._set_iterates(active)
        batch.run()
        out = None
        with self.torch.cuda.stream(self.ctx.stream):
            if keep:
                out = [(batch.obj[x].clone(), batch.grad[x].clone()) for x in range(len(active))]
            ev = self.torch.cuda.Event()
            ev.record(self.ctx.stream)
        return ev, out, len(active)

    def finish(self, token):
        ev, out, n = token
        ev.synchronize()
        return out if out is not None else [None] * n

    def evaluate(self, active, keep=False):
        res = self.finish(self.submit(active, keep))
        self.ctx.sync()
        return res


class PlainEngine(_LibEngine):
    """Each request evaluated on its own (run it with max_active = 1)."""

    def load(self, j: Job):
        super().load(j)
        dev = j.handle.theta.gates.device
        g0 = j.data.iterates[0]
        D = 4 ** g0.n_qubits
        n_par = D + g0.M * D + g0.K * D * D
        torch = self.torch
        j.handle.out = (torch.empty(1, dtype=torch.float64, device=dev), None,
                        torch.empty(n_par, dtype=torch.float64, device=dev))

    def evaluate(self, active, keep=False):
        out = []
        for j in active:
            self._set_iterates([j])
            obj, _, g = j.handle.req.eval(j.handle.theta, want_probs=False, want_grad=True, out=j.handle.out)
            self.ctx.sync()
            out.append((obj.clone(), g.clone()) if keep else None)
        return out


def make_jobs(trace, n_iter: int = 20, data_fn=None) -> List[Job]:
    """Jobs of a trace (arrival, kind, S, seed); data from workloads.serving_request."""
    from . import workloads as W
    data_fn = data_fn or (lambda kind, S, seed: W.serving_request(kind, S, seed, n_iter))
    return [Job(rid=x, arrival=a, kind=k, S=S, data=data_fn(k, S, sd), n_iter=n_iter)
            for x, (a, k, S, sd) in enumerate(trace)]


def reset(jobs: Sequence[Job]):
    """Clear the per-run state of jobs (to replay the same trace on another engine)."""
    for j in jobs:
        j.k, j.footprint = 0, 0
        j.t_admit = j.t_done = math.nan
        j.t_iter, j.results = [], []
        j.handle = None
