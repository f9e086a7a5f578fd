"""The continuous-batching service on the GPU: each request's results in the
mix (requests of one, two and three qubits arriving while others run,
joining and leaving rounds) are identical, bit for bit, to the results of
the same request evaluated alone at the same iterates."""
import sys

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_13490_amd import api
    return api, api.Context(0)


def test_served_results_equal_alone(gpu):
    import torch
    from paper_2008_13490_amd import serving as SV
    api, ctx = gpu
    kinds = ["1q", "2q", "3q", "1q", "2q", "1q", "3q", "2q", "1q", "2q"]
    rng = np.random.default_rng(11)
    trace = [(0.004 * x, k, int(rng.integers(300, 2500)), int(rng.integers(1, 2 ** 40)))
             for x, k in enumerate(kinds)]
    jobs = SV.make_jobs(trace, n_iter=3)
    say("[serving] batched engine")
    out = SV.Scheduler(SV.GPUEngine(ctx), 1 << 36, max_active=4, keep_results=True).run(jobs)
    say(f"[serving] {out}")
    assert out["iterations"] == 30 and out["rounds"] >= 3
    served = {j.rid: j.results for j in jobs}
    SV.reset(jobs)
    say("[serving] plain engine")
    SV.Scheduler(SV.PlainEngine(ctx), 1 << 36, max_active=1, keep_results=True).run(jobs)
    plain = {j.rid: j.results for j in jobs}
    say("[serving] alone")
    for j in jobs:
        d = j.data
        g0 = d.iterates[0]
        req = api.Request(ctx, g0.n_qubits, g0.K, g0.M, d.seqs.offsets, d.seqs.gates, d.counts)
        for k, gk in enumerate(d.iterates):
            th = api.DeviceGateSet.from_numpy(gk.n_qubits, gk.rho, gk.effects, gk.gates)
            obj, _, g = req.eval(th)
            ctx.sync()
            for name, res in (("served", served), ("plain", plain)):
                o2, g2 = res[j.rid][k]
                assert torch.equal(o2, obj) and torch.equal(g2, g), (name, j.rid, j.kind, k)
        req.close()


def test_pipelined_served_results_equal_alone(gpu):
    """Two rounds in flight, requests loaded and unloaded on a host thread,
    the context on its own stream; structured lists (shared-prefix plans,
    batched per kernel) next to random one-, two- and three-qubit lists.  Every
    result equals the request's evaluation alone, bit for bit."""
    import torch
    from paper_2008_13490_amd import serving as SV
    api, _ = gpu
    ctx = api.Context(0, stream=torch.cuda.Stream())
    rng = np.random.default_rng(12)
    n_iter = 3
    jobs = []
    for x, k in enumerate(["2q", "c1", "1q", "3q", "c2", "1q", "2q", "c1", "3q", "1q", "c2", "2q"]):
        if k in ("c1", "c2"):
            w = W.structured_workload(k)
            kind = {"c1": "1q", "c2": "2q"}[k]
            its = [W.noisy_gateset(kind, 1e-3, 0.01, rng) for _ in range(n_iter)]
            data = W.FitRequestData(kind, w.seqs, w.counts, its)
        else:
            data = W.serving_request(k, int(rng.integers(300, 2500)), int(rng.integers(1, 2 ** 40)), n_iter)
        jobs.append(SV.Job(rid=x, arrival=0.003 * x, kind=data.kind, S=data.seqs.S, data=data, n_iter=n_iter))
    say("[serving] pipelined batched engine")
    out = SV.Scheduler(SV.GPUEngine(ctx, capture_graph=False), 1 << 36, max_active=6, keep_results=True,
                       depth=2, prefetch=True).run(jobs)
    ctx.sync()
    say(f"[serving] {out}")
    assert out["iterations"] == len(jobs) * n_iter
    for j in jobs:
        d = j.data
        g0 = d.iterates[0]
        req = api.Request(ctx, g0.n_qubits, g0.K, g0.M, d.seqs.offsets, d.seqs.gates, d.counts)
        for k, gk in enumerate(d.iterates):
            th = api.DeviceGateSet.from_numpy(gk.n_qubits, gk.rho, gk.effects, gk.gates)
            torch.cuda.synchronize()
            obj, _, g = req.eval(th)
            ctx.sync()
            o2, g2 = j.results[k]
            assert torch.equal(o2, obj) and torch.equal(g2, g), (j.rid, j.kind, k)
        req.close()
    ctx.close()
