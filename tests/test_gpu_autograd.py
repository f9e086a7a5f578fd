"""torch.autograd.Function over the HIP path: central finite differences (h = 1e-6)
on eight sampled models of the uneven batch, and the oracle gradient."""
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
    from paper_2008_13490_amd import api, autograd
    return api, autograd, api.Context(0)


def sampled_models(n=8):
    """Eight gate sets of the uneven batch (70% one-qubit, 30% two-qubit), each
    with a reduced number of its random sequences (lengths up to 1024)."""
    plan = W.c3_plan()
    rng = np.random.default_rng(8)
    pick = rng.choice(len(plan), size=n, replace=False)
    out = []
    for j in pick:
        kind, S, seed = plan[int(j)]
        out.append(W.random_workload(kind, min(S, 48), 1024, seed))
    return out


def test_autograd_finite_differences(oracle_lib, gpu):
    import torch
    api, ag, ctx = gpu
    for w in sampled_models():
        m, sl = w.model, w.seqs
        say(f"[autograd] {w.name}: S={sl.S} sumL={int(sl.offsets[-1])}")
        req = api.Request(ctx, m.n_qubits, m.K, m.M, sl.offsets, sl.gates, w.counts)
        rho = torch.tensor(m.rho, device="cuda", requires_grad=True)
        E = torch.tensor(m.effects, device="cuda", requires_grad=True)
        G = torch.tensor(m.gates, device="cuda", requires_grad=True)
        F = ag.gst_nll(rho, E, G, req)
        F.backward()
        ctx.sync()
        g = torch.cat([rho.grad.ravel(), E.grad.ravel(), G.grad.ravel()]).cpu().numpy()
        F0, _, g_or, _, _ = oracle_lib.loglik(m.rho, m.effects, m.gates, sl.offsets, sl.gates, w.counts)
        assert abs(float(F) - F0) <= 1e-10 * abs(F0)
        assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()
        theta = np.concatenate([m.rho, m.effects.ravel(), m.gates.ravel()])
        h = 1e-6

        def nll(th):
            r, e, gg = W.unpack_params(th, m.n_qubits, m.M, m.K)
            with torch.no_grad():
                v = ag.gst_nll(torch.tensor(r, device="cuda"), torch.tensor(e, device="cuda"),
                               torch.tensor(gg, device="cuda"), req)
            return float(v)

        rng = np.random.default_rng(3)
        scale = max(1.0, np.abs(g).max())
        for c in rng.choice(len(theta), size=12, replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[c] += h
            tm[c] -= h
            fd = (nll(tp) - nll(tm)) / (2 * h)
            assert abs(fd - g[c]) <= 1e-6 * scale, (c, fd, g[c])
        v = rng.standard_normal(len(theta))
        v /= np.linalg.norm(v)
        fd = (nll(theta + h * v) - nll(theta - h * v)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * scale


def test_autograd_probs_vjp(oracle_lib, gpu):
    import torch
    api, ag, ctx = gpu
    w = W.structured_workload("c1")
    m, sl = w.model, w.seqs
    say("[autograd] probs backward c1")
    req = api.Request(ctx, m.n_qubits, m.K, m.M, sl.offsets, sl.gates)
    rho = torch.tensor(m.rho, device="cuda", requires_grad=True)
    E = torch.tensor(m.effects, device="cuda", requires_grad=True)
    G = torch.tensor(m.gates, device="cuda", requires_grad=True)
    p = ag.gst_probs(rho, E, G, req)
    Wt = torch.tensor(np.random.default_rng(4).standard_normal(tuple(p.shape)), device="cuda")
    (p * Wt).sum().backward()
    ctx.sync()
    g = torch.cat([rho.grad.ravel(), E.grad.ravel(), G.grad.ravel()]).cpu().numpy()
    want = oracle_lib.vjp(m.rho, m.effects, m.gates, sl.offsets, sl.gates, Wt.cpu().numpy())
    p_or = oracle_lib.probs(m.rho, m.effects, m.gates, sl.offsets, sl.gates)
    # germ-power jumps of the sharing plan: 1e-12 relative on p
    assert np.all(np.abs(p.detach().cpu().numpy() - p_or) <= 1e-12 * np.abs(p_or))
    assert np.abs(g - want).max() <= 1e-10 * np.abs(want).max()
