"""GPU parity of the TP and CPTP parameterizations (estimation modes of thesis
Sec. 6.3.2) against the oracle, and of the likelihood gradient with respect to
the parameters of each mode on the two-qubit GST list.

TP maps are copies and differences in the same order on both sides: bit for
bit.  CPTP gates come from matrix exponentials (Taylor with scaling and
squaring here, Pade in the oracle) and are compared at 1e-13 absolute on the
transfer-matrix entries (bounded by one for CPTP maps) and 1e-10 in the
max-norm relative to the largest component for gradients; the state's
coordinates at 1e-15 absolute.
"""
import sys

import numpy as np
import pytest

from oracle import params as PR
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
    return api, api.Context(0), torch


def targets_of(kind):
    _, Us, n = W.ideal_unitaries(kind)
    return np.array([W.ptm_from_unitary(U) for U in Us]), n


def theta_near(mode, n, M, K, rng, scale):
    """Seeded parameters: TP around the ideal gates with computational-basis
    effects; CPTP with a state near |0..0>, effects of the computational basis,
    small Hamiltonian parts and a dissipator with a diagonal of `scale`."""
    D, d = 4 ** n, 2 ** n
    eff = np.zeros((M - 1, D))
    P = PR.paulis(n)
    for m in range(M - 1):
        proj = np.zeros((d, d))
        proj[m, m] = 1.0
        eff[m] = np.array([np.trace(P[a] @ proj).real for a in range(D)]) / np.sqrt(d)
    if mode == "tp":
        G0, _ = targets_of("1q" if n == 1 else "2q")
        rho = np.zeros(D - 1)
        rho[D - 2] = 1 / np.sqrt(d)   # +Z on the last qubit's coordinate
        g = (G0[:, 1:, :] + rng.normal(size=(K, D - 1, D)) * scale).reshape(-1)
        return np.concatenate([rho, eff.reshape(-1), g])
    A = np.zeros(D)
    A[0] = 1.0
    A[d:] = rng.normal(size=D - d) * scale
    A[1:d] = np.abs(rng.normal(size=d - 1)) * scale
    gates = []
    m = D - 1
    for _ in range(K):
        h = rng.normal(size=m) * scale
        tdiag = scale + np.abs(rng.normal(size=m)) * scale
        pairs = rng.normal(size=m * (m - 1)) * scale * 0.3
        gates.append(np.concatenate([h, tdiag, pairs]))
    return np.concatenate([A, eff.reshape(-1)] + gates)


CASES = [("tp", 1, 2, 3, 0.05), ("tp", 2, 4, 6, 0.05), ("cptp", 1, 2, 3, 0.05), ("cptp", 2, 4, 6, 0.05),
         ("cptp", 1, 2, 3, 0.8), ("cptp", 2, 4, 6, 0.5)]


@pytest.mark.parametrize("mode,n,M,K,scale", CASES)
def test_param_maps_match_oracle(gpu, mode, n, M, K, scale):
    api, ctx, torch = gpu
    rng = np.random.default_rng(11 + n + int(100 * scale))
    G0, _ = targets_of("1q" if n == 1 else "2q")
    th = theta_near(mode, n, M, K, rng, scale)
    say(f"[params] {mode} n={n} M={M} K={K} scale={scale}: {th.size} parameters")
    par = api.Parameterization(ctx, mode, n, M, K, torch.as_tensor(G0, device="cuda") if mode == "cptp" else None)
    assert par.count == PR.param_count(mode, n, M, K) == th.size
    tt = torch.as_tensor(th, device="cuda")
    gs = par.forward(tt)
    rho, E, G = PR.forward(mode, th, n, M, K, G0)
    r_g, E_g, G_g = gs.rho.cpu().numpy(), gs.effects.cpu().numpy(), gs.gates.cpu().numpy()
    assert np.array_equal(E_g, E)
    if mode == "tp":
        assert np.array_equal(r_g, rho) and np.array_equal(G_g, G)
    else:
        assert np.abs(r_g - rho).max() <= 1e-15
        err = np.abs(G_g - G).max()
        say(f"[params] max |dG| = {err:.3g}")
        assert err <= 1e-13
    gbar = rng.normal(size=PR.param_count("full", n, M, K))
    g_g = par.backward(tt, torch.as_tensor(gbar, device="cuda")).cpu().numpy()
    g_o = PR.backward(mode, th, n, M, K, gbar, G0)
    if mode == "tp":
        assert np.array_equal(g_g, g_o)
    else:
        rel = np.abs(g_g - g_o).max() / np.abs(g_o).max()
        say(f"[params] gradient max-norm relative difference {rel:.3g}")
        assert rel <= 1e-10


def test_full_mode_is_the_identity(gpu):
    api, ctx, torch = gpu
    rng = np.random.default_rng(3)
    par = api.Parameterization(ctx, "full", 2, 4, 6)
    th = torch.as_tensor(rng.normal(size=par.count), device="cuda")
    gs = par.forward(th)
    assert torch.equal(torch.cat([gs.rho, gs.effects.reshape(-1), gs.gates.reshape(-1)]), th)
    assert torch.equal(par.backward(th, th), th)


def test_param_errors(gpu):
    api, ctx, torch = gpu
    from paper_2008_13490_amd import _lib
    with pytest.raises(_lib.GSTError):
        api.Parameterization(ctx, "cptp", 3, 8, 5)                       # three qubits
    par = api.Parameterization(ctx, "cptp", 1, 2, 3)
    with pytest.raises(_lib.GSTError):
        par.forward(torch.zeros(par.count, dtype=torch.float64, device="cuda"))   # no targets
    with pytest.raises(ValueError):
        par.forward(torch.zeros(par.count + 1, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("mode", ["tp", "cptp"])
def test_likelihood_gradient_in_mode(oracle_lib, gpu, mode):
    """F(theta) and dF/dtheta on the two-qubit GST list through the resident request:
    parameterization forward, evaluation, parameterization backward; against the
    oracle's forward map, likelihood and chain rule."""
    api, ctx, torch = gpu
    w = W.structured_workload("c2")
    n, M, K = 2, 4, 6
    G0, _ = targets_of("2q")
    rng = np.random.default_rng(21)
    if mode == "tp":
        # the C2 evaluation point itself is trace preserving with a complete POVM
        m = w.model
        th = np.concatenate([m.rho[1:], m.effects[:M - 1].reshape(-1), m.gates[:, 1:, :].reshape(-1)])
    else:
        th = theta_near(mode, n, M, K, rng, 0.03)
    par = api.Parameterization(ctx, mode, n, M, K, torch.as_tensor(G0, device="cuda") if mode == "cptp" else None)
    tt = torch.as_tensor(th, device="cuda")
    req = api.Request(ctx, n, K, M, w.seqs.offsets, w.seqs.gates, w.counts)
    gs = par.forward(tt)
    obj = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(req.n_params, dtype=torch.float64, device="cuda")
    req.eval(gs, want_probs=False, want_grad=True, out=(obj, None, grad))
    g_theta = par.backward(tt, grad).cpu().numpy()
    rho, E, G = PR.forward(mode, th, n, M, K, G0)
    F_o, _, g_full, _, _ = oracle_lib.loglik(rho, E, G, w.seqs.offsets, w.seqs.gates, w.counts)
    g_o = PR.backward(mode, th, n, M, K, g_full, G0)
    F_g = float(obj.cpu())
    say(f"[params] {mode}: F gpu {F_g!r} oracle {F_o!r}")
    assert abs(F_g - F_o) <= 1e-10 * abs(F_o)
    rel = np.abs(g_theta - g_o).max() / np.abs(g_o).max()
    say(f"[params] {mode}: gradient max-norm relative difference {rel:.3g}")
    assert rel <= 1e-10


def test_autograd_through_parameterization(gpu):
    """gst_nll(*gst_gateset(theta, par), request).backward() gives the same dF/dtheta
    as the explicit forward / evaluation / backward calls (bit for bit)."""
    api, ctx, torch = gpu
    from paper_2008_13490_amd import autograd as AG
    w = W.structured_workload("c1")
    n, M, K = 1, 2, 3
    G0, _ = targets_of("1q")
    th = theta_near("cptp", n, M, K, np.random.default_rng(31), 0.03)
    par = api.Parameterization(ctx, "cptp", n, M, K, torch.as_tensor(G0, device="cuda"))
    req = api.Request(ctx, n, K, M, w.seqs.offsets, w.seqs.gates, w.counts)
    theta = torch.tensor(th, device="cuda", requires_grad=True)
    F = AG.gst_nll(*AG.gst_gateset(theta, par), req)
    F.backward()
    tt = torch.as_tensor(th, device="cuda")
    obj, _, grad = req.eval(par.forward(tt), want_probs=False, want_grad=True)
    want = par.backward(tt, grad)
    assert float(F.detach()) == float(obj[0])
    assert torch.equal(theta.grad, want)
