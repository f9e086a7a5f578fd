"""GPU parity of the resident request (prefix-sharing plan) against the oracle."""
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


def run_request(oracle_lib, api, ctx, gs, sl, counts, label, expect_plan=None):
    say(f"[resident] {label}: S={sl.S} D={gs.D} K={gs.K} sumL={int(sl.offsets[-1])}")
    req = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, counts)
    info = req.plan_info()
    say(f"[resident] {label}: plan {info}")
    if expect_plan is not None:
        assert bool(info["plan_used"]) == expect_plan
    dg = api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)
    obj, p, g = req.eval(dg, want_probs=True, want_grad=True)
    ctx.sync()
    F, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    p = p.cpu().numpy()
    mism = np.count_nonzero(p != p_or)
    assert mism == 0, f"{mism} probabilities differ, max {np.abs(p - p_or).max()}"
    Fg = float(obj.cpu()[0])
    assert abs(Fg - F) <= 1e-10 * abs(F), (Fg, F)
    g = g.cpu().numpy()
    assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()
    # probabilities only, and objective only
    obj2, p2, g2 = req.eval(dg, want_probs=True, want_grad=False)
    ctx.sync()
    assert np.array_equal(p2.cpu().numpy(), p_or)
    assert abs(float(obj2.cpu()[0]) - F) <= 1e-10 * abs(F)
    # a second evaluation at another gate set reuses the resident plan
    rng = np.random.default_rng(1)
    gs2 = W.noisy_gateset({1: "1q", 2: "2q"}[gs.n_qubits], 1e-3, 0.01, rng)
    dg2 = api.DeviceGateSet.from_numpy(gs2.n_qubits, gs2.rho, gs2.effects, gs2.gates)
    p_or2 = oracle_lib.probs(gs2.rho, gs2.effects, gs2.gates, sl.offsets, sl.gates)
    c2 = counts.copy()
    c2[p_or2 <= 0] = 0
    req2 = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, c2)
    obj3, p3, g3 = req2.eval(dg2, want_probs=True)
    ctx.sync()
    F3, _, g_or3, _, _ = oracle_lib.loglik(gs2.rho, gs2.effects, gs2.gates, sl.offsets, sl.gates, c2)
    assert np.array_equal(p3.cpu().numpy(), p_or2)
    assert abs(float(obj3.cpu()[0]) - F3) <= 1e-10 * abs(F3)
    assert np.abs(g3.cpu().numpy() - g_or3).max() <= 1e-10 * np.abs(g_or3).max()
    return req


def test_resident_c1(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c1")
    run_request(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c1", expect_plan=True)


def test_resident_c2(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c2")
    run_request(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c2", expect_plan=True)


def test_resident_two_levels(oracle_lib, gpu):
    api, ctx = gpu
    rng = np.random.default_rng(12)
    base = list(rng.integers(0, 6, 60))
    words = [base + list(rng.integers(0, 6, int(rng.integers(30, 60)))) + list(rng.integers(0, 6, k))
             for k in range(5) for _ in range(4)]
    words += [base[:40 + k] for k in range(6)] + [[], base[:3]]
    sl = W.from_words(words)
    gs = W.noisy_gateset("2q", 1e-3, 0.01, rng)
    counts = rng.integers(0, 30, size=(sl.S, gs.M)).astype(np.int32)
    counts[oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates) <= 0] = 0
    req = run_request(oracle_lib, api, ctx, gs, sl, counts, "two-level list", expect_plan=True)
    assert req.plan_info()["levels"] >= 2


def test_resident_random_words_plain(oracle_lib, gpu):
    api, ctx = gpu
    w = W.random_workload("2q", 300, 300, 17, lmin=0)
    run_request(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "random words (no sharing)", expect_plan=False)


def test_resident_vjp(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    w = W.structured_workload("c1")
    gs, sl = w.model, w.seqs
    req = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates)
    assert req.plan_info()["plan_used"] == 1
    Wt = np.random.default_rng(2).standard_normal((sl.S, gs.M))
    dg = api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)
    say("[resident] vjp c1")
    g = req.vjp(dg, torch.as_tensor(Wt, device="cuda")).cpu().numpy()
    ctx.sync()
    want = oracle_lib.vjp(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, Wt)
    assert np.abs(g - want).max() <= 1e-10 * np.abs(want).max()
