"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Probabilities must be bit-identical (both sides accumulate every dot product
with one fused multiply-add per term, ascending, from zero).  The objective is
compared at 1e-10 relative and the gradient at 1e-10 normwise (max-norm), as
stated for the path; gradients are sums whose order differs from the oracle's
sequential loop.
"""
import sys

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-10
GRAD_RTOL = 1e-10


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_13490_amd import api
    return api, api.Context(0)


def to_dev(api, gs, sl):
    return (api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates),
            api.DeviceSeqs.from_numpy(sl.offsets, sl.gates))


def check_case(oracle_lib, api, ctx, gs, sl, counts, label):
    import torch
    say(f"[parity] {label}: S={sl.S} D={gs.D} K={gs.K} sumL={int(sl.offsets[-1])}")
    dg, ds = to_dev(api, gs, sl)
    p_gpu = ctx.probs(dg, ds).cpu().numpy()
    ctx.sync()
    p_or = oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates)
    assert p_gpu.shape == p_or.shape
    mism = np.count_nonzero(p_gpu != p_or)
    assert mism == 0, f"{mism} probabilities differ; max abs {np.abs(p_gpu - p_or).max()}"
    cnt = torch.as_tensor(counts, device="cuda")
    obj, p2, g = ctx.loglik(dg, ds, cnt, want_probs=True)
    ctx.sync()
    F, _, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    assert np.array_equal(p2.cpu().numpy(), p_or)
    Fg = float(obj.cpu()[0])
    assert abs(Fg - F) <= OBJ_RTOL * max(abs(F), 1.0), (Fg, F)
    gg = g.cpu().numpy()
    err = np.abs(gg - g_or).max()
    assert err <= GRAD_RTOL * max(np.abs(g_or).max(), 1e-300), (err, np.abs(g_or).max())
    return p_gpu, gg


def test_c1_full(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c1")
    check_case(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c1 full")


def test_c2_subset(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c2")
    idx = np.arange(0, w.seqs.S, 11)
    sub = w.seqs.subset(idx)
    check_case(oracle_lib, api, ctx, w.model, sub, w.counts[idx], "c2 every 11th")


def test_c2_full(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c2")
    check_case(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c2 full")


@pytest.mark.parametrize("kind,S,lmax,seed", [("2q", 37, 100, 1), ("2q", 203, 300, 2), ("1q", 101, 1024, 3),
                                              ("2q", 5, 1030, 4)])
def test_random_words_ragged(oracle_lib, gpu, kind, S, lmax, seed):
    api, ctx = gpu
    w = W.random_workload(kind, S, lmax, seed, lmin=0)
    check_case(oracle_lib, api, ctx, w.model, w.seqs, w.counts, f"random {kind} S={S} lmax={lmax}")


def test_vjp_matches_oracle(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    w = W.random_workload("2q", 150, 64, 9, lmin=0)
    gs, sl = w.model, w.seqs
    rng = np.random.default_rng(5)
    Wt = rng.standard_normal((sl.S, gs.M))
    dg, ds = to_dev(api, gs, sl)
    say("[parity] vjp 2q S=150")
    g = ctx.vjp(dg, ds, torch.as_tensor(Wt, device="cuda")).cpu().numpy()
    ctx.sync()
    want = oracle_lib.vjp(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, Wt)
    assert np.abs(g - want).max() <= GRAD_RTOL * np.abs(want).max()


def test_edge_cases(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    rng = np.random.default_rng(3)
    gs = W.noisy_gateset("2q", 1e-3, 0.01, rng)
    # empty list
    say("[parity] edge: empty list")
    sl = W.from_words([])
    dg, ds = to_dev(api, gs, sl)
    obj, p, g = ctx.loglik(dg, ds, torch.zeros((0, 4), dtype=torch.int32, device="cuda"), want_probs=True)
    ctx.sync()
    assert float(obj.cpu()[0]) == 0.0 and torch.all(g == 0)
    # only empty sequences and one long one
    say("[parity] edge: empty sequences")
    sl = W.from_words([[], [], list(rng.integers(0, 6, 777)), []])
    counts = rng.integers(0, 10, size=(4, 4)).astype(np.int32)
    # ideal SPAM: an empty sequence has p = 0 exactly on outcomes != 0
    p_or = oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates)
    counts[p_or <= 0] = 0
    check_case(oracle_lib, api, ctx, gs, sl, counts, "edge: empty sequences")


def test_bad_index_and_nonpos(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    rng = np.random.default_rng(4)
    gs = W.noisy_gateset("2q", 1e-3, 0.01, rng)
    say("[parity] error: gate index >= K")
    sl = W.from_words([[0, 1, 9, 2], [3]])
    dg, ds = to_dev(api, gs, sl)
    ctx.probs(dg, ds)
    rc, nbad, nnp = ctx.sync(raise_on_error=False)
    assert rc == -2 and nbad == 1
    say("[parity] error: p <= 0 with N > 0")
    E0 = gs.effects.copy()
    E0[2] = 0.0
    sl = W.from_words([[0, 1], [3], []])
    dg = api.DeviceGateSet.from_numpy(2, gs.rho, E0, gs.gates)
    ds = api.DeviceSeqs.from_numpy(sl.offsets, sl.gates)
    cnt = torch.ones((3, 4), dtype=torch.int32, device="cuda")
    obj, p, g = ctx.loglik(dg, ds, cnt)
    rc, nbad, nnp = ctx.sync(raise_on_error=False)
    p_or = oracle_lib.probs(gs.rho, E0, gs.gates, sl.offsets, sl.gates)
    assert rc == -3 and nnp == int(np.count_nonzero(p_or <= 0)) and float(obj.cpu()[0]) == float("inf")
