"""GPU parity of the resident request (prefix-sharing plan) against the oracle.

Without germ-power jumps the plan's probabilities are bit-identical to the
oracle's.  With jumps (the default) the states after each jump come from
matrix powers of the germ, and the probabilities are checked at the stated
1e-12 relative tolerance; objective and gradient at 1e-10 either way.
"""
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


P_RTOL = 1e-12


def check_probs(p, p_or, exact):
    if exact:
        mism = np.count_nonzero(p != p_or)
        assert mism == 0, f"{mism} probabilities differ, max {np.abs(p - p_or).max()}"
    else:
        rel = np.abs(p - p_or) / np.maximum(np.abs(p_or), 1e-300)
        rel[(p == p_or)] = 0.0
        assert rel.max() <= P_RTOL, (rel.max(), p_or.flat[int(np.argmax(rel))])
        say(f"[resident] max relative probability difference {rel.max():.3g}")


def run_request(oracle_lib, api, ctx, gs, sl, counts, label, expect_plan=None, jump=8):
    say(f"[resident] {label}: S={sl.S} D={gs.D} K={gs.K} sumL={int(sl.offsets[-1])} jump={jump}")
    api.set_plan_jump(ctx, jump)
    try:
        return _run_request(oracle_lib, api, ctx, gs, sl, counts, label, expect_plan)
    finally:
        api.set_plan_jump(ctx, 8)


def _run_request(oracle_lib, api, ctx, gs, sl, counts, label, expect_plan):
    req = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, counts)
    info = req.plan_info()
    say(f"[resident] {label}: plan {info}")
    if expect_plan is not None:
        assert bool(info["plan_used"]) == expect_plan
    exact = info["jump_trunks"] == 0
    dg = api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)
    obj, p, g = req.eval(dg, want_probs=True, want_grad=True)
    ctx.sync()
    F, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    p = p.cpu().numpy()
    check_probs(p, p_or, exact)
    Fg = float(obj.cpu()[0])
    assert abs(Fg - F) <= 1e-10 * abs(F), (Fg, F)
    g = g.cpu().numpy()
    assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()
    # probabilities only, and objective only
    obj2, p2, g2 = req.eval(dg, want_probs=True, want_grad=False)
    ctx.sync()
    assert np.array_equal(p2.cpu().numpy(), p)
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
    check_probs(p3.cpu().numpy(), p_or2, exact)
    assert abs(float(obj3.cpu()[0]) - F3) <= 1e-10 * abs(F3)
    assert np.abs(g3.cpu().numpy() - g_or3).max() <= 1e-10 * np.abs(g_or3).max()
    return req


@pytest.mark.parametrize("jump", [8, 0])
def test_resident_c1(oracle_lib, gpu, jump):
    api, ctx = gpu
    w = W.structured_workload("c1")
    req = run_request(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c1", expect_plan=True, jump=jump)
    assert (req.plan_info()["jump_trunks"] > 0) == (jump > 0)


@pytest.mark.parametrize("jump", [8, 0, 2, 16])
def test_resident_c2(oracle_lib, gpu, jump):
    api, ctx = gpu
    w = W.structured_workload("c2")
    req = run_request(oracle_lib, api, ctx, w.model, w.seqs, w.counts, "c2", expect_plan=True, jump=jump)
    info = req.plan_info()
    assert (info["jump_trunks"] > 0) == (jump > 0)
    if jump == 8:
        assert info["chain_max"] <= 100 and info["fill_tasks"] > 0  # longest trunk: 772 steps


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


def test_resident_crowded_state(oracle_lib, gpu):
    """One stored state receives 300 item adjoints: more source rows than the
    injection kernel loads at once (eight per group of lanes)."""
    api, ctx = gpu
    rng = np.random.default_rng(13)
    base = list(rng.integers(0, 6, 48))
    words = [base + list(rng.integers(0, 6, int(rng.integers(1, 5)))) for _ in range(300)]
    words += [base[:20], [], base]
    sl = W.from_words(words)
    gs = W.noisy_gateset("2q", 1e-3, 0.01, rng)
    counts = rng.integers(0, 30, size=(sl.S, gs.M)).astype(np.int32)
    counts[oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates) <= 0] = 0
    run_request(oracle_lib, api, ctx, gs, sl, counts, "crowded state", expect_plan=True)


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


@pytest.mark.parametrize("kind", ["c2-plan", "1q", "3q"])
def test_request_from_device_pointers(gpu, kind):
    """gst_req_create (device list and counts) builds the same request as
    gst_req_create_host: every output equal bit for bit."""
    import torch
    api, ctx = gpu
    if kind == "c2-plan":
        w = W.structured_workload("c2")
        idx = np.arange(0, w.seqs.S, 7)
        gs, sl, cnt = w.model, w.seqs.subset(idx), w.counts[idx]
    else:
        w = W.random_workload(kind, 150, 60, 51)
        gs, sl, cnt = w.model, w.seqs, w.counts
    say(f"[resident] from device: {kind} S={sl.S}")
    th = api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)
    a = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, cnt)
    seqs = api.DeviceSeqs.from_numpy(sl.offsets, sl.gates)
    b = api.Request.from_device(ctx, gs.n_qubits, gs.K, gs.M, seqs, torch.as_tensor(cnt, device="cuda"))
    assert a.plan_info() == b.plan_info()
    ra = a.eval(th, want_probs=True)
    rb = b.eval(th, want_probs=True)
    ctx.sync()
    for x, y in zip(ra, rb):
        assert torch.equal(x, y)
    a.close()
    b.close()


def test_gate_count_limits(gpu):
    """More gates than gst_max_gates allows, or a gate index >= K, is refused at
    creation (GST_EINVAL, GST_EINDEX) for host and device lists alike."""
    import torch
    from paper_2008_13490_amd import _lib
    api, ctx = gpu
    off = np.array([0, 2, 3], np.int64)
    gts = np.array([0, 1, 2], np.uint8)
    for n in (1, 2, 3):
        K = api.max_gates(n)
        with pytest.raises(_lib.GSTError) as e:
            api.Request(ctx, n, K + 1, 2, off, gts, None)
        assert e.value.code == _lib.GST_EINVAL
        with pytest.raises(_lib.GSTError) as e:
            api.Request.from_device(ctx, n, K + 1, 2, api.DeviceSeqs.from_numpy(off, gts))
        assert e.value.code == _lib.GST_EINVAL
    with pytest.raises(_lib.GSTError) as e:
        api.Request.from_device(ctx, 2, 2, 4, api.DeviceSeqs.from_numpy(off, gts))
    assert e.value.code == _lib.GST_EINDEX
