"""Batched evaluation of several resident requests (one persistent launch).

Each request's result in a batch must be identical, bit for bit, to its
standalone evaluation, and the standalone results must match the oracle
(probabilities bit for bit, or to 1e-12 relative for a sharing plan with
germ-power jumps; objective 1e-10 relative, gradient 1e-10 normwise).  The graph-captured form is replayed several times with other
work and synchronizations between replays, every replay checked against the
eager result at the gate sets current at that time.
"""
import sys

import numpy as np
import pytest

from paper_2008_13490_amd import _lib
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


def _mix():
    """(label, workload-like tuple) of a mixed batch: ragged 1q and 2q random
    lists (plain tiles), one tiny list, the structured 1q list (sharing plan)
    and an empty list."""
    out = []
    for kind, S, lmax, seed in (("1q", 700, 300, 11), ("2q", 500, 200, 12), ("1q", 37, 40, 13),
                                ("2q", 170, 1030, 14)):
        w = W.random_workload(kind, S, lmax, seed)
        out.append((w.name, w.model, w.seqs, w.counts))
    w = W.structured_workload("c1")
    out.append(("c1", w.model, w.seqs, w.counts))
    gs = W.noisy_gateset("2q", 1e-3, 0.01, np.random.default_rng(15))
    empty = W.SeqList(np.zeros(1, np.int64), np.zeros(0, np.uint8), None)
    out.append(("empty-2q", gs, empty, np.zeros((0, gs.M), np.int32)))
    return out


def _requests(api, ctx, mix):
    reqs, thetas = [], []
    for label, gs, sl, counts in mix:
        r = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, counts)
        reqs.append(r)
        thetas.append(api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates))
        say(f"[batch] request {label}: S={sl.S} D={gs.D} K={gs.K} plan={r.plan_info()['plan_used']}")
    return reqs, thetas


def _standalone(ctx, reqs, thetas):
    res = []
    for r, t in zip(reqs, thetas):
        obj, p, g = r.eval(t, want_probs=True, want_grad=True)
        res.append((obj, p, g))
    ctx.sync()
    return [(o.clone(), p.clone(), g.clone()) for o, p, g in res]


def _assert_same(batch, ref, labels):
    import torch
    for x, (o, p, g) in enumerate(ref):
        assert torch.equal(batch.obj[x], o), (labels[x], batch.obj[x], o)
        assert torch.equal(batch.probs[x], p), labels[x]
        assert torch.equal(batch.grad[x], g), labels[x]


def test_batch_equals_standalone_and_oracle(oracle_lib, gpu):
    api, ctx = gpu
    mix = _mix()
    labels = [m[0] for m in mix]
    reqs, thetas = _requests(api, ctx, mix)
    ref = _standalone(ctx, reqs, thetas)
    for (label, gs, sl, counts), (o, p, g), r in zip(mix, ref, reqs):
        say(f"[batch] oracle check {label}")
        F, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
        if r.plan_info()["jump_trunks"] == 0:
            assert np.array_equal(p.cpu().numpy(), p_or), label
        else:  # germ-power jumps: rounding of the matrix powers, 1e-12 relative
            pp = p.cpu().numpy()
            assert np.all(np.abs(pp - p_or) <= 1e-12 * np.abs(p_or)), label
        Fg = float(o.cpu()[0])
        assert abs(Fg - F) <= 1e-10 * max(abs(F), 1e-300), (label, Fg, F)
        gg = g.cpu().numpy()
        assert np.abs(gg - g_or).max() <= 1e-10 * max(np.abs(g_or).max(), 1e-300), label
    say("[batch] eager batch")
    b = api.Batch(ctx, reqs, thetas, want_probs=True, want_grad=True, capture_graph=False)
    for _ in range(2):
        b.run()
        ctx.sync()
        _assert_same(b, ref, labels)
    assert b.nonpos() == [0] * len(reqs)
    # a sub-batch in another order gives the same results for its members
    say("[batch] sub-batch, reversed order")
    sub = [4, 1, 0]
    b2 = api.Batch(ctx, [reqs[x] for x in sub], [thetas[x] for x in sub], want_probs=True, want_grad=True)
    b2.run()
    ctx.sync()
    _assert_same(b2, [ref[x] for x in sub], [labels[x] for x in sub])
    b.close()
    b2.close()


def test_batch_graph_replays(gpu):
    import torch
    api, ctx = gpu
    mix = _mix()
    labels = [m[0] for m in mix]
    reqs, thetas = _requests(api, ctx, mix)
    b = api.Batch(ctx, reqs, thetas, want_probs=True, want_grad=True, capture_graph=True)
    rng = np.random.default_rng(21)
    scratch = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(4):
        say(f"[batch] graph replay {rep}")
        if rep > 0:
            # new gate sets in place (the graph holds the pointers)
            for (label, gs, _, _), t in zip(mix, thetas):
                g2 = W.noisy_gateset({1: "1q", 2: "2q"}[gs.n_qubits], 1e-3, 0.01, rng)
                t.gates.copy_(torch.as_tensor(g2.gates, device="cuda"))
        ref = _standalone(ctx, reqs, thetas)
        scratch.add_(1.0)                        # unrelated eager work between replays
        b.run()
        torch.cuda.synchronize()
        ctx.sync()
        _assert_same(b, ref, labels)
        for r, t in zip(reqs[:2], thetas[:2]):   # more eager library work on the same stream
            r.eval(t, want_probs=False, want_grad=True)
        ctx.sync()
    b.close()


def test_batch_nonpos_is_per_request(oracle_lib, gpu):
    api, ctx = gpu
    good = W.random_workload("2q", 300, 120, 31)
    bad = W.random_workload("1q", 200, 60, 32)
    E0 = bad.model.effects.copy()
    E0[1] = 0.0                                 # p_1 = 0 wherever N_1 > 0
    reqs, thetas = [], []
    for gs, sl, cnt, E in ((good.model, good.seqs, good.counts, good.model.effects),
                           (bad.model, bad.seqs, bad.counts, E0)):
        reqs.append(api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, cnt))
        thetas.append(api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, E, gs.gates))
    p_or = oracle_lib.probs(bad.model.rho, E0, bad.model.gates, bad.seqs.offsets, bad.seqs.gates)
    n_expected = int(np.count_nonzero((p_or <= 0) & (bad.counts > 0)))
    assert n_expected > 0
    say("[batch] nonpos: standalone")
    o_bad, _, _ = reqs[1].eval(thetas[1])
    o_good, _, g_good = reqs[0].eval(thetas[0])
    rc, _, nnp = ctx.sync(raise_on_error=False)
    assert rc == -3 and nnp == n_expected
    assert float(o_bad.cpu()[0]) == float("inf")
    # a failing evaluation does not leak into the next one
    F, _, g_or, _, _ = oracle_lib.loglik(good.model.rho, good.model.effects, good.model.gates, good.seqs.offsets,
                                         good.seqs.gates, good.counts)
    assert abs(float(o_good.cpu()[0]) - F) <= 1e-10 * abs(F)
    say("[batch] nonpos: batched")
    b = api.Batch(ctx, reqs, thetas, want_probs=False, want_grad=True, capture_graph=True)
    b.run()
    assert b.nonpos() == [0, n_expected]
    rc, _, nnp = ctx.sync(raise_on_error=False)
    assert rc == -3 and nnp == n_expected
    import torch
    assert torch.equal(b.obj[0], o_good) and torch.equal(b.grad[0], g_good)
    assert float(b.obj[1].cpu()[0]) == float("inf")
    b.close()


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 8])
def test_one_qubit_gate_counts(oracle_lib, gpu, K):
    """One-qubit requests with K gates: K <= 4 run one chain per lane, larger
    K the 16-lane teams; both must match the oracle and give the same bits
    alone and next to a two-qubit request in a batch."""
    import torch
    api, ctx = gpu
    rng = np.random.default_rng(100 + K)
    pool = [W.noisy_gateset("1q", 1e-3, 0.01, rng) for _ in range(3)]
    G = np.concatenate([g.gates for g in pool])[:K]
    gs = W.GateSet(1, [f"g{k}" for k in range(K)], pool[0].rho, pool[0].effects, np.ascontiguousarray(G))
    sl = W.random_list(300, K, 0, 200, rng)
    counts = W.sample_counts(np.full((sl.S, 2), 0.5), 1000, rng)
    counts[oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates) <= 0] = 0  # empty words
    say(f"[batch] one qubit, K={K}: S={sl.S} sumL={int(sl.offsets[-1])}")
    req = api.Request(ctx, 1, K, 2, sl.offsets, sl.gates, counts)
    th = api.DeviceGateSet.from_numpy(1, gs.rho, gs.effects, gs.gates)
    obj, p, g = req.eval(th, want_probs=True, want_grad=True)
    ctx.sync()
    F, p_or, g_or, _, rc = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    assert rc == 0
    if req.plan_info()["jump_trunks"] == 0:
        assert np.array_equal(p.cpu().numpy(), p_or)
    else:  # germ-power jumps of the sharing plan: 1e-12 relative
        assert np.all(np.abs(p.cpu().numpy() - p_or) <= 1e-12 * np.abs(p_or))
    assert abs(float(obj.cpu()[0]) - F) <= 1e-10 * abs(F)
    assert np.abs(g.cpu().numpy() - g_or).max() <= 1e-10 * np.abs(g_or).max()
    other = W.random_workload("2q", 90, 60, 7)
    r2 = api.Request(ctx, 2, other.model.K, other.model.M, other.seqs.offsets, other.seqs.gates, other.counts)
    t2 = api.DeviceGateSet.from_numpy(2, other.model.rho, other.model.effects, other.model.gates)
    b = api.Batch(ctx, [r2, req], [t2, th], want_probs=True, want_grad=True, capture_graph=True)
    b.run()
    ctx.sync()
    assert torch.equal(b.obj[1], obj) and torch.equal(b.probs[1], p) and torch.equal(b.grad[1], g)
    b.close()


def test_tile_policy(oracle_lib, gpu):
    """A request created under another tile policy (the autotuner's knob)
    gives the same probabilities, the objective and gradient within the
    tolerance, and the same bits alone and in a batch."""
    import torch
    api, ctx = gpu
    w = W.random_workload("2q", 400, 300, 51)
    v = W.random_workload("1q", 500, 300, 52)
    ref = {}
    for n, x in ((2, w), (1, v)):
        r = api.Request(ctx, n, x.model.K, x.model.M, x.seqs.offsets, x.seqs.gates, x.counts)
        t = api.DeviceGateSet.from_numpy(n, x.model.rho, x.model.effects, x.model.gates)
        ref[n] = r.eval(t, want_probs=True)
    ctx.sync()
    for tile, bpc in ((48, 1), (128, 0)):
        say(f"[batch] tile policy {tile} x {bpc}")
        api.tune_set(ctx, 2, tile, bpc)
        api.tune_set(ctx, 1, tile, bpc)
        reqs, ths = [], []
        for n, x in ((2, w), (1, v)):
            reqs.append(api.Request(ctx, n, x.model.K, x.model.M, x.seqs.offsets, x.seqs.gates, x.counts))
            ths.append(api.DeviceGateSet.from_numpy(n, x.model.rho, x.model.effects, x.model.gates))
        outs = [r.eval(t, want_probs=True) for r, t in zip(reqs, ths)]
        ctx.sync()
        b = api.Batch(ctx, reqs, ths, want_probs=True, want_grad=True)
        b.run()
        ctx.sync()
        for x, (n, (o, p, g)) in enumerate(zip((2, 1), outs)):
            o0, p0, g0 = ref[n]
            assert torch.equal(p, p0)
            assert abs(float(o.cpu()[0]) - float(o0.cpu()[0])) <= 1e-12 * abs(float(o0.cpu()[0]))
            assert float((g - g0).abs().max()) <= 1e-12 * float(g0.abs().max())
            assert torch.equal(b.obj[x], o) and torch.equal(b.grad[x], g) and torch.equal(b.probs[x], p)
        b.close()
    api.tune_set(ctx, 2, 0, 0)
    api.tune_set(ctx, 1, 0, 0)


def test_tile_sums_across_chunk_edges(oracle_lib, gpu):
    """The tile partial sums are added in chunks of 32 tiles and then over the
    chunks: lists of 1, 32, 33 (one tile past a chunk) and 65 tiles (the last
    tile ragged) against the oracle, and the same requests in one batch equal
    to their standalone results bit for bit."""
    api, ctx = gpu
    api.tune_set(ctx, 2, 16, 0)  # 16 sequences per tile: the tile counts below are exact
    try:
        mix, reqs, thetas = [], [], []
        for nt, short in ((1, 0), (32, 0), (33, 0), (65, 5)):
            w = W.random_workload("2q", 16 * nt - short, 24, 100 + nt)
            r = api.Request(ctx, 2, w.model.K, w.model.M, w.seqs.offsets, w.seqs.gates, w.counts)
            assert r.plan_info()["plan_used"] == 0
            mix.append((w.name, w.model, w.seqs, w.counts))
            reqs.append(r)
            thetas.append(api.DeviceGateSet.from_numpy(2, w.model.rho, w.model.effects, w.model.gates))
        ref = _standalone(ctx, reqs, thetas)
        for (label, gs, sl, counts), (o, p, g) in zip(mix, ref):
            say(f"[batch] chunk edges: {label}")
            F, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
            assert np.array_equal(p.cpu().numpy(), p_or), label
            assert abs(float(o.cpu()[0]) - F) <= 1e-10 * abs(F), label
            assert np.abs(g.cpu().numpy() - g_or).max() <= 1e-10 * np.abs(g_or).max(), label
        b = api.Batch(ctx, reqs[::-1], thetas[::-1], want_probs=True, want_grad=True)
        b.run()
        ctx.sync()
        _assert_same(b, ref[::-1], [m[0] for m in mix[::-1]])
        b.close()
        with pytest.raises(_lib.GSTError, match="twice"):
            api.Batch(ctx, [reqs[0], reqs[1], reqs[0]], [thetas[0], thetas[1], thetas[0]], want_grad=True)
        for r in reqs:
            r.close()
    finally:
        api.tune_set(ctx, 2)


def test_plans_batched_per_kernel_equal_standalone(gpu):
    """Several sharing-plan requests (two-qubit structured list with three gate
    sets, the one-qubit one with and without counts) next to plain-tile ones:
    the plans run as one launch per kernel and level, and every request's
    results are the same bits as its standalone evaluation, eager and replayed
    from a graph with the gate sets changed in place between replays."""
    import torch
    api, ctx = gpu
    c2 = W.structured_workload("c2")
    c1 = W.structured_workload("c1")
    rnd = W.random_workload("2q", 300, 150, 41)
    rng = np.random.default_rng(42)
    mix = [("c2-a", c2.model, c2.seqs, c2.counts),
           ("c2-b", W.noisy_gateset("2q", 1e-3, 0.01, rng), c2.seqs, c2.counts),
           ("random-2q", rnd.model, rnd.seqs, rnd.counts),
           ("c1", c1.model, c1.seqs, c1.counts),
           ("c2-c", W.noisy_gateset("2q", 2e-3, 0.02, rng), c2.seqs, c2.counts),
           ("c1-probs", c1.model, c1.seqs, None)]
    labels = [m[0] for m in mix]
    reqs, thetas = [], []
    for label, gs, sl, counts in mix:
        r = api.Request(ctx, gs.n_qubits, gs.K, gs.M, sl.offsets, sl.gates, counts)
        reqs.append(r)
        thetas.append(api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates))
        say(f"[plan batch] request {label}: S={sl.S} plan={r.plan_info()['plan_used']}")
    assert sum(r.plan_info()["plan_used"] for r in reqs) == 5

    def standalone():
        out = []
        for r, t in zip(reqs, thetas):
            if r.has_counts:
                o, p, g = r.eval(t, want_probs=True, want_grad=True)
            else:
                o, p, g = None, r.probs(t), None
            out.append((o, p, g))
        ctx.sync()
        return out

    def same(b, ref):
        for x, (o, p, g) in enumerate(ref):
            assert torch.equal(b.probs[x], p), labels[x]
            if o is not None:
                assert torch.equal(b.obj[x], o), (labels[x], b.obj[x], o)
                assert torch.equal(b.grad[x], g), labels[x]

    ref = standalone()
    say("[plan batch] eager")
    b = api.Batch(ctx, reqs, thetas, want_probs=True, want_grad=True, capture_graph=False)
    for _ in range(2):
        b.run()
        ctx.sync()
        same(b, ref)
    assert b.nonpos() == [0] * len(reqs)
    b.close()
    say("[plan batch] graph replays")
    b = api.Batch(ctx, reqs, thetas, want_probs=True, want_grad=True, capture_graph=True)
    for rep in range(3):
        if rep > 0:
            for (label, gs, _, _), t in zip(mix, thetas):
                g2 = W.noisy_gateset({1: "1q", 2: "2q"}[gs.n_qubits], 1e-3, 0.01, rng)
                t.gates.copy_(torch.as_tensor(g2.gates, device="cuda"))
        ref = standalone()
        b.run()
        torch.cuda.synchronize()
        ctx.sync()
        same(b, ref)
    b.close()


def test_many_plans_share_workgroups_and_equal_standalone(gpu):
    """Twenty requests on the structured two-qubit list: enough item chunks
    that the batch gives each request fewer item and fill workgroups than its
    standalone launch (several chunks per workgroup); the chunks keep their
    head rows, so every result is still the same bits as alone."""
    import torch
    api, ctx = gpu
    c2 = W.structured_workload("c2")
    rng = np.random.default_rng(77)
    n = 20
    reqs, thetas = [], []
    for x in range(n):
        gs = c2.model if x == 0 else W.noisy_gateset("2q", 1e-3, 0.01, rng)
        reqs.append(api.Request(ctx, 2, gs.K, gs.M, c2.seqs.offsets, c2.seqs.gates, c2.counts))
        thetas.append(api.DeviceGateSet.from_numpy(2, gs.rho, gs.effects, gs.gates))
    ref = []
    for r, t in zip(reqs, thetas):
        o, p, g = r.eval(t, want_probs=True, want_grad=True)
        ref.append((o, p, g))
    ctx.sync()
    say(f"[plan batch] {n} requests")
    b = api.Batch(ctx, reqs, thetas, want_probs=True, want_grad=True, capture_graph=True)
    for _ in range(2):
        b.run()
        ctx.sync()
        for x, (o, p, g) in enumerate(ref):
            assert torch.equal(b.obj[x], o) and torch.equal(b.probs[x], p) and torch.equal(b.grad[x], g), x
    b.close()
