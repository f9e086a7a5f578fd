"""GPU parity of the three-qubit path (D = 64) against the oracle.

Probabilities must be bit-identical to the oracle's (same fused multiply-add
order); objective 1e-10 relative, gradient 1e-10 normwise.  The full
structured three-qubit list is checked entry by entry against the oracle run
over shards of the list in parallel processes, and through the Euler
identities of the multilinear likelihood (exact at any size).
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


def _dev(api, gs):
    return api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)


def _check(oracle_lib, gs, sl, counts, obj, p, g, label):
    F, p_or, g_or, _, rc = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    assert rc == 0
    p = p.cpu().numpy()
    mism = np.count_nonzero(p != p_or)
    assert mism == 0, f"{label}: {mism} probabilities differ, max {np.abs(p - p_or).max()}"
    Fg = float(obj.cpu()[0])
    assert abs(Fg - F) <= 1e-10 * abs(F), (label, Fg, F)
    g = g.cpu().numpy()
    err = np.abs(g - g_or).max() / np.abs(g_or).max()
    assert err <= 1e-10, (label, err)
    return F


def test_3q_random_ragged(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    w = W.random_workload("3q", 300, 150, 41)
    sl = w.seqs
    # an empty word and a single-gate word among them
    words = [list(sl.word(s)) for s in range(sl.S)]
    words[5] = []
    words[17] = [3]
    sl = W.from_words(words)
    gs = w.model
    # the replaced words keep their counts only where the model gives p > 0
    counts = w.counts.copy()
    counts[oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates) <= 0] = 0
    say(f"[3q] random: S={sl.S} sumL={int(sl.offsets[-1])} K={gs.K} M={gs.M}")
    req = api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, counts)
    obj, p, g = req.eval(_dev(api, gs), want_probs=True, want_grad=True)
    ctx.sync()
    _check(oracle_lib, gs, sl, counts, obj, p, g, "request")
    say("[3q] random: context-level call")
    seqs = api.DeviceSeqs.from_numpy(sl.offsets, sl.gates)
    cnt = torch.as_tensor(counts, device="cuda")
    obj2, p2, g2 = ctx.loglik(_dev(api, gs), seqs, cnt, want_probs=True, want_grad=True)
    ctx.sync()
    assert torch.equal(p2, p) and torch.equal(obj2, obj) and torch.equal(g2, g)
    say("[3q] random: probabilities only and objective only")
    p3 = req.probs(_dev(api, gs))
    obj4, _, _ = req.eval(_dev(api, gs), want_probs=False, want_grad=False)
    ctx.sync()
    assert torch.equal(p3, p) and torch.equal(obj4, obj)


def test_3q_vjp(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    w = W.random_workload("3q", 64, 40, 42)
    gs, sl = w.model, w.seqs
    rng = np.random.default_rng(3)
    Wt = rng.standard_normal((sl.S, gs.M))
    say(f"[3q] vjp: S={sl.S}")
    req = api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, None)
    g = req.vjp(_dev(api, gs), torch.as_tensor(Wt, device="cuda"))
    ctx.sync()
    g_or = oracle_lib.vjp(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, Wt)
    err = np.abs(g.cpu().numpy() - g_or).max() / np.abs(g_or).max()
    assert err <= 1e-10, err


def test_c4_subset(oracle_lib, gpu):
    api, ctx = gpu
    w = W.structured_workload("c4")
    idx = np.arange(0, w.seqs.S, 97)
    sl = w.seqs.subset(idx)
    cnt = w.counts[idx]
    gs = w.model
    say(f"[3q] c4 subset: S={sl.S} sumL={int(sl.offsets[-1])}")
    req = api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, cnt)
    obj, p, g = req.eval(_dev(api, gs), want_probs=True, want_grad=True)
    ctx.sync()
    _check(oracle_lib, gs, sl, cnt, obj, p, g, "c4 subset")


def test_c4_full_against_oracle_and_euler(oracle_lib, gpu):
    """The whole structured three-qubit list: every probability, the objective
    and every gradient entry against the oracle (run over sequence shards in
    parallel processes), and the Euler identities of the multilinear likelihood."""
    from oracle_shards import loglik_sharded
    api, ctx = gpu
    w = W.structured_workload("c4")
    gs, sl = w.model, w.seqs
    say(f"[3q] c4 full: S={sl.S} sumL={int(sl.offsets[-1])}")
    req = api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, w.counts)
    obj, p, g = req.eval(_dev(api, gs), want_probs=True, want_grad=True)
    ctx.sync()
    p = p.cpu().numpy()
    g = g.cpu().numpy()
    F = float(obj.cpu()[0])
    say("[3q] c4 full: oracle over shards")
    F_or, p_or, g_or = loglik_sharded(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, w.counts)
    say("[3q] c4 full: oracle done")
    bad = np.abs(p - p_or) > 1e-12 * np.abs(p_or)
    assert not bad.any(), f"{int(bad.sum())} probabilities differ beyond 1e-12, max {np.abs(p - p_or).max()}"
    assert abs(F - F_or) <= 1e-10 * abs(F_or), (F, F_or)
    err = np.abs(g - g_or).max() / np.abs(g_or).max()
    assert err <= 1e-10, err
    # Euler identities of l = -F (multilinear in rho, in each e_m, in the gates)
    N = w.counts.astype(np.float64)
    D, M, K = 64, gs.M, gs.K
    rho_g, E_g, G_g = g[:D], g[D:D + M * D].reshape(M, D), g[D + M * D:].reshape(K, D, D)
    total = N.sum()
    assert abs(-np.dot(gs.rho, rho_g) - total) <= 1e-10 * total
    for m in range(M):
        t = N[:, m].sum()
        assert abs(-np.dot(gs.effects[m], E_g[m]) - t) <= 1e-10 * max(t, 1.0)
    L = sl.lengths()
    occ = np.zeros((sl.S, K))
    seq_of_step = np.repeat(np.arange(sl.S), L)
    np.add.at(occ, (seq_of_step, sl.gates.astype(np.int64)), 1.0)
    Ns = N.sum(axis=1)
    for k in range(K):
        t = float(np.dot(occ[:, k], Ns))
        assert abs(-np.sum(gs.gates[k] * G_g[k]) - t) <= 1e-10 * t, k


def test_3q_in_batch_and_nonpos(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    a = W.random_workload("3q", 120, 60, 43)
    b = W.random_workload("2q", 200, 80, 44)
    reqs = [api.Request(ctx, x.n_qubits, x.model.K, x.model.M, x.seqs.offsets, x.seqs.gates, x.counts)
            for x in (a, b)]
    th = [_dev(api, x.model) for x in (a, b)]
    ref = [r.eval(t, want_probs=True) for r, t in zip(reqs, th)]
    ctx.sync()
    say("[3q] batch with a two-qubit request")
    bt = api.Batch(ctx, reqs, th, want_probs=True, want_grad=True, capture_graph=True)
    for _ in range(2):
        bt.run()
        ctx.sync()
        for x, (o, p, g) in enumerate(ref):
            assert torch.equal(bt.obj[x], o) and torch.equal(bt.probs[x], p) and torch.equal(bt.grad[x], g)
    assert bt.nonpos() == [0, 0]
    say("[3q] p <= 0 with N > 0")
    E0 = a.model.effects.copy()
    E0[2] = 0.0
    bad = api.DeviceGateSet.from_numpy(3, a.model.rho, E0, a.model.gates)
    o, _, _ = reqs[0].eval(bad)
    rc, _, nnp = ctx.sync(raise_on_error=False)
    n_exp = int(np.count_nonzero(a.counts[:, 2] > 0))
    assert rc == -3 and nnp == n_exp and float(o.cpu()[0]) == float("inf")
    o2, _, _ = reqs[0].eval(th[0])
    ctx.sync()
    assert torch.equal(o2, ref[0][0])


def test_3q_empty_list(gpu):
    import torch
    api, ctx = gpu
    gs = W.noisy_gateset("3q", 1e-3, 0.01, np.random.default_rng(9))
    say("[3q] empty list")
    req = api.Request(ctx, 3, gs.K, gs.M, np.zeros(1, np.int64), np.zeros(0, np.uint8),
                      np.zeros((0, gs.M), np.int32))
    obj, _, g = req.eval(_dev(api, gs))
    ctx.sync()
    assert float(obj.cpu()[0]) == 0.0 and not torch.any(g != 0)


def _structured_3q(seed=7, n_fid=8, spec=((2, 4), (3, 4)), powers=(1, 2, 4, 8, 16, 32)):
    rng = np.random.default_rng(seed)
    gs = W.noisy_gateset("3q", 1e-3, 0.01, rng)
    fids = W.shortlex_words((1, 2), n_fid)
    germs = W.random_germs(gs.K, list(spec), rng)
    sl = W.structured_list(fids, fids, germs, list(powers))
    words = [list(sl.word(s)) for s in range(sl.S)]
    words += [words[5], [], words[len(words) // 3], []]   # duplicates and empty words
    sl = W.from_words(words)
    import oracle
    p = oracle.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates)
    counts = W.sample_counts(p, 1000, rng)
    return gs, sl, counts


def test_3q_grouped_plan(oracle_lib, gpu):
    """A structured three-qubit list runs on the grouped-chain plan (tiles of
    sixteen chains on the matrix cores): probabilities bit-identical to the
    oracle, objective and gradient within 1e-10; probabilities-only, vjp and a
    second evaluation give the same bits."""
    import torch
    api, ctx = gpu
    gs, sl, counts = _structured_3q()
    req = api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, counts)
    info = req.plan_info()
    say(f"[3q] grouped plan: S={sl.S} sumL={int(sl.offsets[-1])} {info}")
    assert info["grouped"] == 1 and info["tiles"] > 0
    th = _dev(api, gs)
    obj, p, g = req.eval(th, want_probs=True, want_grad=True)
    ctx.sync()
    _check(oracle_lib, gs, sl, counts, obj, p, g, "grouped plan")
    obj2, p2, g2 = req.eval(th, want_probs=True, want_grad=True)
    p3 = req.probs(th)
    ctx.sync()
    assert torch.equal(obj2, obj) and torch.equal(p2, p) and torch.equal(g2, g) and torch.equal(p3, p)
    rng = np.random.default_rng(3)
    Wt = rng.standard_normal((sl.S, gs.M))
    gv = req.vjp(th, torch.as_tensor(Wt, device="cuda"))
    ctx.sync()
    g_or = oracle_lib.vjp(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, Wt)
    err = np.abs(gv.cpu().numpy() - g_or).max() / np.abs(g_or).max()
    assert err <= 1e-10, err


def test_3q_grouped_plan_in_batch_and_nonpos(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    gs, sl, counts = _structured_3q(seed=8, n_fid=6, powers=(1, 2, 4, 8))
    b = W.random_workload("2q", 200, 80, 44)
    reqs = [api.Request(ctx, 3, gs.K, gs.M, sl.offsets, sl.gates, counts),
            api.Request(ctx, 2, b.model.K, b.model.M, b.seqs.offsets, b.seqs.gates, b.counts)]
    assert reqs[0].plan_info()["grouped"] == 1
    th = [_dev(api, gs), _dev(api, b.model)]
    ref = [r.eval(t, want_probs=True) for r, t in zip(reqs, th)]
    ctx.sync()
    say("[3q] grouped plan in a batch")
    bt = api.Batch(ctx, reqs, th, want_probs=True, want_grad=True, capture_graph=True)
    for _ in range(2):
        bt.run()
        ctx.sync()
        for x, (o, p, g) in enumerate(ref):
            assert torch.equal(bt.obj[x], o) and torch.equal(bt.probs[x], p) and torch.equal(bt.grad[x], g)
    say("[3q] grouped plan: p <= 0 with N > 0")
    E0 = gs.effects.copy()
    E0[2] = 0.0
    bad = api.DeviceGateSet.from_numpy(3, gs.rho, E0, gs.gates)
    o, _, _ = reqs[0].eval(bad)
    rc, _, nnp = ctx.sync(raise_on_error=False)
    assert rc == -3 and nnp == int(np.count_nonzero(counts[:, 2] > 0)) and float(o.cpu()[0]) == float("inf")
    o2, _, _ = reqs[0].eval(th[0])
    ctx.sync()
    assert torch.equal(o2, ref[0][0])


def test_3q_grouped_plans_batched_per_kernel(gpu):
    """Several grouped-chain plans in one batch run as one launch per kernel and
    level (request = blockIdx.y): two gate sets on one list, a second list with
    other levels, next to a two-qubit request and a three-qubit list without
    sharing.  Every result equals the request's standalone result bit for bit,
    eagerly and on graph replays, and a request with p <= 0 counts only its own."""
    import torch
    api, ctx = gpu
    gs_a, sl_a, cnt_a = _structured_3q(seed=8, n_fid=6, powers=(1, 2, 4, 8))
    gs_b = W.noisy_gateset("3q", 2e-3, 0.02, np.random.default_rng(21))
    gs_c, sl_c, cnt_c = _structured_3q(seed=11, n_fid=5, spec=((2, 3), (3, 3)), powers=(1, 2, 4, 8, 16, 32, 64))
    plain3 = W.random_workload("3q", 90, 40, 45)
    two = W.random_workload("2q", 150, 60, 46)
    reqs = [api.Request(ctx, 3, gs_a.K, gs_a.M, sl_a.offsets, sl_a.gates, cnt_a),
            api.Request(ctx, 3, gs_a.K, gs_a.M, sl_a.offsets, sl_a.gates, cnt_a),
            api.Request(ctx, 3, gs_c.K, gs_c.M, sl_c.offsets, sl_c.gates, cnt_c),
            api.Request(ctx, 2, two.model.K, two.model.M, two.seqs.offsets, two.seqs.gates, two.counts),
            api.Request(ctx, 3, plain3.model.K, plain3.model.M, plain3.seqs.offsets, plain3.seqs.gates,
                        plain3.counts)]
    grouped = [r.plan_info()["grouped"] for r in reqs]
    assert grouped[:3] == [1, 1, 1] and grouped[4] == 0
    th = [_dev(api, gs_a), _dev(api, gs_b), _dev(api, gs_c), _dev(api, two.model), _dev(api, plain3.model)]
    ref = [r.eval(t, want_probs=True) for r, t in zip(reqs, th)]
    ctx.sync()
    for capture in (False, True):
        say(f"[3q] grouped plans batched per kernel, capture={capture}")
        bt = api.Batch(ctx, reqs, th, want_probs=True, want_grad=True, capture_graph=capture)
        for _ in range(2):
            bt.run()
            ctx.sync()
            for x, (o, p, g) in enumerate(ref):
                assert torch.equal(bt.obj[x], o), x
                assert torch.equal(bt.probs[x], p), x
                assert torch.equal(bt.grad[x], g), x
        assert bt.nonpos() == [0] * len(reqs)
    say("[3q] grouped plans batched: p <= 0 with N > 0 in one request")
    E0 = gs_c.effects.copy()
    E0[2] = 0.0
    th_bad = list(th)
    th_bad[2] = api.DeviceGateSet.from_numpy(3, gs_c.rho, E0, gs_c.gates)
    bt = api.Batch(ctx, reqs, th_bad, want_probs=True, want_grad=True, capture_graph=True)
    bt.run()
    rc, _, _ = ctx.sync(raise_on_error=False)
    n_exp = int(np.count_nonzero(cnt_c[:, 2] > 0))
    assert bt.nonpos() == [0, 0, n_exp, 0, 0]
    assert float(bt.obj[2].cpu()[0]) == float("inf")
    for x in (0, 1, 3, 4):
        assert torch.equal(bt.obj[x], ref[x][0]) and torch.equal(bt.grad[x], ref[x][2]), x


def test_c4_full_batched_equals_standalone(gpu):
    """The whole c4 list for two gate sets in one batch (the batched long level
    with its two-row event window, two tiles per CU): each request's
    probabilities, objective and gradient are the bits of its standalone
    evaluation."""
    import torch
    api, ctx = gpu
    w = W.structured_workload("c4")
    sets = [w.model, W.noisy_gateset("3q", W.LAMBDA, W.SIGMA, np.random.default_rng(81))]
    say(f"[3q] c4 full batched: S={w.seqs.S}")
    reqs = [api.Request(ctx, 3, g.K, g.M, w.seqs.offsets, w.seqs.gates, w.counts) for g in sets]
    assert all(r.plan_info()["grouped"] == 1 for r in reqs)
    th = [_dev(api, g) for g in sets]
    ref = [r.eval(t, want_probs=True) for r, t in zip(reqs, th)]
    ctx.sync()
    bt = api.Batch(ctx, reqs, th, want_probs=True, want_grad=True, capture_graph=True)
    for _ in range(2):
        bt.run()
        ctx.sync()
        for x, (o, p, g) in enumerate(ref):
            assert torch.equal(bt.obj[x], o), x
            assert torch.equal(bt.probs[x], p), x
            assert torch.equal(bt.grad[x], g), x
    assert bt.nonpos() == [0, 0]
