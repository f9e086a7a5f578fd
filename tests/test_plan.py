"""The prefix-sharing plan, checked on the CPU.

The plan (a trie of the sequences, thesis Eq. GSTFullFiducialsGerms: F_q g^l F_p
shares F_p g^l between measurement fiducials and powers) is executed here by
a small numpy interpreter that follows the same schedule as the kernels
(trunks forward, items from stored states, injections, trunks backward) and
compared with the oracle.  Probabilities must be bit-identical: the
interpreter uses the same fused multiply-add order as the oracle, and sharing
reuses identical operations.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_13490_amd", "csrc")


@pytest.fixture(scope="module")
def planlib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("plan") / "libplanprobe.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(ROOT, "tests", "plan_probe.cpp"), os.path.join(CSRC, "gst_plan.cpp"), "-o", out],
                   check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.plan_build.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, P]
    lib.plan_copy.argtypes = [P] * 9
    lib.plan_copy_records.argtypes = [P] * 4
    lib.plan_copy_segments.argtypes = [P] * 5
    lib.plan_set_jump.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.plan_jump_sizes.argtypes = [P]
    lib.plan_copy_jumps.argtypes = [P] * 7
    lib.plan_n_ops.restype = ctypes.c_int64
    lib.plan_copy_ops.argtypes = [P] * 3
    lib.plan_copy_sources.argtypes = [P] * 2
    return lib


def get_plan(lib, sl, K, min_trunk=24, reanchor=8, ratio=0.8):
    K = int(K)
    sizes = np.zeros(13, np.int64)
    off = np.ascontiguousarray(sl.offsets, np.int64)
    g = np.ascontiguousarray(sl.gates if sl.gates.size else np.zeros(1, np.uint8), np.uint8)
    lib.plan_build(off.ctypes.data, g.ctypes.data, sl.S, K, min_trunk, reanchor, ratio, sizes.ctypes.data)
    used, nI, nT, nTS, nJ, nSrc, nL, nN, sumL, nR, root, nIS, nSeg = [int(x) for x in sizes]
    P = dict(used=bool(used), items=np.zeros((nI, 4), np.int64), trunk_ptr=np.zeros(nT + 1, np.int64),
             trunk_anchor=np.zeros(nT, np.int64), trunk_gates=np.zeros(max(nTS, 1), np.uint8),
             trunk_inj=np.zeros(max(nTS, 1), np.int32), inj_loc=np.zeros(max(nJ, 1), np.int64),
             inj_ptr=np.zeros(nJ + 1, np.int64), inj_src=np.zeros(max(nSrc, 1), np.int64),
             level_ptr=np.zeros(nL + 1, np.int64), n_nodes=nN, sum_len=sumL, n_levels=nL)
    lib.plan_copy(*[P[k].ctypes.data for k in ["items", "trunk_ptr", "trunk_anchor", "trunk_gates", "trunk_inj",
                                              "inj_loc", "inj_ptr", "inj_src", "level_ptr"]])
    if used:
        P["item_step_ptr"] = np.zeros(nI + 1, np.int64)
        P["rec_b"] = np.zeros(max(nR, 1), np.int64)
        P["rec_f"] = np.zeros(max(nR, 1), np.int64)
        P["rec_gate_ptr"] = np.zeros(K + 1, np.int64)
        lib.plan_copy_records(P["item_step_ptr"].ctypes.data, P["rec_b"].ctypes.data, P["rec_f"].ctypes.data,
                              P["rec_gate_ptr"].ctypes.data)
        P["rec_b"], P["rec_f"] = P["rec_b"][:nR], P["rec_f"][:nR]
        P["root_slot"] = root
        P["seg_ptr"] = np.zeros(nT + 1, np.int64)
        P["seg_start"] = np.zeros(max(nSeg, 1), np.int32)
        P["seg_count"] = np.zeros(max(nSeg, 1), np.int32)
        P["seg_pattern"] = np.zeros(max(nSeg, 1), np.uint32)
        P["seg_gate3"] = np.zeros(max(nSeg, 1), np.uint8)
        lib.plan_copy_segments(*[P[k].ctypes.data for k in ["seg_ptr", "seg_start", "seg_count", "seg_pattern",
                                                              "seg_gate3"]])
        js = np.zeros(3, np.int64)
        lib.plan_jump_sizes(js.ctypes.data)
        levels, nJT, nF = [int(x) for x in js]
        P["jump_levels"] = levels
        P["jump_trunks"] = nJT
        P["jump_pattern"] = np.zeros(max(nT, 1), np.uint32)
        P["jump_gate3"] = np.zeros(max(nT, 1), np.uint8)
        P["fill_first"] = np.zeros(max(nF, 1), np.int64)
        P["fill_in"] = np.zeros(max(nF, 1), np.int64)
        P["fill_n"] = np.zeros(max(nF, 1), np.int32)
        P["fill_pattern"] = np.zeros(max(nF, 1), np.uint32)
        P["fill_gate3"] = np.zeros(max(nF, 1), np.uint8)
        lib.plan_copy_jumps(*[P[k].ctypes.data for k in ["jump_pattern", "jump_gate3", "fill_first", "fill_in",
                                                           "fill_n", "fill_pattern", "fill_gate3"]])
        for k in ("jump_pattern", "jump_gate3"):
            P[k] = P[k][:nT]
        for k in ("fill_first", "fill_in", "fill_n", "fill_pattern", "fill_gate3"):
            P[k] = P[k][:nF]
        nOp = int(lib.plan_n_ops())
        P["op_ptr"] = np.zeros(nT + 1, np.int64)
        P["op_desc"] = np.zeros(max(nOp, 1), np.uint32)
        P["op_slot"] = np.zeros(max(nOp, 1), np.int32)
        lib.plan_copy_ops(P["op_ptr"].ctypes.data, P["op_desc"].ctypes.data, P["op_slot"].ctypes.data)
        P["op_desc"], P["op_slot"] = P["op_desc"][:nOp], P["op_slot"][:nOp]
        P["item_src"] = np.zeros(max(nI, 1), np.int32)
        P["trunk_src"] = np.zeros(max(nT, 1), np.int32)
        lib.plan_copy_sources(P["item_src"].ctypes.data, P["trunk_src"].ctypes.data)
        P["item_src"], P["trunk_src"] = P["item_src"][:nI], P["trunk_src"][:nT]
    P["trunk_gates"] = P["trunk_gates"][:nTS]
    P["trunk_inj"] = P["trunk_inj"][:nTS]
    P["inj_loc"] = P["inj_loc"][:nJ]
    P["inj_src"] = P["inj_src"][:nSrc]
    return P


_libm = ctypes.CDLL("libm.so.6")
_libm.fma.argtypes = [ctypes.c_double] * 3
_libm.fma.restype = ctypes.c_double
fma = _libm.fma  # correctly rounded fused multiply-add (C99)


def fma_matvec(G, f):
    out = np.empty_like(f)
    for i in range(len(f)):
        acc = 0.0
        for j in range(len(f)):
            acc = fma(G[i, j], f[j], acc)
        out[i] = acc
    return out


def run_plan(P, gs, sl, counts):
    """Executes the plan: probabilities (same fma order) and gradient (float64)."""
    D, M, K = gs.D, gs.M, gs.K
    G, E, rho = gs.gates, gs.effects, gs.rho
    nTS = len(P["trunk_gates"])
    states = np.zeros((nTS, D))
    tp, ta, tg = P["trunk_ptr"], P["trunk_anchor"], P["trunk_gates"]
    for t in range(len(ta)):            # levels are in order of t
        f = rho.copy() if ta[t] < 0 else states[ta[t]].copy()
        for j in range(tp[t], tp[t + 1]):
            f = fma_matvec(G[tg[j]], f)
            states[j] = f
    S = sl.S
    probs = np.zeros((S, M))
    grad_rho = np.zeros(D)
    grad_E = np.zeros((M, D))
    grad_G = np.zeros((K, D, D))
    item_adj = np.zeros((len(P["items"]), D))
    for q, (s, beg, end, anc) in enumerate(P["items"]):
        f = rho.copy() if anc < 0 else states[anc].copy()
        fs = [f]
        for x in range(beg, end):
            f = fma_matvec(G[sl.gates[x]], f)
            fs.append(f)
        for m in range(M):
            acc = 0.0
            for j in range(D):
                acc = fma(E[m, j], f[j], acc)
            probs[s, m] = acc
        dp = np.where(counts[s] > 0, -counts[s] / np.where(probs[s] > 0, probs[s], 1.0), 0.0)
        grad_E += np.outer(dp, f)
        b = dp @ E
        for x in range(end - 1, beg - 1, -1):
            k = sl.gates[x]
            grad_G[k] += np.outer(b, fs[x - beg])
            b = G[k].T @ b
        if anc < 0:
            grad_rho += b
        else:
            item_adj[q] = b
    trunk_adj = np.zeros((len(ta), D))
    inj = np.zeros((len(P["inj_loc"]), D))
    lp = P["level_ptr"]
    for lvl in range(P["n_levels"] - 1, -1, -1):
        for slot in range(len(P["inj_loc"])):
            v = np.zeros(D)
            for z in range(P["inj_ptr"][slot], P["inj_ptr"][slot + 1]):
                src = P["inj_src"][z]
                v += item_adj[src] if src >= 0 else trunk_adj[-src - 1]
            inj[slot] = v
        for t in range(lp[lvl], lp[lvl + 1]):
            b = np.zeros(D)
            for j in range(tp[t + 1] - 1, tp[t] - 1, -1):
                if P["trunk_inj"][j] >= 0:
                    b = b + inj[P["trunk_inj"][j]]
                fprev = (rho if ta[t] < 0 else states[ta[t]]) if j == tp[t] else states[j - 1]
                k = tg[j]
                grad_G[k] += np.outer(b, fprev)
                b = G[k].T @ b
            if ta[t] < 0:
                grad_rho += b
            else:
                trunk_adj[t] = b
    # the gradient GEMM's view: arenas of states and adjoints, records grouped by gate
    if "rec_b" in P:
        nIS = int(P["item_step_ptr"][-1])
        FA = np.zeros((1 + nTS + nIS, D))
        BA = np.zeros((nTS + nIS, D))
        FA[0] = rho
        FA[1:1 + nTS] = states
        item_adj2 = np.zeros((len(P["items"]), D))
        for q, (s, beg, end, anc) in enumerate(P["items"]):
            f = rho.copy() if anc < 0 else states[anc].copy()
            row0 = int(P["item_step_ptr"][q])
            for x in range(beg, end):
                FA[1 + nTS + row0 + x - beg] = f
                f = fma_matvec(G[sl.gates[x]], f)
            dp = np.where(counts[s] > 0, -counts[s] / np.where(probs[s] > 0, probs[s], 1.0), 0.0)
            b = dp @ E
            for x in range(end - 1, beg - 1, -1):
                BA[nTS + row0 + x - beg] = b
                b = G[sl.gates[x]].T @ b
            item_adj2[q] = b
        tadj = np.zeros((len(ta), D))
        inj2 = np.zeros((len(P["inj_loc"]), D))
        for lvl in range(P["n_levels"] - 1, -1, -1):
            for slot in range(len(P["inj_loc"])):
                if P["inj_loc"][slot] < 0:
                    continue
                inj2[slot] = sum((item_adj2[src] if src >= 0 else tadj[-src - 1]
                                  for src in P["inj_src"][P["inj_ptr"][slot]:P["inj_ptr"][slot + 1]]), np.zeros(D))
            for t in range(lp[lvl], lp[lvl + 1]):
                b = np.zeros(D)
                for j in range(tp[t + 1] - 1, tp[t] - 1, -1):
                    if P["trunk_inj"][j] >= 0:
                        b = b + inj2[P["trunk_inj"][j]]
                    BA[j] = b
                    b = G[tg[j]].T @ b
                tadj[t] = b
        root = P["root_slot"]
        drho = sum((item_adj2[src] if src >= 0 else tadj[-src - 1]
                    for src in P["inj_src"][P["inj_ptr"][root]:P["inj_ptr"][root + 1]]), np.zeros(D))
        drho = drho + sum((item_adj2[q] for q in range(len(P["items"])) if P["items"][q, 3] < 0), np.zeros(D))
        dG2 = np.zeros((K, D, D))
        gp = P["rec_gate_ptr"]
        for k in range(K):
            for r in range(gp[k], gp[k + 1]):
                dG2[k] += np.outer(BA[P["rec_b"][r]], FA[P["rec_f"][r]])
        scale = np.abs(grad_G).max()
        assert np.abs(dG2 - grad_G).max() <= 1e-10 * scale
        assert np.abs(drho - grad_rho).max() <= 1e-10 * np.abs(grad_rho).max()
    return probs, np.concatenate([grad_rho, grad_E.ravel(), grad_G.ravel()])


def test_plan_c1_structure_and_execution(planlib, oracle_lib):
    w = W.structured_workload("c1")
    P = get_plan(planlib, w.seqs, w.model.K)
    assert P["used"]
    # every sequence is one item; items are sorted by remaining length
    assert sorted(P["items"][:, 0].tolist()) == list(range(w.seqs.S))
    rem = P["items"][:, 2] - P["items"][:, 1]
    assert np.all(np.diff(rem) <= 0)
    steps = len(P["trunk_gates"]) + rem.sum()
    assert steps < 0.2 * P["sum_len"]
    gs = w.model
    p, g = run_plan(P, gs, w.seqs, w.counts)
    _, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, w.seqs.offsets, w.seqs.gates, w.counts)
    assert np.array_equal(p, p_or)
    assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()


def test_plan_c2_sharing_ratio(planlib):
    w = W.structured_workload("c2")
    P = get_plan(planlib, w.seqs, w.model.K)
    assert P["used"] and P["n_levels"] == 1
    rem = P["items"][:, 2] - P["items"][:, 1]
    steps = len(P["trunk_gates"]) + rem.sum()
    # the germ chains dominate: sharing saves more than 10x
    assert steps * 10 < P["sum_len"]
    # every item starts at a stored state or at rho, and its remaining word is a suffix of its own word
    for s, beg, end, anc in P["items"][::97]:
        assert w.seqs.offsets[s] <= beg <= end == w.seqs.offsets[s + 1]


def test_plan_multilevel_and_random(planlib, oracle_lib):
    rng = np.random.default_rng(12)
    # a long common prefix, then long branches at depth > reanchor depth: two levels
    base = list(rng.integers(0, 3, 40))
    words = [base + list(rng.integers(0, 3, int(rng.integers(20, 40)))) + list(rng.integers(0, 3, k))
             for k in range(6) for _ in range(3)]
    words += [base[:30 + k] for k in range(5)] + [[]]
    sl = W.from_words(words)
    gs = W.noisy_gateset("1q", 1e-3, 0.01, rng)
    counts = rng.integers(0, 20, size=(sl.S, gs.M)).astype(np.int32)
    counts[oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates) <= 0] = 0
    P = get_plan(planlib, sl, gs.K, min_trunk=8, reanchor=4, ratio=1.0)
    assert P["used"] and P["n_levels"] >= 2
    p, g = run_plan(P, gs, sl, counts)
    _, p_or, g_or, _, _ = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    assert np.array_equal(p, p_or)
    assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()
    # random words share almost nothing: the plan is declined
    wr = W.random_workload("2q", 300, 200, 3)
    P = get_plan(planlib, wr.seqs, 6)
    assert not P["used"]


def pattern_gates(pat, g3):
    per = pat & 0xff
    return [(pat >> 8) & 0xff, (pat >> 16) & 0xff, (pat >> 24) & 0xff, int(g3)][:per]


def segments_word(P, t):
    """Rebuilds trunk t's gate word from its periodic segments; a jump segment
    (period 0) stands for 2^e repetitions of its pattern per jump."""
    out = []
    for sg in range(P["seg_ptr"][t], P["seg_ptr"][t + 1]):
        pat = int(P["seg_pattern"][sg])
        assert P["seg_start"][sg] == len(out)
        if pat & 0xff == 0:
            stride, e = (pat >> 8) & 0xff, pat >> 16
            assert e < P["jump_levels"]
            gates = pattern_gates(int(P["jump_pattern"][t]), P["jump_gate3"][t])
            assert stride == (1 << e) * len(gates)
            out += gates * ((1 << e) * int(P["seg_count"][sg]))
        else:
            out += pattern_gates(pat, P["seg_gate3"][sg]) * int(P["seg_count"][sg])
    return out


def jump_matrices(P, G, t):
    """Trunk t's jump pattern product to the powers 2^e, e < jump_levels
    (plain numpy)."""
    out = []
    A = np.eye(G.shape[1])
    for g in pattern_gates(int(P["jump_pattern"][t]), P["jump_gate3"][t]):
        A = G[g] @ A
    for e in range(P["jump_levels"]):
        out.append(A)
        A = A @ A
    return out


def chain_schedule(P, G, rho, inj):
    """The trunk sweeps as the kernels order them with germ-power jumps: the
    chain over segments (a jump applies its matrix and stores only the state
    after it), then the fill tasks; the reverse sweep likewise with the
    transposes, adding inj[slot] at the states that receive injections.
    Returns the state and adjoint arenas and how often each row was written."""
    D = G.shape[1]
    tp, ta, tg, ti = P["trunk_ptr"], P["trunk_anchor"], P["trunk_gates"], P["trunk_inj"]
    nTS = len(tg)
    FA = np.full((1 + nTS, D), np.nan)
    FA[0] = rho
    BA = np.full((nTS, D), np.nan)
    wf = np.zeros(nTS, np.int64)
    wb = np.zeros(nTS, np.int64)
    tadj = np.zeros((len(ta), D))
    segs = lambda t: range(P["seg_ptr"][t], P["seg_ptr"][t + 1])
    for t in range(len(ta)):
        f = FA[0] if ta[t] < 0 else FA[1 + ta[t]]
        base = tp[t]
        J = jump_matrices(P, G, t)
        for sg in segs(t):
            st, cnt, pat = int(P["seg_start"][sg]), int(P["seg_count"][sg]), int(P["seg_pattern"][sg])
            if pat & 0xff == 0:
                stride = (pat >> 8) & 0xff
                for c in range(cnt):
                    f = J[pat >> 16] @ f
                    j = base + st + (c + 1) * stride - 1
                    FA[1 + j] = f
                    wf[j] += 1
            else:
                gates = pattern_gates(pat, P["seg_gate3"][sg])
                for c in range(cnt):
                    for q, g in enumerate(gates):
                        f = G[g] @ f
                        j = base + st + c * len(gates) + q
                        FA[1 + j] = f
                        wf[j] += 1
    for q in range(len(P["fill_first"])):
        first, n = int(P["fill_first"][q]), int(P["fill_n"][q])
        gates = pattern_gates(int(P["fill_pattern"][q]), P["fill_gate3"][q])
        f = FA[P["fill_in"][q]]
        for j in range(n - 1):
            f = G[gates[j % len(gates)]] @ f
            FA[1 + first + j] = f
            wf[first + j] += 1
    for t in range(len(ta) - 1, -1, -1):
        b = np.zeros(D)
        base = tp[t]
        J = jump_matrices(P, G, t)
        for sg in reversed(segs(t)):
            st, cnt, pat = int(P["seg_start"][sg]), int(P["seg_count"][sg]), int(P["seg_pattern"][sg])
            if pat & 0xff == 0:
                stride = (pat >> 8) & 0xff
                last = base + st + cnt * stride - 1
                if ti[last] >= 0:
                    b = b + inj[ti[last]]
                for c in range(cnt - 1, -1, -1):
                    j = base + st + (c + 1) * stride - 1
                    BA[j] = b
                    wb[j] += 1
                    b = J[pat >> 16].T @ b
            else:
                gates = pattern_gates(pat, P["seg_gate3"][sg])
                last = base + st + cnt * len(gates) - 1
                if ti[last] >= 0:
                    b = b + inj[ti[last]]
                for j in range(last, base + st - 1, -1):
                    BA[j] = b
                    wb[j] += 1
                    b = G[tg[j]].T @ b
        tadj[t] = b
    for q in range(len(P["fill_first"])):
        first, n = int(P["fill_first"][q]), int(P["fill_n"][q])
        gates = pattern_gates(int(P["fill_pattern"][q]), P["fill_gate3"][q])
        b = BA[first + n - 1]
        for j in range(n - 1, 0, -1):
            b = G[gates[j % len(gates)]].T @ b
            BA[first + j - 1] = b
            wb[first + j - 1] += 1
    return FA, BA, tadj, wf, wb


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_trunk_segments_rebuild_words(planlib, name):
    w = W.structured_workload(name)
    P = get_plan(planlib, w.seqs, w.model.K)
    tp = P["trunk_ptr"]
    nseg = 0
    for t in range(len(tp) - 1):
        word = segments_word(P, t)
        assert word == list(P["trunk_gates"][tp[t]:tp[t + 1]])
        nseg += P["seg_ptr"][t + 1] - P["seg_ptr"][t]
    # germ powers compress: far fewer segments than steps
    assert nseg * 4 < len(P["trunk_gates"])


def test_random_words_rejected_early(planlib):
    """Random words share only their first few levels: the plan is refused by
    the depth-by-depth prefix count, without building the whole trie (a
    10M-step list must be refused in well under a second)."""
    import time
    rng = np.random.default_rng(7)
    sl = W.random_list(20000, 6, 1, 1024, rng)
    t0 = time.perf_counter()
    P = get_plan(planlib, sl, 6)
    dt = time.perf_counter() - t0
    assert not P["used"]
    assert dt < 1.0, dt
    # a list whose words repeat is still planned (identical words share everything)
    words = [list(rng.integers(0, 6, size=200)) for _ in range(5)] * 40
    P = get_plan(planlib, W.from_words(words), 6)
    assert P["used"] and P["n_nodes"] <= 1 + 5 * 200 and P["sum_len"] == 200 * 200


@pytest.mark.parametrize("name,jump", [("c1", 8), ("c2", 8), ("c2", 4), ("c2", 16), ("c2", 2)])
def test_germ_power_jumps(planlib, name, jump):
    """Germ-power jumps (a run of a periodic pattern applied 2^e repetitions at
    a time by the matrix power) plus the fill tasks write every trunk state and
    adjoint exactly once, and give the values of the plain step-by-step
    sweeps up to rounding; injections land only where the chain stores."""
    w = W.structured_workload(name)
    G, rho = w.model.gates, w.model.rho
    D = G.shape[1]
    planlib.plan_set_jump(jump, 4)
    try:
        P = get_plan(planlib, w.seqs, w.model.K)
    finally:
        planlib.plan_set_jump(8, 3)
    assert P["used"] and len(P["fill_first"]) > 0 and P["jump_trunks"] > 0
    tp, ta, tg, ti = P["trunk_ptr"], P["trunk_anchor"], P["trunk_gates"], P["trunk_inj"]
    for t in range(len(ta)):
        assert segments_word(P, t) == list(tg[tp[t]:tp[t + 1]])
    rng = np.random.default_rng(3)
    inj = rng.standard_normal((len(P["inj_loc"]), D))
    FA, BA, tadj, wf, wb = chain_schedule(P, G, rho, inj)
    assert np.all(wf == 1) and np.all(wb == 1)
    # plain sweeps (levels in order; the anchors are states of earlier trunks)
    F = np.zeros((1 + len(tg), D))
    F[0] = rho
    B = np.zeros((len(tg), D))
    for t in range(len(ta)):
        f = F[0] if ta[t] < 0 else F[1 + ta[t]]
        for j in range(tp[t], tp[t + 1]):
            f = G[tg[j]] @ f
            F[1 + j] = f
    tadj0 = np.zeros_like(tadj)
    for t in range(len(ta) - 1, -1, -1):
        b = np.zeros(D)
        for j in range(tp[t + 1] - 1, tp[t] - 1, -1):
            if ti[j] >= 0:
                b = b + inj[ti[j]]
            B[j] = b
            b = G[tg[j]].T @ b
        tadj0[t] = b
    assert np.abs(FA - F).max() <= 1e-13 * np.abs(F).max()
    assert np.abs(BA - B).max() <= 1e-12 * np.abs(B).max()
    assert np.abs(tadj - tadj0).max() <= 1e-12 * np.abs(tadj0).max()
    # the chain is much shorter than the trunk: count chain mat-vecs of the longest trunk
    t = int(np.argmax(np.diff(tp)))
    chain = sum(int(P["seg_count"][sg]) if P["seg_pattern"][sg] & 0xff == 0
                else int(P["seg_count"][sg]) * int(P["seg_pattern"][sg] & 0xff)
                for sg in range(P["seg_ptr"][t], P["seg_ptr"][t + 1]))
    if name == "c2" and jump == 8:
        assert chain * 4 < tp[t + 1] - tp[t]


@pytest.mark.parametrize("name,jump", [("c1", 8), ("c2", 8), ("c2", 0)])
def test_trunk_ops(planlib, name, jump):
    """The trunk kernels' op lists: spans add up to the trunk, expanding the ops
    (a gate, or a jump standing for 2^e repetitions of the trunk's pattern)
    gives the trunk's word, and every state that receives an injection ends an
    op and carries its slot there."""
    w = W.structured_workload(name)
    planlib.plan_set_jump(jump, 3)
    try:
        P = get_plan(planlib, w.seqs, w.model.K)
    finally:
        planlib.plan_set_jump(8, 3)
    tp, tg, ti = P["trunk_ptr"], P["trunk_gates"], P["trunk_inj"]
    op = P["op_ptr"]
    n_jump_ops = 0
    for t in range(len(tp) - 1):
        word, pos = [], 0
        for o in range(op[t], op[t + 1]):
            d = int(P["op_desc"][o])
            span = (d >> 8) & 0xff
            if d & 0x80:
                n_jump_ops += 1
                e = d & 0x7f
                gates = pattern_gates(int(P["jump_pattern"][t]), P["jump_gate3"][t])
                assert span == (1 << e) * len(gates)
                word += gates * (1 << e)
                # no injection inside a jump
                assert np.all(ti[tp[t] + pos:tp[t] + pos + span - 1] < 0)
            else:
                assert span == 1
                word.append(d & 0x7f)
            pos += span
            assert P["op_slot"][o] == ti[tp[t] + pos - 1]
        assert pos == tp[t + 1] - tp[t]
        assert word == list(tg[tp[t]:tp[t + 1]])
    assert (n_jump_ops > 0) == (jump > 0)


@pytest.mark.parametrize("name,jump", [("c1", 8), ("c2", 8), ("c2", 0), ("multilevel", 8)])
def test_source_rows(planlib, name, jump):
    """The adjoints that reach stored states in source order: the row of an
    item or trunk is its position in the injection lists (none when anchored
    at rho, that is for the root slot's sources), so the sources of slot s
    are the consecutive rows inj_ptr[s] .. inj_ptr[s + 1] - 1."""
    rng = np.random.default_rng(5)
    planlib.plan_set_jump(jump, 3)
    try:
        if name == "multilevel":
            P = get_plan(planlib, multilevel_list(rng), 3, min_trunk=8, reanchor=4, ratio=1.0)
            assert P["n_levels"] >= 2
        else:
            w = W.structured_workload(name)
            P = get_plan(planlib, w.seqs, w.model.K)
    finally:
        planlib.plan_set_jump(8, 3)
    assert P["used"]
    ip, src, root = P["inj_ptr"], P["inj_src"], P["root_slot"]
    n_rows = int(ip[root])
    assert np.array_equal(P["item_src"] < 0, P["items"][:, 3] < 0)
    assert np.array_equal(P["trunk_src"] < 0, P["trunk_anchor"] < 0)
    rows = np.full(n_rows, -1)
    for q, z in enumerate(P["item_src"]):
        if z >= 0:
            assert src[z] == q and rows[z] < 0
            rows[z] = z
    for t, z in enumerate(P["trunk_src"]):
        if z >= 0:
            assert src[z] == -(t + 1) and rows[z] < 0
            rows[z] = z
    assert np.array_equal(rows, np.arange(n_rows))  # every row has exactly one writer
    # the root slot's sources are the trunks anchored at rho, which have no row
    assert sorted(-src[ip[root]:ip[root + 1]] - 1) == sorted(np.nonzero(P["trunk_anchor"] < 0)[0])


def multilevel_list(rng):
    """Two levels of trunks (a long common prefix, long branches below the
    re-anchoring depth) with items anchored on both."""
    base = list(rng.integers(0, 3, 40))
    words = [base + list(rng.integers(0, 3, int(rng.integers(20, 40)))) + list(rng.integers(0, 3, k))
             for k in range(6) for _ in range(3)]
    words += [base[:30 + k] for k in range(5)] + [[]]
    return W.from_words(words)


def crowded_list(rng, n_items=300):
    """A long shared prefix whose last state receives n_items sources."""
    base = list(rng.integers(0, 3, 48))
    words = [base + list(rng.integers(0, 3, int(rng.integers(1, 5)))) for _ in range(n_items)]
    return W.from_words(words + [base[:20], []])


def test_source_rows_crowded_state(planlib):
    """A slot with hundreds of sources: more rows than the injection kernel
    loads at once (eight per group of lanes)."""
    rng = np.random.default_rng(6)
    P = get_plan(planlib, crowded_list(rng), 3, min_trunk=24, reanchor=8, ratio=1.0)
    assert P["used"]
    assert np.diff(P["inj_ptr"]).max() > 192
