"""The grouped-chain sharing plan (csrc/gst_plan64.*), executed on the CPU.

The library's plan builder runs here through a small probe; a numpy
interpreter executes the plan the way the three-qubit kernels do (chains of a
tile stepped together level by level, readouts per seed slot, the reverse
sweep with seeds and the adjoints chains deliver to their anchors, the
gradient from the (adjoint, parent state) records grouped by gate) and the
result is compared with the oracle.  This pins the plan's bookkeeping before
any kernel runs it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_13490_amd", "csrc")
TC = 16


@pytest.fixture(scope="module")
def plib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("plan64") / "libplan64probe.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(ROOT, "tests", "plan64_probe.cpp"), os.path.join(CSRC, "gst_plan64.cpp"), "-o", out],
                   check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.plan64_build.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, P]
    lib.plan64_tiles.argtypes = [P] * 9
    lib.plan64_events.argtypes = [P] * 7
    lib.plan64_records.argtypes = [P] * 6
    lib.plan64_ts.argtypes = [P] * 2
    lib.plan64_set_max_events.argtypes = [ctypes.c_int]
    return lib


def get_plan(lib, sl, K, ratio=0.5, fill=0.0, chunk=8192):
    off = np.ascontiguousarray(sl.offsets, np.int64)
    g = np.ascontiguousarray(sl.gates if sl.gates.size else np.zeros(1, np.uint8), np.uint8)
    z = np.zeros(15, np.int64)
    lib.plan64_build(off.ctypes.data, g.ctypes.data, sl.S, int(K), ratio, fill, chunk, z.ctypes.data)
    used, n_rows, T, L, C, NS, NE, NR, NW, TS, root_slot, NRC, NN, NCH, NTS = [int(x) for x in z]
    P = dict(used=used, n_rows=n_rows, n_tiles=T, n_levels=L, n_chains=C, n_slots=NS, root_slot=root_slot,
             n_nodes=NN)
    if not used:
        return P
    a = dict(level_tile_ptr=np.zeros(L + 1, np.int64), row0=np.zeros(T, np.int64), len=np.zeros(T, np.int32),
             cols=np.zeros(T, np.int32), word=np.zeros(T, np.int64), tev=np.zeros(T, np.int64),
             anchor=np.zeros(T * TC, np.int64), chain=np.zeros(T * TC, np.int64), words=np.zeros(max(NW, 1), np.uint8))
    lib.plan64_tiles(*[a[k].ctypes.data for k in ["level_tile_ptr", "row0", "len", "cols", "word", "tev", "anchor",
                                                  "chain", "words"]])
    b = dict(ev_ptr=np.zeros(TS + 1, np.int64), ev_col=np.zeros(max(NE, 1), np.int32),
             ev_src=np.zeros(max(NE, 1), np.int64), slot_row=np.zeros(NS, np.int64),
             slot_ptr=np.zeros(NS + 1, np.int64), slot_seq=np.zeros(sl.S, np.int64),
             root_chains=np.zeros(max(NRC, 1), np.int64))
    lib.plan64_events(*[b[k].ctypes.data for k in ["ev_ptr", "ev_col", "ev_src", "slot_row", "slot_ptr", "slot_seq",
                                                   "root_chains"]])
    c = dict(rec_b=np.zeros(max(NR, 1), np.int64), rec_f=np.zeros(max(NR, 1), np.int64),
             rec_gate_ptr=np.zeros(K + 1, np.int64), chunk_beg=np.zeros(max(NCH, 1), np.int64),
             chunk_end=np.zeros(max(NCH, 1), np.int64), gate_chunk_ptr=np.zeros(K + 1, np.int64))
    lib.plan64_records(*[c[k].ctypes.data for k in ["rec_b", "rec_f", "rec_gate_ptr", "chunk_beg", "chunk_end",
                                                    "gate_chunk_ptr"]])
    d = dict(ts_tile=np.zeros(max(NTS, 1), np.int64), ts_step=np.zeros(max(NTS, 1), np.int32))
    lib.plan64_ts(d["ts_tile"].ctypes.data, d["ts_step"].ctypes.data)
    P.update(a)
    P.update(b)
    P.update(c)
    P.update(d)
    P["root_chains"] = P["root_chains"][:NRC]
    P["n_events"], P["n_records"] = NE, NR
    return P


def run_plan(P, gs, counts):
    """The plan executed with numpy: (objective, probs, gradient)."""
    D, M, K = gs.D, gs.M, gs.K
    G, E, rho = gs.gates, gs.effects, gs.rho
    FA = np.zeros((P["n_rows"], D))
    BA = np.zeros((P["n_rows"], D))
    FA[0] = rho
    ltp = P["level_tile_ptr"]
    for lev in range(P["n_levels"]):
        for ti in range(ltp[lev], ltp[lev + 1]):
            V = FA[P["anchor"][ti * TC:(ti + 1) * TC]].T.copy()
            w0 = P["word"][ti]
            for t in range(P["len"][ti]):
                V = G[P["words"][w0 + t]] @ V
                FA[P["row0"][ti] + t * TC: P["row0"][ti] + (t + 1) * TC] = V.T
    S = len(P["slot_seq"])
    probs = np.zeros((S, M))
    INJ = np.zeros((P["n_slots"] + P["n_chains"], D))
    F = 0.0
    dE = np.zeros((M, D))
    for x in range(P["n_slots"]):
        f = FA[P["slot_row"][x]]
        p = E @ f
        dps = np.zeros(M)
        for s in P["slot_seq"][P["slot_ptr"][x]:P["slot_ptr"][x + 1]]:
            probs[s] = p
            N = counts[s].astype(float)
            F -= np.sum(np.where(N > 0, N * np.log(np.where(N > 0, p, 1.0)), 0.0))
            dps += np.where(N > 0, -N / np.where(N > 0, p, 1.0), 0.0)
        INJ[x] = E.T @ dps
        dE += np.outer(dps, f)
    for lev in reversed(range(P["n_levels"])):
        for ti in range(ltp[lev], ltp[lev + 1]):
            Bm = np.zeros((D, TC))
            w0 = P["word"][ti]
            for t in reversed(range(P["len"][ti])):
                e = P["tev"][ti] + t
                for k in range(P["ev_ptr"][e], P["ev_ptr"][e + 1]):
                    Bm[:, P["ev_col"][k]] += INJ[P["ev_src"][k]]
                BA[P["row0"][ti] + t * TC: P["row0"][ti] + (t + 1) * TC] = Bm.T
                Bm = G[P["words"][w0 + t]].T @ Bm
            for c in range(P["cols"][ti]):
                INJ[P["n_slots"] + P["chain"][ti * TC + c]] = Bm[:, c]
    # the gradient GEMM as the kernel runs it: chunks of tile-steps of one gate
    # (each sixteen records: the tile's rows at step t against the rows before)
    dG = np.zeros((K, D, D))
    for k in range(K):
        for ch in range(P["gate_chunk_ptr"][k], P["gate_chunk_ptr"][k + 1]):
            for x in range(P["chunk_beg"][ch], P["chunk_end"][ch]):
                ti, t = P["ts_tile"][x], P["ts_step"][x]
                rb = P["row0"][ti] + t * TC + np.arange(TC)
                rf = (P["row0"][ti] + (t - 1) * TC + np.arange(TC)) if t > 0 else P["anchor"][ti * TC:(ti + 1) * TC]
                assert P["words"][P["word"][ti] + t] == k
                dG[k] += BA[rb].T @ FA[rf]
    drho = np.zeros(D)
    if P["root_slot"] >= 0:
        drho += INJ[P["root_slot"]]
    for ch in P["root_chains"]:
        drho += INJ[P["n_slots"] + ch]
    return F, probs, np.concatenate([drho, dE.ravel(), dG.ravel()])


def small_structured(kind, seed, n_fid, germ_spec, powers, dup=True):
    rng = np.random.default_rng(seed)
    gs = W.noisy_gateset(kind, 1e-3, 0.02, rng)
    fids = W.shortlex_words((1, 2), n_fid)
    germs = W.random_germs(gs.K, germ_spec, rng)
    sl = W.structured_list(fids, fids, germs, powers)
    words = [list(sl.word(s)) for s in range(sl.S)]
    if dup:
        words += [words[3], [], words[len(words) // 2], []]   # duplicate words and empty words
    sl = W.from_words(words)
    return gs, sl


@pytest.mark.parametrize("kind,n_fid,spec,powers", [
    ("3q", 6, [(2, 3), (3, 3)], [1, 2, 4, 8]),
    ("2q", 7, [(2, 2), (3, 2)], [1, 2, 4, 8, 16]),
    ("1q", 6, [(3, 1)], [1, 2, 4, 8, 16, 32]),
])
def test_plan64_executes_to_the_oracle(oracle_lib, plib, kind, n_fid, spec, powers):
    gs, sl = small_structured(kind, 5, n_fid, spec, powers)
    rng = np.random.default_rng(6)
    p_true = oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates)
    counts = W.sample_counts(p_true, 1000, rng)
    # small lists: few chains per group, tiles partly empty; the policy is not under
    # test here, nor the event bound of the three-qubit kernels (K <= 5)
    plib.plan64_set_max_events(64)
    try:
        P = get_plan(plib, sl, gs.K, ratio=10.0, fill=0.0)
    finally:
        plib.plan64_set_max_events(6)
    assert P["used"]
    assert P["n_nodes"] - 1 < 0.5 * int(sl.offsets[-1])
    F, p, g = run_plan(P, gs, counts)
    F_or, p_or, g_or, _, rc = oracle_lib.loglik(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates, counts)
    assert rc == 0
    assert np.abs(p - p_or).max() <= 1e-12 * np.abs(p_or).max()
    assert abs(F - F_or) <= 1e-10 * abs(F_or)
    assert np.abs(g - g_or).max() <= 1e-10 * np.abs(g_or).max()


def test_plan64_structure(plib):
    """Every trie node owns one live row; every record's rows are live; tiles
    hold one word; events name existing INJ rows; chains deliver once."""
    gs, sl = small_structured("3q", 7, 6, [(2, 3), (3, 4)], [1, 2, 4, 8, 16])
    P = get_plan(plib, sl, gs.K, fill=0.0)
    assert P["used"]
    T = P["n_tiles"]
    live = np.zeros(P["n_rows"], bool)
    for ti in range(T):
        for c in range(P["cols"][ti]):
            live[P["row0"][ti] + np.arange(P["len"][ti]) * TC + c] = True
    assert live.sum() == P["n_nodes"] - 1
    assert live[P["rec_b"]].all() and (live[P["rec_f"]] | (P["rec_f"] == 0)).all()
    assert len(P["rec_b"]) == P["n_nodes"] - 1 and len(set(P["rec_b"].tolist())) == len(P["rec_b"])
    assert (P["ev_src"][:P["n_events"]] < P["n_slots"] + P["n_chains"]).all()
    chains = P["chain"][P["chain"] >= 0]
    assert sorted(chains.tolist()) == list(range(P["n_chains"]))
    # every chain delivers to exactly one anchor: an event or the root
    delivered = P["ev_src"][:P["n_events"]]
    delivered = delivered[delivered >= P["n_slots"]] - P["n_slots"]
    assert sorted(delivered.tolist() + P["root_chains"].tolist()) == list(range(P["n_chains"]))
    # the column table: per tile-step, byte c < 15 counts the events of columns
    # <= c (events ascend by column), byte 15 is the most events of one column
    plib.plan64_cend.restype = ctypes.c_int64
    plib.plan64_cend.argtypes = [ctypes.c_void_p]
    TS = len(P["ev_ptr"]) - 1
    assert plib.plan64_cend(None) == TS * 16
    cend = np.zeros(TS * 16, np.uint8)
    plib.plan64_cend(cend.ctypes.data)
    cend = cend.reshape(TS, 16).astype(np.int64)
    for ts in range(TS):
        cols = P["ev_col"][P["ev_ptr"][ts]:P["ev_ptr"][ts + 1]]
        assert (np.diff(cols) >= 0).all()
        per = np.bincount(cols, minlength=16)
        assert (cend[ts, :15] == np.cumsum(per)[:15]).all()
        assert cend[ts, 15] == per.max()
    # anchors of level-l tiles lie on tiles of lower levels
    ltp = P["level_tile_ptr"]
    for lev in range(P["n_levels"]):
        lo = P["row0"][ltp[lev]] if ltp[lev] < T else P["n_rows"]
        for ti in range(ltp[lev], ltp[lev + 1]):
            assert (P["anchor"][ti * TC:ti * TC + P["cols"][ti]] < lo).all()


def test_plan64_default_options_take_the_test_lists(plib):
    """The library's default options (event bound of the kernels included)
    accept the structured three-qubit lists of the GPU tests."""
    import test_gpu_3q as T3
    for args in (dict(), dict(seed=8, n_fid=6, powers=(1, 2, 4, 8))):
        gs, sl, _ = T3._structured_3q(**args)
        assert get_plan(plib, sl, gs.K)["used"]


def test_plan64_refuses_random_lists(plib):
    rng = np.random.default_rng(8)
    sl = W.random_list(400, 5, 1, 80, rng)
    assert not get_plan(plib, sl, 5)["used"]


@pytest.mark.slow
def test_plan64_c4_statistics(plib):
    w = W.structured_workload("c4")
    P = get_plan(plib, w.seqs, w.model.K)
    assert P["used"]
    # one long level: the critical path of the sweeps is about one germ power chain
    ltp = P["level_tile_ptr"]
    crit = sum(int(P["len"][ltp[l]:ltp[l + 1]].max()) for l in range(P["n_levels"]))
    assert crit <= int(np.diff(w.seqs.offsets).max()) + 64
    live = P["n_nodes"] - 1
    # far fewer rows than steps, tiles mostly full
    assert live < int(w.seqs.offsets[-1]) / 20
    assert live >= 0.75 * (P["n_rows"] - 1)
