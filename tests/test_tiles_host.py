"""The batch kernels' tile lists, built by the library's host code on the CPU.

A persistent tile kernel writes each tile's partial sums into row `local` of
its own request's slab.  For random batches this checks that the list the
library builds names every row of every request exactly once, never a row at
or beyond the request's tile count, that tiles come longest first, and that
the library's own pre-launch check rejects a corrupted list."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_13490_amd", "csrc")


@pytest.fixture(scope="module")
def tiles(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tiles") / "libtilesprobe.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(ROOT, "tests", "tiles_probe.cpp"), os.path.join(CSRC, "gst_tiles.cpp"), "-o", out],
                   check=True)
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.tiles_batch.argtypes = [ctypes.c_int, P, P, P, P, ctypes.c_long, ctypes.c_long, ctypes.c_long]
    lib.tiles_batch.restype = ctypes.c_long
    lib.tiles_msg.restype = ctypes.c_char_p
    return lib


def run_batch(lib, lengths, tile_seqs, corrupt=-1, corrupt_local=0):
    offs = [np.concatenate([[0], np.cumsum(L)]).astype(np.int64) for L in lengths]
    ptrs = (ctypes.c_void_p * len(offs))(*[o.ctypes.data for o in offs])
    S = np.array([len(L) for L in lengths], np.int64)
    ts = np.array(tile_seqs, np.int64)
    cap = int(sum((s + t - 1) // t for s, t in zip(S, ts)))
    out = np.zeros((max(cap, 1), 4), np.int64)
    n = lib.tiles_batch(len(offs), ptrs, S.ctypes.data, ts.ctypes.data, out.ctypes.data, cap, corrupt, corrupt_local)
    return n, out[:max(n, 0)], offs, lib.tiles_msg().decode()


def test_random_batches_cover_every_slab_row_once(tiles):
    rng = np.random.default_rng(11)
    for trial in range(40):
        n_req = int(rng.integers(1, 9))
        lengths = [rng.integers(0, 300, size=int(rng.integers(0, 600))) for _ in range(n_req)]
        tile_seqs = [int(rng.choice([1, 16, 32, 64, 128])) for _ in range(n_req)]
        n, t, offs, msg = run_batch(tiles, lengths, tile_seqs)
        assert n >= 0, msg
        for r in range(n_req):
            S = len(lengths[r])
            n_tiles = (S + tile_seqs[r] - 1) // tile_seqs[r]
            mine = t[t[:, 0] == r]
            assert sorted(mine[:, 1].tolist()) == list(range(n_tiles))   # every row once, all < n_tiles
            covered = np.zeros(S, int)
            for _, local, q0, q1 in mine:
                assert q1 - q0 == min(tile_seqs[r], S - q0) and q0 == local * tile_seqs[r]
                covered[q0:q1] += 1
            assert (covered == 1).all()
        # longest tiles first
        cost = []
        for r, local, q0, q1 in t:
            L = np.sort(lengths[r])[::-1]
            cost.append(int(L[q0:q1].sum()))
        assert all(a >= b for a, b in zip(cost, cost[1:]))


@pytest.mark.parametrize("bad", ["beyond", "negative", "duplicate"])
def test_pre_launch_check_rejects_a_corrupted_list(tiles, bad):
    lengths = [np.arange(100) % 37, np.arange(40) % 11]
    n, t, _, _ = run_batch(tiles, lengths, [16, 16])
    assert n == 7 + 3
    victim = int(np.nonzero(t[:, 0] == 1)[0][0])
    local = {"beyond": 3, "negative": -1, "duplicate": int(t[np.nonzero(t[:, 0] == 1)[0][1], 1])}[bad]
    n2, _, _, msg = run_batch(tiles, lengths, [16, 16], corrupt=victim, corrupt_local=local)
    assert n2 == -1 and msg
