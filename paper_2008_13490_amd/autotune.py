"""Tile autotuner for the batched tile kernels.

For each qubit count the tile kernels cut a request's length-sorted
sequences into tiles (a tile is the unit a workgroup or a wave takes from
the work queue and the unit of the partial sums) and run a persistent grid
of some workgroups per CU.  Both trade load balance and the per-tile
reduction against parallelism, and the best choice depends on the lengths.
The autotuner measures: it builds a request from a sample of the target
length distribution for every candidate policy (``gst_tune_set`` before the
request is created), times evaluations with gradient, and keeps the fastest.
The chosen policy is fixed into the requests created afterwards, so results
stay the same alone and in a batch.
"""
from __future__ import annotations

import itertools
import time
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

from . import api
from . import workloads as W

# candidate (sequences per tile, workgroups per CU; 0 = as many as fit)
CANDIDATES = {
    1: [(64, 0), (128, 0), (256, 0), (64, 1)],
    2: [(16, 0), (32, 0), (64, 0), (16, 1), (32, 1)],
    3: [(4, 0), (8, 0), (16, 0), (32, 0)],
}


def _time_batch(ctx, batch, reps: int) -> float:
    import torch
    batch.run()  # warm-up (and workspace growth)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.run()
    ctx.sync()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(ctx: api.Context, samples: Dict[int, Tuple[int, int, int, int]], reps: int = 3, seed: int = 1,
         candidates: Optional[Dict[int, Sequence[Tuple[int, int]]]] = None, apply: bool = True) -> dict:
    """samples: n_qubits -> (n_requests, S, lmin, lmax): a batch of that many
    requests (own gate sets, random words) to tune on.  It should fill the
    GPU several times over: the policy of a persistent launch matters over
    many tiles, not over one round.  Returns {n_qubits: {"best": (tile,
    bpc), "ms": {candidate: ms}}} and, with ``apply``, leaves the best policy
    set on ``ctx`` (the default stays unless another is >3% faster)."""
    cands = candidates or CANDIDATES
    out = {}
    kind = {1: "1q", 2: "2q", 3: "3q"}
    for n, (n_req, S, lmin, lmax) in samples.items():
        rng = np.random.default_rng(seed + n)
        data = []
        for _ in range(n_req):
            gs = W.noisy_gateset(kind[n], W.LAMBDA, W.SIGMA, rng)
            sl = W.random_list(S, gs.K, lmin, lmax, rng)
            counts = W.sample_counts(np.full((S, gs.M), 1.0 / gs.M), W.N_SHOTS, rng)
            data.append((gs, sl, counts))
        thetas = [api.DeviceGateSet.from_numpy(n, gs.rho, gs.effects, gs.gates) for gs, _, _ in data]
        ms = {}
        for tile, bpc in cands[n]:
            api.tune_set(ctx, n, tile, bpc)
            reqs = [api.Request(ctx, n, gs.K, gs.M, sl.offsets, sl.gates, c) for gs, sl, c in data]
            b = api.Batch(ctx, reqs, thetas, want_probs=False, want_grad=True)
            ms[(tile, bpc)] = _time_batch(ctx, b, reps) * 1e3
            b.close()
            for r in reqs:
                r.close()
        default = tuple(cands[n][0])
        best = min(ms, key=ms.get)
        if ms[best] > 0.97 * ms[default]:
            best = default
        api.tune_set(ctx, n, *(best if apply else (0, 0)))
        out[n] = {"best": best, "ms": {f"{t}x{b}": v for (t, b), v in ms.items()}}
    return out
