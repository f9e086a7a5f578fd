"""The oracle over a long sequence list in parallel (test helper).

The list is cut into contiguous shards of sequences; each spawned process
runs the unchanged oracle on its shard, and the shard results are put
together in ascending order: probabilities concatenated, objectives and
gradients added shard by shard.  Nothing here touches the GPU."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def _shard(args):
    import oracle
    rho, E, G, offsets, gates, counts = args
    F, p, g, nbad, rc = oracle.loglik(rho, E, G, offsets, gates, counts)
    return F, p, g, rc


def loglik_sharded(rho, E, G, offsets, gates, counts, workers: int = 0):
    """(F, p [S, M], grad) of the whole list, shards summed in ascending order."""
    S = len(offsets) - 1
    workers = workers or min(16, os.cpu_count() or 1)
    n = max(1, min(workers * 4, S))
    cuts = np.linspace(0, S, n + 1).astype(np.int64)
    jobs = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        off = np.ascontiguousarray(offsets[a:b + 1] - offsets[a])
        gts = np.ascontiguousarray(gates[offsets[a]:offsets[b]])
        jobs.append((rho, E, G, off, gts, np.ascontiguousarray(counts[a:b])))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_shard, jobs))
    assert all(rc == 0 for *_, rc in parts)
    F = 0.0
    g = np.zeros_like(parts[0][2])
    for Fi, _, gi, _ in parts:
        F += Fi
        g += gi
    return F, np.concatenate([pi for _, pi, _, _ in parts]), g
