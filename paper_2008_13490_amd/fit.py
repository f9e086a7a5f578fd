"""The GST fit around the GPU likelihood (thesis Sec. 6.3.1-6.3.2).

``run_fit`` chains the library's steps: linear-inversion estimates from the
bare experiments (``gst_lgst``), gauge optimization toward the targets
(``gst_gauge_optimize``), the starting parameters of the estimation mode,
iterative MLGST on lists of growing length with the evaluations on the GPU
(``gst_mlgst``), and a final gauge optimization of the estimate.  Every
number is computed by ``libgst.so``; this module only sequences the calls.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import api


@dataclasses.dataclass
class FitResult:
    theta: np.ndarray               # parameters of the estimation mode
    rho: np.ndarray                 # the estimate after the final gauge optimization
    effects: np.ndarray
    gates: np.ndarray
    reports: List[dict]             # per MLGST stage
    lgst: tuple                     # (rho, E, G) of LGST after gauge optimization
    seconds: dict                   # wall time per step


def cptp_start(effects: np.ndarray, K: int, D: int, eps: float = 1e-3) -> np.ndarray:
    """CPTP parameters next to the targets: the state e_0 (|0..0>), the given
    first M - 1 effects, and per gate a zero Hamiltonian part with the dissipator
    factor eps * identity (T = 0 is a stationary point of C = T T^dagger)."""
    m = D - 1
    gate = np.concatenate([np.zeros(m), np.full(m, eps), np.zeros(m * (m - 1))])
    A = np.zeros(D)
    A[0] = 1.0
    return np.concatenate([A, np.asarray(effects)[:-1].ravel()] + [gate] * K)


def stage_ends(stage_end: List[int]) -> List[int]:
    """The distinct ends of the MLGST stages (the first stage, LGST's own list,
    is contained in the next)."""
    out = []
    for e in stage_end[1:]:
        if not out or e != out[-1]:
            out.append(e)
    return out


def run_fit(ctx: api.Context, seqs, counts, stage_end, prep_fids, meas_fids, target, mode: str = "tp",
            max_iter: int = 500, gtol: float = 1e-9, requests: Optional[list] = None) -> FitResult:
    """``seqs`` (SeqList), ``counts`` [S, M]: the whole list, its stages ending at
    ``stage_end`` (stage 0 = the LGST words); ``target``: a gate set with the
    ideal gates (rho, effects, gates arrays).  ``requests``: resident requests of
    the stages, if already created."""
    n, M, K = target.n_qubits, target.M, target.K
    D = 4 ** n
    sec = {}
    t0 = time.perf_counter()
    e0 = stage_end[0]
    r, E, G = api.lgst(n, M, K, seqs.offsets[:e0 + 1], seqs.gates[:seqs.offsets[e0]], counts[:e0], prep_fids,
                       meas_fids)
    sec["lgst"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    r, E, G, _, _ = api.gauge_optimize(n, r, E, G, target.rho, target.effects, target.gates)
    sec["gauge_lgst"] = time.perf_counter() - t0
    if mode == "tp":
        theta0 = api.contract_tp(r, E, G)
        targets = None
    else:
        theta0 = cptp_start(E, K, D)
        targets = torch.as_tensor(np.ascontiguousarray(target.gates), device=ctx._dev())
    t0 = time.perf_counter()
    if requests is None:
        requests = []
        for e in stage_ends(stage_end):
            sub = seqs.subset(np.arange(e))
            requests.append(api.Request(ctx, n, K, M, sub.offsets, sub.gates, counts[:e]))
    sec["requests"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    theta, reports = api.mlgst(ctx, requests, mode, theta0, targets, max_iter=max_iter, gtol=gtol)
    sec["mlgst"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    par = api.Parameterization(ctx, mode, n, M, K, targets)
    gs = par.forward(torch.as_tensor(theta, device=ctx._dev()))
    rf, Ef, Gf = (t.cpu().numpy() for t in (gs.rho, gs.effects, gs.gates))
    rf, Ef, Gf, _, _ = api.gauge_optimize(n, rf, Ef, Gf, target.rho, target.effects, target.gates)
    sec["gauge_final"] = time.perf_counter() - t0
    return FitResult(theta, rf, Ef, Gf, reports, (r, E, G), sec)
