"""The GST fit around the GPU likelihood (thesis Sec. 6.3.1-6.3.2).

``run_fit`` chains the library's steps: linear-inversion estimates from the
bare experiments (``gst_lgst``), gauge optimization toward the targets
(``gst_gauge_optimize``), the starting parameters of the estimation mode (TP:
the estimate's free entries, its gates depolarized just enough that every
probability with a positive count is positive),
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


def cptp_start(effects: np.ndarray, K: int, D: int, eps: float = 1e-2, mix: float = 5e-2) -> np.ndarray:
    """CPTP parameters next to the targets: the state with Cholesky diagonal
    (1, mix, ..., mix) (|0..0> slightly mixed), the given first M - 1 effects (the
    targets' projectors: every probability then positive), and per gate a zero
    Hamiltonian part with the dissipator factor eps * identity (T = 0 is a
    stationary point of C = T T^dagger)."""
    m = D - 1
    d = int(round(np.sqrt(D)))
    gate = np.concatenate([np.zeros(m), np.full(m, eps), np.zeros(m * (m - 1))])
    A = np.zeros(D)
    A[0] = 1.0
    A[1:d] = mix
    return np.concatenate([A, np.asarray(effects)[:-1].ravel()] + [gate] * K)


# depolarizing strengths tried for a feasible TP start: 0, 2^-10, ..., 2^-1
SHRINK_STEPS = (0.0,) + tuple(2.0 ** -k for k in range(10, 0, -1))


def shrink_tp(theta: np.ndarray, D: int, M: int, K: int, delta: float) -> np.ndarray:
    """TP parameters with every gate followed by depolarizing of strength delta:
    rows 1.. of the transfer matrices times (1 - delta)."""
    th = np.array(theta, np.float64, copy=True)
    g0 = (D - 1) + (M - 1) * D
    th[g0:] *= (1.0 - delta)
    return th


def feasible_tp_start(ctx: api.Context, req: api.Request, theta: np.ndarray, n: int, M: int, K: int):
    """The first of the shrunk starts whose likelihood is finite on `req` (every
    probability with a positive count positive); returns (theta, delta)."""
    D = 4 ** n
    par = api.Parameterization(ctx, "tp", n, M, K)
    for delta in SHRINK_STEPS:
        th = shrink_tp(theta, D, M, K, delta)
        gs = par.forward(torch.as_tensor(th, device=ctx._dev()))
        obj, _, _ = req.eval(gs, want_probs=False, want_grad=False)
        F = float(obj.cpu())
        ctx.sync(raise_on_error=False)
        if np.isfinite(F):
            return th, delta
    raise RuntimeError("no feasible TP start")


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
    t0 = time.perf_counter()
    if requests is None:
        requests = []
        for e in stage_ends(stage_end):
            sub = seqs.subset(np.arange(e))
            requests.append(api.Request(ctx, n, K, M, sub.offsets, sub.gates, counts[:e]))
    sec["requests"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    if mode == "tp":   # gst_mlgst depolarizes an infeasible start itself
        theta0 = api.contract_tp(r, E, G)
        targets = None
    else:
        theta0 = cptp_start(target.effects, K, D)
        targets = torch.as_tensor(np.ascontiguousarray(target.gates), device=ctx._dev())
    sec["start"] = time.perf_counter() - t0
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
