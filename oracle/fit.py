"""The fit around the likelihood (test infrastructure only).

Thesis Sec. 6.3.1: the objects of Eq. GSTFullFiducialsGerms are determined only
up to the GST gauge (E -> E M^-1, G -> M G M^-1, rho -> M rho).  The fit starts
from linear-inversion GST: the matrix AB of the frequencies of the bare
experiments <<E_J| F_i^(M) F_j^(P) |rho>> (rows J + N i, columns j) and, per
gate, the same with G_k between the fiducials; a pseudo-inverse of AB turns
them into estimates of rho, E_J and G_k in one gauge.  The estimates are then
refined by maximizing the likelihood on lists of growing length (iterative
MLGST), and finally brought close to the target gates by a gauge
transformation (gauge optimization).

Plain definitions with numpy / scipy as the library steps:

* lgst: AB = U S V^T truncated to rank D; with Ahat = U_D^T AB V_D,
  G_k = Ahat^-1 U_D^T B_k V_D, rho = Ahat^-1 U_D^T b (b = the column of the
  empty preparation fiducial), E_J = c_J^T V_D (c_J = the row block of the
  empty measurement fiducial).  Each singular pair is signed so that the
  largest-magnitude entry of its V column is positive.
* gauge_objective / gauge_opt: sum_k ||M G_k M^-1 - T_k||_F^2 + w (||M rho -
  rho_T||^2 + sum_m ||M^-T e_m - e_T,m||^2), minimized over M with scipy's
  L-BFGS-B from the least-squares solution of the same relations multiplied
  through by M (linear in M).
* contract_tp: the TP parameters of an estimate (the entries TP leaves free).
* mlgst: each stage minimizes the negative log-likelihood (the oracle's
  loglik) of its sequences, in the chosen parameterization, with the plain
  L-BFGS below (its line search treats a step into p <= 0, objective +inf, as
  too long), starting from the previous stage's parameters; a start with
  some p <= 0 where N > 0 is first moved inward (feasible_tp_start: the gates
  depolarized; feasible_cptp_start: the effects mixed with 1/M).  The likelihood is
  bounded only where every sequence's probabilities sum to one (TP, CPTP).
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np
import scipy.optimize as so

from . import binding as B
from . import params as PR


def _word_rows(offsets, gates) -> Dict[Tuple[int, ...], int]:
    rows = {}
    for s in range(len(offsets) - 1):
        w = tuple(int(g) for g in gates[offsets[s]:offsets[s + 1]])
        rows.setdefault(w, s)
    return rows


def frequencies(counts) -> np.ndarray:
    c = np.asarray(counts, np.float64)
    n = c.sum(axis=1, keepdims=True)
    return c / np.where(n > 0, n, 1.0)


def ab_matrices(offsets, gates, freqs, prep_fids, meas_fids, K):
    """AB [N n_meas, n_prep] and B_k [K, N n_meas, n_prep] of the frequencies
    [S, N] of the listed sequences."""
    rows = _word_rows(offsets, gates)
    f = np.asarray(freqs, np.float64)
    M = f.shape[1]
    nm, npp = len(meas_fids), len(prep_fids)
    AB = np.zeros((M * nm, npp))
    Bk = np.zeros((K, M * nm, npp))
    for i, fq in enumerate(meas_fids):
        for j, fp in enumerate(prep_fids):
            AB[M * i:M * (i + 1), j] = f[rows[tuple(fp) + tuple(fq)]]
            for k in range(K):
                Bk[k, M * i:M * (i + 1), j] = f[rows[tuple(fp) + (k,) + tuple(fq)]]
    return AB, Bk


def lgst(offsets, gates, counts, prep_fids, meas_fids, n_qubits: int, K: int):
    """Linear-inversion estimates (rho [D], E [M, D], G [K, D, D]) in the gauge of
    the truncated singular vectors, from outcome counts."""
    return lgst_freqs(offsets, gates, frequencies(counts), prep_fids, meas_fids, n_qubits, K)


def lgst_freqs(offsets, gates, freqs, prep_fids, meas_fids, n_qubits: int, K: int):
    D = 4 ** n_qubits
    AB, Bk = ab_matrices(offsets, gates, freqs, prep_fids, meas_fids, K)
    M = AB.shape[0] // len(meas_fids)
    U, s, Vt = np.linalg.svd(AB, full_matrices=False)
    U, V = U[:, :D], Vt[:D].T
    for c in range(D):
        if V[np.argmax(np.abs(V[:, c])), c] < 0:
            U[:, c] = -U[:, c]
            V[:, c] = -V[:, c]
    Ahat_inv = np.linalg.inv(U.T @ AB @ V)
    G = np.array([Ahat_inv @ U.T @ Bk[k] @ V for k in range(K)])
    j0 = [tuple(f) for f in prep_fids].index(())
    i0 = [tuple(f) for f in meas_fids].index(())
    rho = Ahat_inv @ U.T @ AB[:, j0]
    E = AB[M * i0:M * (i0 + 1), :] @ V
    return rho, E, G


def gauge_transform(rho, E, G, Mg):
    Mi = np.linalg.inv(Mg)
    return Mg @ rho, E @ Mi, np.array([Mg @ g @ Mi for g in G])


def gauge_objective(x, rho, E, G, rT, ET, GT, w: float):
    """Objective and gradient with respect to the entries of M (row-major)."""
    D = rho.shape[0]
    Mg = x.reshape(D, D)
    Mi = np.linalg.inv(Mg)
    f = 0.0
    gM = np.zeros((D, D))
    for g, t in zip(G, GT):
        R = Mg @ g @ Mi - t
        f += np.sum(R * R)
        # d/dM ||M g M^-1 - t||^2 = 2 (R (g M^-1)^T - X^T R M^-T), X = M g M^-1
        X = Mg @ g @ Mi
        gM += 2 * (R @ (g @ Mi).T - X.T @ R @ Mi.T)
    r = Mg @ rho - rT
    f += w * np.dot(r, r)
    gM += w * 2 * np.outer(r, rho)
    for e, t in zip(E, ET):
        q = Mi.T @ e - t            # the effect as a column: (e^T M^-1)^T
        f += w * np.dot(q, q)
        # d(M^-T e) = -M^-T dM^T M^-T e
        gM += -w * 2 * np.outer(Mi.T @ e, Mi @ q)
    return f, gM.reshape(-1)


def gauge_linear_start(rho, E, G, rT, ET, GT, w: float = 1.0) -> np.ndarray:
    """X minimizing the quadratic sum_k ||X G_k - T_k X||_F^2 + w (||X rho - rho_T||^2
    + sum_m ||X^T e_T,m - e_m||^2) (the gauge relations multiplied through by X):
    linear least squares over the entries of X."""
    D = rho.shape[0]
    rows, rhs = [], []
    for g, t in zip(G, GT):
        for a in range(D):
            for b in range(D):
                r = np.zeros((D, D))
                r[a, :] += g[:, b]          # (X g)_ab = sum_c X_ac g_cb
                r[:, b] -= t[a, :]          # (t X)_ab = sum_c t_ac X_cb
                rows.append(r.reshape(-1))
                rhs.append(0.0)
    sw = np.sqrt(w)
    for i in range(D):
        r = np.zeros((D, D))
        r[i, :] = rho
        rows.append(sw * r.reshape(-1))
        rhs.append(sw * rT[i])
    for e, t in zip(E, ET):
        for j in range(D):
            r = np.zeros((D, D))
            r[:, j] = t                     # (X^T t)_j = sum_i X_ij t_i
            rows.append(sw * r.reshape(-1))
            rhs.append(sw * e[j])
    x, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
    return x.reshape(D, D)


def gauge_opt(rho, E, G, rT, ET, GT, w: float = 1.0, gtol: float = 1e-13, maxiter: int = 2000, start=None):
    """From the linear start (or `start`), scipy's L-BFGS-B on gauge_objective."""
    D = rho.shape[0]
    X0 = gauge_linear_start(rho, E, G, rT, ET, GT, w) if start is None else start
    res = so.minimize(gauge_objective, np.asarray(X0, np.float64).reshape(-1), args=(rho, E, G, rT, ET, GT, w), jac=True,
                      method="L-BFGS-B", options={"gtol": gtol, "ftol": 1e-15, "maxiter": maxiter, "maxcor": 10})
    Mg = res.x.reshape(D, D)
    return Mg, gauge_transform(rho, E, G, Mg), res.fun


def contract_tp(rho, E, G) -> np.ndarray:
    """TP parameters of the nearest TP point in the entries that TP fixes: the free
    entries as they are (rho[1:], the first M - 1 effects, rows 1.. of the gates);
    the map sets rho[0], the last effect and the first rows."""
    return np.concatenate([rho[1:], E[:-1].ravel(), G[:, 1:, :].ravel()])


def mode_is_tp(mode) -> bool:
    return PR.mode_id(mode) == PR.TP


def feasible_cptp_start(theta, n: int, M: int, K: int, G0, offsets, gates, counts):
    """The CPTP start with its free effects mixed with the uniform POVM,
    e_m <- (1 - delta) e_m + delta vec(1)/M, by the smallest delta in 0, 2^-10,
    ..., 1/2 whose likelihood is finite (gates and state are physical)."""
    D = 4 ** n
    u = np.zeros(D)
    u[0] = np.sqrt(np.sqrt(D)) / M
    for delta in [0.0] + [2.0 ** -k for k in range(10, 0, -1)]:
        th = np.array(theta, np.float64, copy=True)
        e = th[D:D + (M - 1) * D].reshape(M - 1, D)
        th[D:D + (M - 1) * D] = ((1.0 - delta) * e + delta * u[None, :]).reshape(-1)
        F, _ = nll_in_mode(th, "cptp", n, M, K, G0, offsets, gates, counts)
        if np.isfinite(F):
            return th, delta
    raise RuntimeError("no feasible CPTP start")


def feasible_tp_start(theta, n: int, M: int, K: int, offsets, gates, counts):
    """The TP start with every gate followed by depolarizing of the smallest
    strength delta in 0, 2^-10, 2^-9, ..., 1/2 (rows 1.. of the transfer matrices
    times 1 - delta) whose likelihood is finite; returns (theta, delta)."""
    D = 4 ** n
    g0 = (D - 1) + (M - 1) * D
    for delta in [0.0] + [2.0 ** -k for k in range(10, 0, -1)]:
        th = np.array(theta, np.float64, copy=True)
        th[g0:] = th[g0:] * (1.0 - delta)
        F, _ = nll_in_mode(th, "tp", n, M, K, None, offsets, gates, counts)
        if np.isfinite(F):
            return th, delta
    raise RuntimeError("no feasible TP start")


def nll_in_mode(theta, mode, n, M, K, G0, offsets, gates, counts):
    rho, E, G = PR.forward(mode, theta, n, M, K, G0)
    F, _, g, nbad, _ = B.loglik(rho, E, G, offsets, gates, counts, raise_nonpos=False)
    if nbad or not np.isfinite(F):
        return np.inf, np.zeros_like(theta)
    return F, PR.backward(mode, theta, n, M, K, g, G0)


def mlgst(stages: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]], theta0, mode, n: int, M: int, K: int,
          G0=None, maxiter: int = 1000, gtol: float = 1e-10) -> List[Tuple[np.ndarray, float]]:
    """Iterative MLGST: per stage (offsets, gates, counts), minimize the negative
    log-likelihood from the previous stage's parameters; returns [(theta, F)].
    The optimizer sees F per shot (F / sum N, the same minimizer) so that its
    tolerances do not depend on the number of shots."""
    theta = np.asarray(theta0, np.float64).copy()
    out = []
    for off, gts, cnt in stages:
        if mode_is_tp(mode):
            theta, _ = feasible_tp_start(theta, n, M, K, off, gts, cnt)
        else:
            theta, _ = feasible_cptp_start(theta, n, M, K, G0, off, gts, cnt)
        scale = 1.0 / max(1.0, float(np.asarray(cnt, np.float64).sum()))

        def f(th):
            F, g = nll_in_mode(th, mode, n, M, K, G0, off, gts, cnt)
            return F * scale, g * scale

        theta, fx, _ = lbfgs(f, theta, gtol=gtol, maxiter=maxiter)
        out.append((theta.copy(), float(fx) / scale))
    return out


def lbfgs(f, x0, m: int = 10, gtol: float = 1e-10, maxiter: int = 1000):
    """A plain limited-memory BFGS (two-loop recursion, memory m, initial scaling
    s^T y / y^T y) with a strong Wolfe line search (c1 = 1e-4, c2 = 0.9:
    bracketing by doubling from the unit step, then bisection; a non-finite
    objective counts as too long); pairs with s^T y <= 0 are skipped.  Stops when
    max |g| <= gtol, after maxiter iterations, or when no step decreases f."""
    x = np.asarray(x0, np.float64).copy()
    fx, g = f(x)
    if not np.isfinite(fx):
        return x, fx, g
    S, Y = [], []
    for it in range(maxiter):
        if np.max(np.abs(g)) <= gtol:
            break
        q = g.copy()
        alphas = []
        for s, y in reversed(list(zip(S, Y))):
            a = np.dot(s, q) / np.dot(y, s)
            alphas.append(a)
            q -= a * y
        if S:
            q *= np.dot(S[-1], Y[-1]) / np.dot(Y[-1], Y[-1])
        for (s, y), a in zip(zip(S, Y), reversed(alphas)):
            b = np.dot(y, q) / np.dot(y, s)
            q += (a - b) * s
        d = -q
        gd = np.dot(g, d)
        if not gd < 0:
            break

        def phi(a):
            xn = x + a * d
            fn, gn = f(xn)
            return xn, fn, gn, np.dot(gn, d)

        c1, c2 = 1e-4, 0.9
        a_prev, f_prev, a = 0.0, fx, 1.0
        found, zoom, lo, hi, f_lo = False, False, 0.0, 0.0, fx
        for ls in range(60):
            xn, fn, gn, dn = phi(a)
            if not np.isfinite(fn) or fn > fx + c1 * a * gd or (ls > 0 and fn >= f_prev):
                lo, f_lo, hi, zoom = a_prev, f_prev, a, True
                break
            if abs(dn) <= -c2 * gd:
                found = True
                break
            if dn >= 0:
                lo, f_lo, hi, zoom = a, fn, a_prev, True
                break
            a_prev, f_prev, a = a, fn, 2 * a
        if zoom:
            for _ in range(60):
                a = 0.5 * (lo + hi)
                xn, fn, gn, dn = phi(a)
                if not np.isfinite(fn) or fn > fx + c1 * a * gd or fn >= f_lo:
                    hi = a
                else:
                    if abs(dn) <= -c2 * gd:
                        found = True
                        break
                    if dn * (hi - lo) >= 0:
                        hi = lo
                    lo, f_lo = a, fn
        if not found:
            if lo > 0 and np.isfinite(f_lo) and f_lo <= fx + c1 * lo * gd and f_lo < fx:
                a = lo
                xn, fn, gn, dn = phi(a)
            else:
                break
        s, y = xn - x, gn - g
        if np.dot(s, y) > 1e-300:
            S.append(s)
            Y.append(y)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x, fx, g = xn, fn, gn
    return x, fx, g
