"""Gate-set parameterizations of the fit (test infrastructure only).

The thesis runs GST in three estimation modes (Sec. 6.3.2): fully unconstrained
maps ("Full"), trace-preserving maps ("TP") and completely positive
trace-preserving channels ("CPTP"), with the quantum operations of Sec. 2.4.
This module writes out the maps from a parameter vector theta to the full
parameterization (rho [D], effects [M][D], gates [K][D][D] as Pauli transfer
matrices in the normalized Pauli basis, Eq. paulitransfermatrix) and the chain
rule back, as plain definitions:

* TP: row 0 of every gate is e_0 (trace preservation), rho[0] = 1/sqrt(d)
  (unit trace), and the effects are complete: the last one is vec(1) minus the
  others (sum_m E_m = 1).  theta = [rho[1:] | e_0 .. e_{M-2} | rows 1.. of each gate].
* CPTP: every gate is G_k = exp(L_k) G0_k (Eq. GateDecompositionLindbladCorrespondence)
  with G0_k a fixed target and L_k the transfer matrix of a generator in the
  form of Eq. masterequation,
      L(rho) = -i [H, rho] + sum_{j,k >= 1} C_jk (P_j rho P_k - {P_k P_j, rho} / 2),
  H = sum_{k >= 1} h_k P_k / 2 (Eq. GateDecompositionHamiltonian) and C = T T^dagger
  positive semidefinite (T lower triangular, real diagonal), so exp(L) is CPTP.
  rho = A A^dagger / tr(A A^dagger) (A lower triangular, real diagonal); effects as TP.
  theta = [A | e_0 .. e_{M-2} | per gate: h (D-1), T].
  A and T are stored as their real diagonals, then the entries below the
  diagonal in row-major order as (real, imaginary) pairs.

The backward map is the chain rule written out one parameter at a time: the
exact directional derivative of the full parameters along each coordinate of
theta (for the gates: the Frechet derivative of the matrix exponential,
scipy.linalg.expm_frechet), dotted with the full gradient.
"""
from __future__ import annotations

import functools
from typing import Optional, Tuple

import numpy as np
import scipy.linalg as sla

FULL, TP, CPTP = 0, 1, 2
_MODES = {"full": FULL, "tp": TP, "cptp": CPTP}

_S = (np.eye(2, dtype=complex), np.array([[0, 1], [1, 0]], dtype=complex),
      np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], dtype=complex))


def mode_id(mode) -> int:
    return _MODES[mode] if isinstance(mode, str) else int(mode)


@functools.lru_cache(maxsize=None)
def paulis(n: int) -> np.ndarray:
    """The unnormalized Pauli products P_i (Eq. paulibasis), i = sum_q a_q 4^(n-1-q),
    qubit 0 the leftmost tensor factor: array [4^n, 2^n, 2^n]."""
    out = []
    for i in range(4 ** n):
        M = np.ones((1, 1), dtype=complex)
        for q in range(n):
            M = np.kron(M, _S[(i >> (2 * (n - 1 - q))) & 3])
        out.append(M)
    return np.array(out)


@functools.lru_cache(maxsize=None)
def _generator_bases(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Transfer matrices (in the normalized basis, entry [a][b] = tr(P_a X(P_b)) / d)
    of the maps X_k(rho) = -i [P_k / 2, rho] (k = 1..D-1) and
    Z_jk(rho) = P_j rho P_k - (P_k P_j rho + rho P_k P_j) / 2 (j, k = 1..D-1)."""
    P = paulis(n)
    D, d = P.shape[0], P.shape[1]
    ham = np.zeros((D - 1, D, D))
    for k in range(1, D):
        for b in range(D):
            Xb = -0.5j * (P[k] @ P[b] - P[b] @ P[k])
            for a in range(D):
                v = np.trace(P[a] @ Xb) / d
                assert abs(v.imag) < 1e-15
                ham[k - 1, a, b] = v.real
    # Z[j][k][a][b], by traces of four Pauli products
    t1 = np.einsum("axy,jyz,bzw,kwx->jkab", P, P, P, P, optimize=True)   # tr(P_a P_j P_b P_k)
    t2 = np.einsum("axy,kyz,jzw,bwx->jkab", P, P, P, P, optimize=True)   # tr(P_a P_k P_j P_b)
    t3 = np.einsum("axy,byz,kzw,jwx->jkab", P, P, P, P, optimize=True)   # tr(P_a P_b P_k P_j)
    Z = (t1 - 0.5 * t2 - 0.5 * t3) / d
    return ham, np.ascontiguousarray(Z[1:, 1:])


def hamiltonian_ptm(h: np.ndarray, n: int) -> np.ndarray:
    """Transfer matrix of rho -> -i [H, rho], H = sum_{k>=1} h_k P_k / 2."""
    ham, _ = _generator_bases(n)
    return np.einsum("k,kab->ab", h, ham)


def dissipator_ptm(C: np.ndarray, n: int) -> np.ndarray:
    """Transfer matrix of rho -> sum_jk C_jk (P_j rho P_k - {P_k P_j, rho} / 2) for a
    Hermitian (D-1) x (D-1) matrix C (real for Hermitian C)."""
    _, Z = _generator_bases(n)
    L = np.einsum("jk,jkab->ab", C, Z)
    assert np.abs(L.imag).max() <= 1e-13 * max(1.0, np.abs(C).max())
    return L.real


def _tri_from_reals(x: np.ndarray, m: int) -> np.ndarray:
    """Lower-triangular complex m x m matrix from m real diagonal entries followed
    by (real, imaginary) pairs of the strict lower triangle in row-major order."""
    T = np.zeros((m, m), dtype=complex)
    T[np.arange(m), np.arange(m)] = x[:m]
    p = m
    for j in range(m):
        for k in range(j):
            T[j, k] = x[p] + 1j * x[p + 1]
            p += 2
    return T


def _tri_size(m: int) -> int:
    return m + m * (m - 1)


def param_count(mode, n: int, M: int, K: int) -> int:
    D = 4 ** n
    mode = mode_id(mode)
    if mode == FULL:
        return D + M * D + K * D * D
    spam = (D - 1 if mode == TP else D) + (M - 1) * D
    return spam + K * D * (D - 1)


def _split(mode, theta, n, M, K):
    D = 4 ** n
    theta = np.asarray(theta, np.float64)
    assert theta.shape == (param_count(mode, n, M, K),)
    nr = D - 1 if mode == TP else D
    r = theta[:nr]
    e = theta[nr:nr + (M - 1) * D].reshape(M - 1, D)
    g = theta[nr + (M - 1) * D:].reshape(K, D * (D - 1))
    return r, e, g


def _complete_effects(e: np.ndarray, D: int) -> np.ndarray:
    """e_0 .. e_{M-2} as given, e_{M-1} = vec(1) - e_0 - ... - e_{M-2} (subtracted in
    ascending order); vec(1) = (sqrt(d), 0, ..., 0) in the normalized basis."""
    last = np.zeros(D)
    last[0] = np.sqrt(np.sqrt(D))   # sqrt(d), d = sqrt(D)
    for m in range(e.shape[0]):
        last = last - e[m]
    return np.vstack([e, last[None, :]])


def cptp_gate_generator(tg: np.ndarray, n: int) -> np.ndarray:
    """L of one CPTP gate from its parameters (h, T)."""
    D = 4 ** n
    h = tg[:D - 1]
    T = _tri_from_reals(tg[D - 1:], D - 1)
    return hamiltonian_ptm(h, n) + dissipator_ptm(T @ T.conj().T, n)


def _cholesky_state(x: np.ndarray, n: int) -> np.ndarray:
    d = 2 ** n
    A = _tri_from_reals(x, d)
    N = A @ A.conj().T
    rho = N / np.trace(N).real
    P = paulis(n)
    v = np.array([np.trace(P[i] @ rho) for i in range(4 ** n)]) / np.sqrt(d)
    assert np.abs(v.imag).max() < 1e-14
    return v.real


def forward(mode, theta, n: int, M: int, K: int, G0: Optional[np.ndarray] = None):
    """theta -> (rho [D], effects [M, D], gates [K, D, D])."""
    mode = mode_id(mode)
    D = 4 ** n
    if mode == FULL:
        theta = np.asarray(theta, np.float64)
        return theta[:D].copy(), theta[D:D + M * D].reshape(M, D).copy(), theta[D + M * D:].reshape(K, D, D).copy()
    r, e, g = _split(mode, theta, n, M, K)
    E = _complete_effects(e, D)
    if mode == TP:
        rho = np.concatenate([[1.0 / np.sqrt(np.sqrt(D))], r])   # tr(P_0 rho) / sqrt(d) = 1 / sqrt(d)
        G = np.zeros((K, D, D))
        G[:, 0, 0] = 1.0
        G[:, 1:, :] = g.reshape(K, D - 1, D)
        return rho, E, G
    assert G0 is not None and G0.shape == (K, D, D)
    rho = _cholesky_state(r, n)
    G = np.array([sla.expm(cptp_gate_generator(g[k], n)) @ G0[k] for k in range(K)])
    return rho, E, G


def backward(mode, theta, n: int, M: int, K: int, grad_full, G0: Optional[np.ndarray] = None) -> np.ndarray:
    """d(objective)/d(theta) from the gradient with respect to the full parameters
    ([rho | effects | gates], the layout of the likelihood gradient)."""
    mode = mode_id(mode)
    D = 4 ** n
    gf = np.asarray(grad_full, np.float64)
    if mode == FULL:
        return gf.copy()
    gr, ge, gG = gf[:D], gf[D:D + M * D].reshape(M, D), gf[D + M * D:].reshape(K, D, D)
    r, e, g = _split(mode, theta, n, M, K)
    out = []
    # state
    if mode == TP:
        out.append(gr[1:])
    else:
        d = 2 ** n
        A = _tri_from_reals(r, d)
        N = A @ A.conj().T
        t = np.trace(N).real
        P = paulis(n)
        gx = np.zeros(D)
        for i in range(D):
            x = np.zeros(D)
            x[i] = 1.0
            dA = _tri_from_reals(x, d)
            dN = dA @ A.conj().T + A @ dA.conj().T
            drho = dN / t - N * np.trace(dN).real / t ** 2
            dv = np.array([np.trace(P[a] @ drho).real for a in range(D)]) / np.sqrt(d)
            gx[i] = np.dot(gr, dv)
        out.append(gx)
    # effects: e_m enters E_m with +1 and E_{M-1} with -1
    out.append((ge[:M - 1] - ge[M - 1][None, :]).reshape(-1))
    # gates
    for k in range(K):
        if mode == TP:
            out.append(gG[k, 1:, :].reshape(-1))
            continue
        tg = g[k]
        L = cptp_gate_generator(tg, n)
        T = _tri_from_reals(tg[D - 1:], D - 1)
        gk = np.zeros(tg.size)
        for i in range(tg.size):
            if i < D - 1:
                dh = np.zeros(D - 1)
                dh[i] = 1.0
                dL = hamiltonian_ptm(dh, n)
            else:
                x = np.zeros(tg.size - (D - 1))
                x[i - (D - 1)] = 1.0
                dT = _tri_from_reals(x, D - 1)
                dL = dissipator_ptm(dT @ T.conj().T + T @ dT.conj().T, n)
            dG = sla.expm_frechet(L, dL, compute_expm=False) @ G0[k]
            gk[i] = np.sum(gG[k] * dG)
        out.append(gk)
    return np.concatenate(out)
