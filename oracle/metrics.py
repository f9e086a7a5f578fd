"""Post-fit metrics of the estimates (test infrastructure only).

* avg_gate_fidelity: Eq. gatemetricsaveragegatefidelity, the average over pure
  states of <psi| G_ac(G_id^-1(|psi><psi|)) |psi> for a unitary target, taken
  exactly as the mean over a complex projective 2-design (the states of d + 1
  mutually unbiased bases: the integrand is quadratic in |psi><psi|).  The
  actual operation is given by its Pauli transfer matrix.
* diamond_unitary: Eq. appdiamondunitaryResult (App. H) for the unitaries U, V:
  with lambda the eigenvalues of W = U^dagger V, 1 if the origin lies in their
  convex hull (all successive argument gaps at most pi), else max |l_j - l_k| / 2.
* hamiltonian_decomposition: App. J, L = log G (the principal matrix
  logarithm, Eq. GateDecompositionMatrixLog), projected onto the form of
  -i[H, .] with H = sum_k h_k P_k / 2 (Eqs. GateDecompositionHamiltonian,
  GateDecompositionHamiltonianPTM, GateDecompositionHamiltonianProjection), the
  decomposition error gamma = ||G - exp(L^H)||_F, the rotation angle |h| and
  axis h / |h| (Eqs. GSTHamiltonianAngle, GSTHamiltonianAxis).
* hamiltonian_decomposition_toward: App. J's other route, for gates whose
  transfer matrix has no real principal logarithm (eigenvalues on the
  negative real axis, like the ideal CZ and CNOT): the coefficients h that
  minimize gamma(h) = ||G - exp(L^H(h))||_F directly, starting from the
  Hamiltonian of the intended target unitary U, H_U = i log U with the
  principal branch of each eigenvalue's argument (the target's logarithm);
  scipy's L-BFGS-B with the gradient from the Frechet derivative of exp.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.linalg as sla

from .params import paulis

# commuting triples whose joint eigenbases are mutually unbiased (two qubits):
# labels a0 * 4 + a1 with I, X, Y, Z = 0..3
_MUB_SETS_2Q = [(3 * 4 + 0, 0 * 4 + 3), (1 * 4 + 0, 0 * 4 + 1), (2 * 4 + 0, 0 * 4 + 2),
                (1 * 4 + 2, 2 * 4 + 3), (2 * 4 + 1, 3 * 4 + 2)]


@functools.lru_cache(maxsize=None)
def mub_states(n: int) -> np.ndarray:
    """The d (d + 1) states of d + 1 mutually unbiased bases, as rows."""
    P = paulis(n)
    if n == 1:
        sets = [(1,), (2,), (3,)]
    elif n == 2:
        sets = _MUB_SETS_2Q
    else:
        raise ValueError("one or two qubits")
    out = []
    for s in sets:
        A = sum((j + 1) * P[k] for j, k in enumerate(s))   # distinct eigenvalues on the joint eigenbasis
        _, V = np.linalg.eigh(A)
        out.extend(V.T)
    return np.array(out)


def _vec(rho, n):
    P = paulis(n)
    return np.array([np.trace(P[i] @ rho).real for i in range(4 ** n)]) / np.sqrt(2 ** n)


def _mat(v, n):
    return np.einsum("i,ixy->xy", v, paulis(n)) / np.sqrt(2 ** n)


def avg_gate_fidelity(G: np.ndarray, U: np.ndarray) -> float:
    """F_avg of the operation with transfer matrix G against the unitary U."""
    d = U.shape[0]
    n = int(round(np.log2(d)))
    acc = 0.0
    states = mub_states(n)
    for psi in states:
        proj = np.outer(psi, psi.conj())
        back = U.conj().T @ proj @ U           # G_id^-1 (|psi><psi|)
        out = _mat(G @ _vec(back, n), n)
        acc += np.real(psi.conj() @ out @ psi)
    return acc / len(states)


def diamond_unitary(U: np.ndarray, V: np.ndarray) -> float:
    lam = np.linalg.eigvals(U.conj().T @ V)
    phi = np.sort(np.mod(np.angle(lam), 2 * np.pi))
    gaps = np.diff(np.concatenate([phi, [phi[0] + 2 * np.pi]]))
    if np.all(gaps <= np.pi):
        return 1.0
    return float(np.max(np.abs(lam[:, None] - lam[None, :])) / 2)


@functools.lru_cache(maxsize=None)
def supercommutator(n: int) -> np.ndarray:
    """s[k][j][i] = Tr([P_k, P_j] P_i) / (2 N i) (Eq. GateDecompositionHamiltonianPTM)."""
    P = paulis(n)
    D, N = P.shape[0], P.shape[1]
    s = np.zeros((D, D, D))
    for k in range(D):
        for j in range(D):
            C = P[k] @ P[j] - P[j] @ P[k]
            for i in range(D):
                v = np.trace(C @ P[i]) / (2 * N * 1j)
                assert abs(v.imag) < 1e-12
                s[k, j, i] = v.real
    return s


def hamiltonian_decomposition(G: np.ndarray):
    """(h [D] with h_0 = 0, gamma, angle |h|, axis h / |h|) of the transfer matrix G."""
    D = G.shape[0]
    n = int(round(np.log(D) / np.log(4)))
    L = sla.logm(G)
    assert np.abs(np.imag(L)).max() < 1e-10, "no real principal logarithm"
    L = np.real(L)
    s = supercommutator(n)
    h = np.zeros(D)
    for k in range(1, D):
        den = np.sum(np.abs(s[k]))
        if den:
            h[k] = np.sum(L.T * s[k]) / den     # sum_ij L_ij s_kji
    LH = np.einsum("k,kji->ij", h, s)
    gamma = float(np.linalg.norm(G - sla.expm(LH)))
    phi = float(np.linalg.norm(h))
    axis = h / phi if phi > 0 else np.zeros(D)
    return h, gamma, phi, axis


def hamiltonian_ptm(h: np.ndarray) -> np.ndarray:
    """L^H of Eq. GateDecompositionHamiltonianPTM: L^H_ij = sum_k h_k s_kji."""
    D = h.shape[0]
    n = int(round(np.log(D) / np.log(4)))
    return np.einsum("k,kji->ij", h, supercommutator(n))


def target_hamiltonian(U: np.ndarray) -> np.ndarray:
    """h (h_0 = 0) of H = i log U, each eigenvalue's argument in (-pi, pi]: U = exp(-iH)
    up to a global phase, H = sum_k h_k P_k / 2."""
    N = U.shape[0]
    n = int(round(np.log2(N)))
    w, V = np.linalg.eig(U)
    theta = np.angle(w)
    theta[theta <= -np.pi + 1e-12] = np.pi        # the principal argument of -1 is pi
    H = -(V * theta) @ np.linalg.inv(V)          # i log U = i V diag(i theta) V^-1
    P = paulis(n)
    h = np.array([2.0 * np.trace(P[k] @ H).real / N for k in range(N * N)])
    h[0] = 0.0
    return h


def _gamma2(x, G):
    h = np.concatenate([[0.0], x])
    L = hamiltonian_ptm(h)
    E = sla.expm(L)
    R = G - E
    # d||R||^2 / dh_k = -2 <R, Dexp_L(dL/dh_k)>, dL/dh_k = s_k^T
    s = supercommutator(int(round(np.log(G.shape[0]) / np.log(4))))
    g = np.array([-2.0 * np.sum(R * sla.expm_frechet(L, s[k].T, compute_expm=False)) for k in range(1, G.shape[0])])
    return float(np.sum(R * R)), g


def hamiltonian_decomposition_toward(G: np.ndarray, U: np.ndarray, gtol: float = 1e-14):
    """(h [D] with h_0 = 0, gamma, angle |h|, axis h / |h|): h minimizing
    ||G - exp(L^H(h))||_F from the target's Hamiltonian."""
    import scipy.optimize as so
    D = G.shape[0]
    x0 = target_hamiltonian(U)[1:]
    res = so.minimize(_gamma2, x0, args=(G,), jac=True, method="L-BFGS-B",
                      options={"gtol": gtol, "ftol": 1e-30, "maxiter": 2000, "maxcor": 20})
    h = np.concatenate([[0.0], res.x])
    gamma = float(np.linalg.norm(G - sla.expm(hamiltonian_ptm(h))))
    phi = float(np.linalg.norm(h))
    axis = h / phi if phi > 0 else np.zeros(D)
    return h, gamma, phi, axis
