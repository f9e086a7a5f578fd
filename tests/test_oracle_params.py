"""Pins of the oracle's gate-set parameterizations (Full / TP / CPTP estimation
modes, thesis Sec. 6.3.2) against what the mathematics fixes: the constraints
themselves (trace preservation, completeness, the Choi matrix of Eq. choimatrix
positive semidefinite), closed forms of simple generators (a Hamiltonian
rotation, dephasing, amplitude damping), the dissipator against its Kraus form
in Hilbert space, and the chain rule against central differences."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import params as PR
from paper_2008_13490_amd import workloads as W


def random_theta(mode, n, M, K, rng, scale=0.1):
    th = rng.normal(size=PR.param_count(mode, n, M, K)) * scale
    if PR.mode_id(mode) == PR.CPTP:
        # a state parameter with a dominant |0><0| component
        th[0] = 1.0
    return th


def ideal_targets(kind):
    _, Us, n = W.ideal_unitaries(kind)
    return np.array([W.ptm_from_unitary(U) for U in Us]), n


def matrix_from_vec(v, n):
    """Operator sum_i v_i P_i / sqrt(d) from its normalized Pauli coordinates."""
    P = PR.paulis(n)
    return np.einsum("i,ixy->xy", v, P) / np.sqrt(2 ** n)


def choi(G, n):
    """Choi matrix (Eq. choimatrix) of the map with transfer matrix G:
    J = (1/N) sum_ij |i><j| (x) E(|i><j|), E(X) from the Pauli coordinates of X."""
    d = 2 ** n
    P = PR.paulis(n)
    J = np.zeros((d * d, d * d), dtype=complex)
    for i in range(d):
        for j in range(d):
            X = np.zeros((d, d), dtype=complex)
            X[i, j] = 1.0
            x = np.array([np.trace(P[a] @ X) for a in range(d * d)]) / np.sqrt(d)
            EX = matrix_from_vec(G @ x, n)
            J[i * d:(i + 1) * d, j * d:(j + 1) * d] = EX / d
    return J


def test_parameter_counts():
    # full: the thesis's 1616 for two qubits, four outcomes, six gates
    assert PR.param_count("full", 2, 4, 6) == 1616
    # TP: 15 state + 3 x 16 effect + 6 x 240 gate parameters; CPTP: 16 state parameters
    assert PR.param_count("tp", 2, 4, 6) == 15 + 48 + 1440
    assert PR.param_count("cptp", 2, 4, 6) == 16 + 48 + 1440
    assert PR.param_count("tp", 1, 2, 3) == 3 + 4 + 3 * 12


@pytest.mark.parametrize("n,M,K", [(1, 2, 3), (2, 4, 6)])
def test_tp_constraints_and_chain_rule(n, M, K):
    rng = np.random.default_rng(1)
    D = 4 ** n
    th = random_theta("tp", n, M, K, rng)
    rho, E, G = PR.forward("tp", th, n, M, K)
    assert np.isclose(np.trace(matrix_from_vec(rho, n)).real, 1.0, atol=1e-15)
    assert np.allclose(matrix_from_vec(E.sum(0), n), np.eye(2 ** n), atol=1e-14)
    assert np.all(G[:, 0, :] == np.eye(D)[0])
    # trace preservation of every gate: tr(E(X)) = tr(X) for random X
    X = rng.normal(size=D)
    for k in range(K):
        assert np.isclose((G[k] @ X)[0], X[0], atol=1e-15)
    # the maps are affine: the chain rule is exact against differences
    gbar = rng.normal(size=PR.param_count("full", n, M, K))
    g = PR.backward("tp", th, n, M, K, gbar)
    f = lambda t: np.dot(gbar, np.concatenate([a.ravel() for a in PR.forward("tp", t, n, M, K)]))
    for i in rng.choice(th.size, 25, replace=False):
        e = np.zeros(th.size)
        e[i] = 1.0
        assert abs((f(th + e) - f(th - e)) / 2 - g[i]) <= 1e-12 * max(1, abs(g[i]))


@pytest.mark.parametrize("kind", ["1q", "2q"])
def test_cptp_gates_are_cptp(kind):
    rng = np.random.default_rng(2)
    G0, n = ideal_targets(kind)
    K, D, M = G0.shape[0], 4 ** n, 2 ** n
    th = random_theta("cptp", n, M, K, rng, scale=0.2)
    rho, E, G = PR.forward("cptp", th, n, M, K, G0)
    for k in range(K):
        J = choi(G[k], n)
        assert np.allclose(J, J.conj().T, atol=1e-14)
        assert np.linalg.eigvalsh(J).min() >= -1e-13          # completely positive
        d = 2 ** n
        Jt = J.reshape(d, d, d, d)
        assert np.allclose(np.einsum("iaja->ij", Jt), np.eye(d) / d, atol=1e-13)   # trace preserving
        assert np.allclose(G[k][0], np.eye(D)[0], atol=1e-14)
    R = matrix_from_vec(rho, n)
    assert np.isclose(np.trace(R).real, 1.0, atol=1e-14)
    assert np.linalg.eigvalsh(R).min() >= -1e-14
    assert np.allclose(matrix_from_vec(E.sum(0), n), np.eye(2 ** n), atol=1e-14)


def test_cptp_zero_generator_and_hamiltonian_closed_form():
    """h = 0, T = 0 gives the target; T = 0 gives exp(-i H) with H = sum h_k P_k / 2
    (Eq. GateDecompositionHamiltonian) applied after the target."""
    rng = np.random.default_rng(3)
    for kind in ("1q", "2q"):
        G0, n = ideal_targets(kind)
        K, D, M = G0.shape[0], 4 ** n, 2 ** n
        th = np.zeros(PR.param_count("cptp", n, M, K))
        th[0] = 1.0
        rho, E, G = PR.forward("cptp", th, n, M, K, G0)
        assert np.allclose(G, G0, atol=1e-15)
        h = rng.normal(size=D - 1) * 0.3
        P = PR.paulis(n)
        H = np.einsum("k,kxy->xy", h, P[1:]) / 2
        U = sla.expm(-1j * H)
        L = PR.hamiltonian_ptm(h, n)
        assert np.allclose(sla.expm(L), W.ptm_from_unitary(U), atol=1e-14)


def test_pure_state_parameter():
    """A = diag(1, 0, ...) is |0..0><0..0|: Pauli coordinates 1/sqrt(d) on the
    products of I and Z only."""
    for n in (1, 2):
        d, D = 2 ** n, 4 ** n
        x = np.zeros(D)
        x[0] = 0.7   # the normalization removes the scale
        v = PR._cholesky_state(x, n)
        want = np.zeros(D)
        for i in range(D):
            digits = [(i >> (2 * q)) & 3 for q in range(n)]
            if all(a in (0, 3) for a in digits):
                want[i] = 1 / np.sqrt(d)
        assert np.allclose(v, want, atol=1e-15)


def test_dephasing_and_amplitude_damping_closed_forms():
    """One qubit: C = gamma on Z gives the dephasing PTM diag(1, e^{-2g}, e^{-2g}, 1);
    the jump operator sigma^- = |0><1| = (X + iY)/2 with rate t (C = t a a^dagger,
    a = (1/2, i/2, 0)) gives amplitude damping towards |0>."""
    g = 0.37
    C = np.zeros((3, 3), dtype=complex)
    C[2, 2] = g
    G = sla.expm(PR.dissipator_ptm(C, 1))
    assert np.allclose(G, np.diag([1, np.exp(-2 * g), np.exp(-2 * g), 1]), atol=1e-15)
    t = 0.8
    a = np.array([0.5, 0.5j, 0.0])
    G = sla.expm(PR.dissipator_ptm(t * np.outer(a, a.conj()), 1))
    want = np.array([[1, 0, 0, 0],
                     [0, np.exp(-t / 2), 0, 0],
                     [0, 0, np.exp(-t / 2), 0],
                     [1 - np.exp(-t), 0, 0, np.exp(-t)]])
    assert np.allclose(G, want, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2])
def test_dissipator_against_kraus_form(n):
    """sum_jk C_jk (P_j rho P_k - {P_k P_j, rho}/2) with C = T T^dagger equals
    sum_g (A_g rho A_g^dagger - {A_g^dagger A_g, rho}/2), A_g = sum_j T_jg P_j,
    in Hilbert space on random Hermitian rho."""
    rng = np.random.default_rng(4)
    D, d = 4 ** n, 2 ** n
    T = np.tril(rng.normal(size=(D - 1, D - 1)) + 1j * rng.normal(size=(D - 1, D - 1)))
    T[np.arange(D - 1), np.arange(D - 1)] = T.diagonal().real
    L = PR.dissipator_ptm(T @ T.conj().T, n)
    P = PR.paulis(n)
    As = [np.einsum("j,jxy->xy", T[:, g], P[1:]) for g in range(D - 1)]
    for _ in range(3):
        X = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
        R = X + X.conj().T
        out = sum(A @ R @ A.conj().T - 0.5 * (A.conj().T @ A @ R + R @ A.conj().T @ A) for A in As)
        x = np.array([np.trace(P[a] @ R) for a in range(D)]).real / np.sqrt(d)
        assert np.allclose(matrix_from_vec(L @ x, n), out, atol=1e-12 * np.abs(out).max())


@pytest.mark.parametrize("kind", ["1q", "2q"])
def test_cptp_chain_rule_central_differences(kind):
    rng = np.random.default_rng(5)
    G0, n = ideal_targets(kind)
    K, M = G0.shape[0], 2 ** n
    th = random_theta("cptp", n, M, K, rng, scale=0.15)
    gbar = rng.normal(size=PR.param_count("full", n, M, K))
    g = PR.backward("cptp", th, n, M, K, gbar, G0)
    f = lambda t: np.dot(gbar, np.concatenate([a.ravel() for a in PR.forward("cptp", t, n, M, K, G0)]))
    idx = np.arange(th.size) if n == 1 else rng.choice(th.size, 40, replace=False)
    h = 1e-5
    for i in idx:
        e = np.zeros(th.size)
        e[i] = h
        fd = (f(th + e) - f(th - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])
