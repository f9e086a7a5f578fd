"""Pins of the oracle's fit (LGST, gauge optimization, MLGST; thesis Sec. 6.3.1)
against what the mathematics fixes: linear inversion of exact probabilities
recovers the gate set up to the gauge M = (F V)^-1 given by the prepared states
and the singular vectors; the gauge objective's gradient against central
differences; gauge optimization of an exact gauge transform of the target
returns the target; the maximum-likelihood fit of data with exact frequencies
returns the generating gate set's probabilities; the plain L-BFGS on the
Rosenbrock function."""
import numpy as np
import pytest

from oracle import fit as FT
from oracle import params as PR
from paper_2008_13490_amd import workloads as W

FIDS_1Q = [(), (1,), (2,), (1, 1)]
GERMS_1Q = [(0,), (1,), (2,), (1, 2)]


def one_qubit_fit_list(max_lengths=(1, 2, 4, 8)):
    words, ends = W.fit_words(FIDS_1Q, FIDS_1Q, GERMS_1Q, max_lengths, 3)
    return W.from_words(words), ends


def exact_probs(oracle_lib, gs, sl):
    return oracle_lib.probs(gs.rho, gs.effects, gs.gates, sl.offsets, sl.gates)


@pytest.mark.parametrize("kind", ["1q", "2q"])
def test_lgst_recovers_gate_set_up_to_the_gauge(oracle_lib, kind):
    rng = np.random.default_rng(1)
    truth = W.noisy_gateset(kind, 1e-3, 0.01, rng)
    if kind == "1q":
        prep, meas, germs = FIDS_1Q, FIDS_1Q, GERMS_1Q
    else:
        prep, meas, germs = W.FIT_PREP_FIDUCIALS_2Q, W.FIT_MEAS_FIDUCIALS_2Q, [(k,) for k in range(6)]
    words, ends = W.fit_words(prep, meas, germs, (), truth.K)
    sl = W.from_words(words)
    f = exact_probs(oracle_lib, truth, sl)
    rho, E, G = FT.lgst_freqs(sl.offsets, sl.gates, f, prep, meas, truth.n_qubits, truth.K)
    # the gauge: G_lgst = M G M^-1 with M = (F V)^-1, F the prepared states
    AB, _ = FT.ab_matrices(sl.offsets, sl.gates, f, prep, meas, truth.K)
    U, s, Vt = np.linalg.svd(AB, full_matrices=False)
    V = Vt[:truth.D].T
    for c in range(truth.D):
        if V[np.argmax(np.abs(V[:, c])), c] < 0:
            V[:, c] = -V[:, c]
    Fm = np.array([np.linalg.multi_dot([truth.gates[g] for g in reversed(w)] + [truth.rho])
                   if w else truth.rho for w in prep]).T
    Mg = np.linalg.inv(Fm @ V)
    for k in range(truth.K):
        assert np.allclose(G[k], Mg @ truth.gates[k] @ np.linalg.inv(Mg), atol=1e-10)
    assert np.allclose(rho, Mg @ truth.rho, atol=1e-12)
    assert np.allclose(E, truth.effects @ np.linalg.inv(Mg), atol=1e-12)
    # gauge invariance: the estimate predicts every sequence
    rw = W.random_list(50, truth.K, 1, 20, rng)
    p_est = oracle_lib.probs(rho, E, G, rw.offsets, rw.gates)
    assert np.allclose(p_est, exact_probs(oracle_lib, truth, rw), atol=1e-10)


def test_gauge_objective_gradient():
    rng = np.random.default_rng(2)
    D = 4
    T = W.noisy_gateset("1q", 1e-3, 0.05, rng)
    est = W.noisy_gateset("1q", 2e-3, 0.05, rng)
    x = (np.eye(D) + 0.05 * rng.normal(size=(D, D))).reshape(-1)
    f0, g = FT.gauge_objective(x, est.rho, est.effects, est.gates, T.rho, T.effects, T.gates, 0.7)
    h = 1e-6
    for i in range(D * D):
        e = np.zeros(D * D)
        e[i] = h
        fp, _ = FT.gauge_objective(x + e, est.rho, est.effects, est.gates, T.rho, T.effects, T.gates, 0.7)
        fm, _ = FT.gauge_objective(x - e, est.rho, est.effects, est.gates, T.rho, T.effects, T.gates, 0.7)
        assert abs((fp - fm) / (2 * h) - g[i]) <= 1e-7 * max(1.0, abs(g[i]))


def test_gauge_opt_undoes_a_gauge_transform():
    rng = np.random.default_rng(3)
    for kind in ("1q", "2q"):
        T = W.noisy_gateset(kind, 1e-3, 0.02, rng)
        M0 = np.eye(T.D) + 0.05 * rng.normal(size=(T.D, T.D))
        rho, E, G = FT.gauge_transform(T.rho, T.effects, T.gates, M0)
        Mg, (r2, E2, G2), fmin = FT.gauge_opt(rho, E, G, T.rho, T.effects, T.gates)
        # from an objective of order 0.1 down to the optimizer's stopping rule
        f0, _ = FT.gauge_objective(np.eye(T.D).reshape(-1), rho, E, G, T.rho, T.effects, T.gates, 1.0)
        assert f0 > 1e-3 and fmin <= 1e-15
        assert np.allclose(G2, T.gates, atol=1e-7) and np.allclose(r2, T.rho, atol=1e-7)
        assert np.allclose(Mg, np.linalg.inv(M0), atol=1e-7)


def test_mlgst_on_exact_frequencies_returns_the_truth(oracle_lib):
    """Counts proportional to the exact probabilities (10^7 shots per sequence):
    the ML estimate reproduces them, up to the rounding of the counts."""
    rng = np.random.default_rng(4)
    truth = W.noisy_gateset("1q", 5e-3, 0.03, rng)
    # a slightly mixed initial state: every probability positive (an interior point,
    # where the likelihood is stationary at the generating gate set)
    truth.rho = truth.rho * np.array([1.0, 1.0, 1.0, 0.98])
    sl, ends = one_qubit_fit_list()
    p = exact_probs(oracle_lib, truth, sl)
    counts = np.round(p * 1e7).astype(np.int64)
    assert counts.max() < 2 ** 31
    counts = counts.astype(np.int32)
    rho, E, G = FT.lgst(sl.offsets, sl.gates, counts, FIDS_1Q, FIDS_1Q, 1, 3)
    target = W.noisy_gateset("1q", 0.0, 0.0, rng)
    _, (rho, E, G), _ = FT.gauge_opt(rho, E, G, target.rho, target.effects, target.gates)
    theta0 = FT.contract_tp(rho, E, G)
    stages = []
    for e in ends[1:]:
        sub = sl.subset(np.arange(e))
        stages.append((sub.offsets, sub.gates, counts[:e]))
    out = FT.mlgst(stages, theta0, "tp", 1, 2, 3)
    th = out[-1][0]
    r, Ef, Gf = PR.forward("tp", th, 1, 2, 3)
    assert np.allclose(oracle_lib.probs(r, Ef, Gf, sl.offsets, sl.gates), p, atol=2e-6)
    # the fitted stage objectives do not exceed the truth's
    for (off, gts, cnt), (_, F) in zip(stages, out):
        F_truth = oracle_lib.loglik(truth.rho, truth.effects, truth.gates, off, gts, cnt)[0]
        assert F <= F_truth * (1 + 1e-12)


def test_plain_lbfgs_rosenbrock():
    def f(x):
        a, b = x
        return (1 - a) ** 2 + 100 * (b - a * a) ** 2, np.array([-2 * (1 - a) - 400 * a * (b - a * a),
                                                                200 * (b - a * a)])
    x, fx, g = FT.lbfgs(f, np.array([-1.2, 1.0]), gtol=1e-10, maxiter=5000)
    assert np.allclose(x, [1.0, 1.0], atol=1e-8) and fx < 1e-16
