"""Predictions of repeated gate applications and the statistical distance on the
GPU (thesis Eqs. GSTPrediction, statisticaldistance) against the oracle.

gst_predict runs the powers in blocks of 32 repetitions: within the first block
the probabilities are the plain evaluation bit for bit; later blocks start from
states reached with a matrix power of the gate and are checked at 1e-12
relative.  The distance kernel adds the same terms in the same order as the
oracle and is compared bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_2008_13490_amd import workloads as W

pytestmark = pytest.mark.gpu

BLOCK = 32


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_13490_amd import api
    return api, api.Context(0)


def check_predictions(p, want):
    """Bit for bit within the first block; beyond it 1e-12 relative, where a
    probability below 1e-12 (an outcome of probability zero, e.g. of the
    ideal gates, computed as a rounding residue of a few 1e-17) is held to
    1e-24 absolute."""
    assert p.shape == want.shape
    head = p[:, :, :BLOCK]
    assert np.array_equal(head, want[:, :, :BLOCK])
    rel = np.abs(p - want) / np.maximum(np.abs(want), 1e-12)
    rel[p == want] = 0.0
    assert rel.max() <= 1e-12, rel.max()
    return rel.max()


C2_PREPS = [list(w) for w in W.PREDICTION_PREPS_2Q.values()]
C1_PREPS = [[], [1, 1], [2], [1, 2, 1]]


@pytest.mark.parametrize("name,preps", [("c1", C1_PREPS), ("c2", C2_PREPS)])
def test_predict_matches_oracle(oracle_lib, gpu, name, preps):
    api, ctx = gpu
    m = W.structured_workload(name).model
    gates = list(range(m.K))
    r_max = 150
    say(f"[predict] {name}: {len(preps)} preparations x {len(gates)} gates, r <= {r_max}")
    dg = api.DeviceGateSet.from_numpy(m.n_qubits, m.rho, m.effects, m.gates)
    p = api.predict(ctx, dg, preps, gates, r_max).cpu().numpy()
    want = oracle_lib.predict(m.rho, m.effects, m.gates, preps, gates, r_max)
    say(f"[predict] {name}: max relative difference {check_predictions(p, want):.3g}")


def test_predict_thousand_repetitions(oracle_lib, gpu):
    """The prediction test's range r <= 1000 with the two-qubit estimate and the
    ideal gate set; the statistical distance between the two predictions agrees
    with the oracle's to 1e-12."""
    api, ctx = gpu
    pw = W.prediction_workload(1000)
    out = {}
    for label, gs in (("estimate", pw.estimate), ("ideal", pw.ideal)):
        say(f"[predict] {label}: r <= {pw.r_max}")
        dg = api.DeviceGateSet.from_numpy(gs.n_qubits, gs.rho, gs.effects, gs.gates)
        out[label] = api.predict(ctx, dg, pw.preps, pw.gates, pw.r_max)
    p = out["estimate"].cpu().numpy()
    sub = [0, 3]   # two preparations through the oracle (every gate, every r)
    preps = [pw.preps[x] for x in sub]
    want = oracle_lib.predict(pw.estimate.rho, pw.estimate.effects, pw.estimate.gates, preps, pw.gates, pw.r_max)
    check_predictions(p[sub], want)
    d = api.tv_distance(ctx, out["estimate"], out["ideal"]).cpu().numpy()
    wi = oracle_lib.predict(pw.ideal.rho, pw.ideal.effects, pw.ideal.gates, preps, pw.gates, pw.r_max)
    check_predictions(out["ideal"].cpu().numpy()[sub], wi)
    d_or = oracle_lib.tv_distance(want, wi)
    assert np.all(np.abs(d[sub] - d_or) <= 1e-12)
    assert d.shape == (len(pw.preps), len(pw.gates), pw.r_max + 1) and np.all((d >= 0) & (d <= 1))


def test_tv_distance_kernel(oracle_lib, gpu):
    import torch
    api, ctx = gpu
    rng = np.random.default_rng(8)
    for m in (2, 4, 8):
        P = rng.dirichlet(np.ones(m), size=1000)
        Q = rng.dirichlet(np.ones(m), size=1000)
        d = api.tv_distance(ctx, torch.as_tensor(P, device="cuda"), torch.as_tensor(Q, device="cuda"))
        assert np.array_equal(d.cpu().numpy(), oracle_lib.tv_distance(P, Q))


def test_predict_edges(oracle_lib, gpu):
    api, ctx = gpu
    m = W.structured_workload("c1").model
    dg = api.DeviceGateSet.from_numpy(m.n_qubits, m.rho, m.effects, m.gates)
    for r_max in (0, 1, BLOCK - 1, BLOCK, BLOCK + 1):
        p = api.predict(ctx, dg, [[], [2, 1]], [0, 2], r_max).cpu().numpy()
        want = oracle_lib.predict(m.rho, m.effects, m.gates, [[], [2, 1]], [0, 2], r_max)
        check_predictions(p, want)
    from paper_2008_13490_amd import _lib
    with pytest.raises(_lib.GSTError):
        api.predict(ctx, dg, [[]], [m.K], 10)          # gate index out of range
    with pytest.raises(_lib.GSTError):
        api.predict(ctx, dg, [[0] * 65], [0], 10)      # preparation longer than 64 gates
    names, Us, n = W.ideal_unitaries("3q")
    rho3 = np.zeros(64)
    rho3[0] = 1 / np.sqrt(8)
    E3 = np.zeros((8, 64))
    G3 = np.array([W.ptm_from_unitary(U) for U in Us])
    dg3 = api.DeviceGateSet.from_numpy(3, rho3, E3, G3)
    with pytest.raises(_lib.GSTError):
        api.predict(ctx, dg3, [[]], [0], 10)           # one or two qubits only
