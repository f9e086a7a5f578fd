"""Seeded synthetic GST workloads: gate sets, sequence lists and outcome counts.

This module only *prepares inputs*.  It encodes gates as Pauli-transfer
matrices (thesis Sec. 2.4.1, Eqs. paulibasis / paulitransfermatrix), lists
gate sequences with the fiducial x germ-power x fiducial structure of
Sec. 6.3.1 (Eq. GSTFullFiducialsGerms), and samples outcome counts from a
"black box" that is emulated in Hilbert space (state vectors and unitaries, no
transfer matrices).  It never evaluates the probability chain, the likelihood
or its gradient on transfer matrices: that is the method, and it lives in the
HIP library (product) and in ``oracle/`` (test infrastructure) only.

Conventions (thesis Sec. 2.1.3 and Sec. 2.4.1):
  * qubit 0 is the most significant bit of a basis index and the leftmost
    tensor factor;
  * Pauli index ``i = sum_q a_q 4**(n-1-q)`` with ``a in {I:0, X:1, Y:2, Z:3}``;
  * normalized basis ``P_i / sqrt(d)``, ``d = 2**n``, ``D = d*d``;
  * a gate word is stored in time order ``s_1 .. s_L`` (the matrix product is
    the reverse, Sec. 2.2.2).

Sequence lists are CSR: ``offsets`` int64 ``[S+1]`` and ``gates`` uint8
``[offsets[S]]``.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Pauli basis and transfer-matrix encoding (Sec. 2.4.1)
# ---------------------------------------------------------------------------
_I2 = np.eye(2, dtype=np.complex128)
_SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI_1Q = (_I2, _SX, _SY, _SZ)


_PAULI_CACHE: dict = {}


def pauli_basis(n: int) -> np.ndarray:
    """Unnormalized n-qubit Pauli products ``P_i``, shape ``[4**n, 2**n, 2**n]``.

    Index ``i`` has base-4 digits ``a_0 .. a_{n-1}`` (qubit 0 most significant),
    so ``P_1 = I x .. x I x sigma^x`` as in Eq. paulibasis.  (Cached; the
    returned array is read-only.)
    """
    if n not in _PAULI_CACHE:
        b = _pauli_basis(n)
        b.setflags(write=False)
        _PAULI_CACHE[n] = b
    return _PAULI_CACHE[n]


def _pauli_basis(n: int) -> np.ndarray:
    out = []
    for digits in itertools.product(range(4), repeat=n):
        m = np.ones((1, 1), dtype=np.complex128)
        for a in digits:
            m = np.kron(m, PAULI_1Q[a])
        out.append(m)
    return np.array(out)


def ptm_from_kraus(kraus: Sequence[np.ndarray]) -> np.ndarray:
    """Transfer matrix ``G_ij = Tr(P_i E(P_j)) / d`` of ``E(r) = sum_a K_a r K_a^+``."""
    d = kraus[0].shape[0]
    n = int(round(np.log2(d)))
    P = pauli_basis(n)
    D = d * d
    img = np.zeros((D, d, d), dtype=np.complex128)
    for K in kraus:
        img += np.einsum("ab,jbc,dc->jad", K, P, K.conj(), optimize=True)
    G = np.einsum("iab,jba->ij", P, img, optimize=True) / d
    return np.ascontiguousarray(G.real)


def ptm_from_unitary(U: np.ndarray) -> np.ndarray:
    return ptm_from_kraus([U])


def vec_operator(A: np.ndarray) -> np.ndarray:
    """Coefficients ``Tr(P_i A) / sqrt(d)`` of a Hermitian operator (Eqs. GSTVectorizedRho/EJ)."""
    d = A.shape[0]
    n = int(round(np.log2(d)))
    P = pauli_basis(n)
    return np.ascontiguousarray(np.einsum("iab,ba->i", P, A).real / np.sqrt(d))


def depolarizing_ptm(lam: float, n: int) -> np.ndarray:
    """Global symmetric depolarizing ``F r + (1-F) I/d`` with ``F = 1 - lam`` (Eq. singletDepolarizingChannelSymmetricMixture)."""
    D = 4 ** n
    return np.diag(np.concatenate([[1.0], np.full(D - 1, 1.0 - lam)]))


# ---------------------------------------------------------------------------
# Elementary unitaries (Sec. 2.2.1, App. B)
# ---------------------------------------------------------------------------
def rx(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)


def on_qubit(U1: np.ndarray, q: int, n: int) -> np.ndarray:
    m = np.ones((1, 1), dtype=np.complex128)
    for k in range(n):
        m = np.kron(m, U1 if k == q else _I2)
    return m


def cz(q0: int, q1: int, n: int) -> np.ndarray:
    d = 2 ** n
    diag = np.ones(d, dtype=np.complex128)
    for J in range(d):
        b0 = (J >> (n - 1 - q0)) & 1
        b1 = (J >> (n - 1 - q1)) & 1
        if b0 and b1:
            diag[J] = -1
    return np.diag(diag)


def cnot(control: int, target: int, n: int) -> np.ndarray:
    d = 2 ** n
    U = np.zeros((d, d), dtype=np.complex128)
    for J in range(d):
        bc = (J >> (n - 1 - control)) & 1
        J2 = J ^ (bc << (n - 1 - target))
        U[J2, J] = 1
    return U


def expm_hermitian(H: np.ndarray, t: float) -> np.ndarray:
    """``exp(-i t H)`` for Hermitian ``H`` via its eigendecomposition."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * t * w)) @ V.conj().T


# ---------------------------------------------------------------------------
# Gate sets
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class GateSet:
    n_qubits: int
    names: List[str]
    rho: np.ndarray        # [D]
    effects: np.ndarray    # [M, D]
    gates: np.ndarray      # [K, D, D] row-major
    unitaries: Optional[np.ndarray] = None  # [K, d, d] coherent parts (None for general CPTP sets)
    lam: float = 0.0       # global depolarizing strength applied after every gate

    @property
    def D(self) -> int:
        return 4 ** self.n_qubits

    @property
    def M(self) -> int:
        return self.effects.shape[0]

    @property
    def K(self) -> int:
        return self.gates.shape[0]

    def n_params(self) -> int:
        return self.D + self.M * self.D + self.K * self.D * self.D


def ideal_unitaries(kind: str) -> Tuple[List[str], List[np.ndarray], int]:
    """Ideal gate lists of the workload families (thesis Tab. GSTPulseImplementations, App. B)."""
    h = np.pi / 2
    if kind == "1q":
        n = 1
        return ["Gi", "Gx", "Gy"], [_I2.copy(), rx(h), ry(h)], n
    if kind == "2q":
        n = 2
        return (["Gii", "Gxi", "Gix", "Gyi", "Giy", "Gcz"],
                [np.eye(4, dtype=np.complex128), on_qubit(rx(h), 0, n), on_qubit(rx(h), 1, n),
                 on_qubit(ry(h), 0, n), on_qubit(ry(h), 1, n), cz(0, 1, n)], n)
    if kind == "3q":
        n = 3
        X3 = np.kron(np.kron(rx(h), rx(h)), rx(h))
        Y3 = np.kron(np.kron(ry(h), ry(h)), ry(h))
        return (["Giii", "Gxxx", "Gyyy", "Gcz01", "Gcz12"],
                [np.eye(8, dtype=np.complex128), X3, Y3, cz(0, 1, n), cz(1, 2, n)], n)
    raise ValueError(kind)


def random_axis(rng: np.random.Generator, D: int) -> np.ndarray:
    v = rng.standard_normal(D - 1)
    return v / np.linalg.norm(v)


def noisy_gateset(kind: str, lam: float, sigma: float, rng: np.random.Generator) -> GateSet:
    """Ideal gates composed with a seeded over-rotation and global depolarizing.

    ``U_k = exp(-i delta_k H_k / 2) U_k^ideal`` with ``H_k = sum_{j>=1} h_kj P_j``,
    ``h_k`` uniform on the unit sphere and ``delta_k ~ N(0, sigma^2)`` (the
    axis-angle form of Eqs. GSTGateHamiltonian-GSTHamiltonianAxis); then
    ``G_k = diag(1, (1-lam) 1) R(U_k)``.  Global depolarizing commutes with
    every unitary channel, so the order of the composition is immaterial.
    """
    _, Us, n = ideal_unitaries(kind)
    D = 4 ** n
    axes, deltas = [], []
    for _ in Us:
        axes.append(random_axis(rng, D))
        deltas.append(rng.normal(0.0, sigma))
    return gateset_from_rotations(kind, lam, axes, deltas)


def gateset_from_rotations(kind: str, lam: float, axes, deltas) -> GateSet:
    """The gate set of ``kind`` with over-rotation axes ``axes[k]`` (unit
    vectors over the non-identity Paulis) and angles ``deltas[k]``, composed
    with global depolarizing of strength ``lam``; ideal SPAM."""
    names, Us, n = ideal_unitaries(kind)
    d = 2 ** n
    P = pauli_basis(n)
    dep = depolarizing_ptm(lam, n)
    coh, G = [], []
    for U0, h, delta in zip(Us, axes, deltas):
        H = np.einsum("j,jab->ab", h, P[1:])
        U = expm_hermitian(H, delta / 2.0) @ U0
        coh.append(U)
        G.append(dep @ ptm_from_unitary(U))
    rho = vec_operator(np.diag(np.eye(d)[0]).astype(np.complex128))
    E = np.array([vec_operator(np.diag(np.eye(d)[m]).astype(np.complex128)) for m in range(d)])
    return GateSet(n, names, rho, E, np.ascontiguousarray(np.array(G)), np.array(coh), lam)


# ---------------------------------------------------------------------------
# Predictions of repeated gate applications (Sec. 6.3, Eq. GSTPrediction)
# ---------------------------------------------------------------------------
# The four initial states of the prediction test (Eqs. GSTInitialStatePrep00 -
# GSTInitialStatePrepPsi), as time-ordered words over the two-qubit gates
# (Gii, Gxi, Gix, Gyi, Giy, Gcz).  The thesis's singlet preparation ends with
# CNOT(0 -> 1); this gate set has CZ, and CNOT(0 -> 1) = (1 x Ry) CZ (1 x Ry^-1)
# with Ry = Ry(pi/2) and Ry^-1 = Ry^3 up to phase, i.e. Giy Giy Giy Gcz Giy.
PREDICTION_PREPS_2Q = {
    "00": (),
    "10": (1, 1),
    "++": (4, 3),
    "psi-": (2, 2, 1, 1, 3, 4, 4, 4, 5, 4),
}


@dataclasses.dataclass
class PredictionWorkload:
    estimate: GateSet      # the gate set whose predictions are evaluated
    ideal: GateSet         # ideal gates and SPAM (the reference distribution p^(id))
    preps: List[Tuple[int, ...]]
    gates: List[int]
    r_max: int


def prediction_workload(r_max: int = 1000) -> PredictionWorkload:
    """Two-qubit predictions for r = 0 .. r_max repetitions of every gate from the
    four initial states; the estimate is the C2 evaluation point (1e-3
    depolarizing and N(0, 0.01) over-rotations), the reference the ideal set."""
    estimate = noisy_gateset("2q", LAMBDA, SIGMA, _streams("c2")[3])
    names, Us, n = ideal_unitaries("2q")
    G = np.ascontiguousarray(np.array([ptm_from_unitary(U) for U in Us]))
    ideal = GateSet(n, names, estimate.rho.copy(), estimate.effects.copy(), G, np.array(Us), 0.0)
    return PredictionWorkload(estimate, ideal, list(PREDICTION_PREPS_2Q.values()), list(range(6)), r_max)


# ---------------------------------------------------------------------------
# Sequence lists (Sec. 6.3.1, Eq. GSTFullFiducialsGerms)
# ---------------------------------------------------------------------------
def shortlex_words(alphabet: Sequence[int], count: int) -> List[Tuple[int, ...]]:
    """First ``count`` words over ``alphabet`` in shortlex order, starting with the empty word."""
    out: List[Tuple[int, ...]] = []
    length = 0
    while len(out) < count:
        for w in itertools.product(alphabet, repeat=length):
            out.append(tuple(w))
            if len(out) == count:
                break
        length += 1
    return out


def _is_power(w: Tuple[int, ...]) -> bool:
    L = len(w)
    for p in range(1, L):
        if L % p == 0 and w == w[:p] * (L // p):
            return True
    return False


def random_germs(K: int, spec: Sequence[Tuple[int, int]], rng: np.random.Generator) -> List[Tuple[int, ...]]:
    """Every single-gate word, then ``count`` distinct random words per ``(length, count)`` in ``spec``
    that are not powers of shorter words."""
    germs: List[Tuple[int, ...]] = [(k,) for k in range(K)]
    seen = set(germs)
    for length, count in spec:
        pool = [w for w in itertools.product(range(K), repeat=length) if not _is_power(w) and w not in seen]
        if count > len(pool):
            raise ValueError(f"only {len(pool)} germs of length {length} exist")
        pick = rng.choice(len(pool), size=count, replace=False)
        for i in sorted(pick.tolist()):
            germs.append(tuple(pool[i]))
            seen.add(tuple(pool[i]))
    return germs


@dataclasses.dataclass
class SeqList:
    offsets: np.ndarray   # int64 [S+1]
    gates: np.ndarray     # uint8 [sum L]
    # optional structure labels (p, q, germ, power); -1 for bare sequences
    labels: Optional[np.ndarray] = None

    @property
    def S(self) -> int:
        return len(self.offsets) - 1

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def word(self, s: int) -> np.ndarray:
        return self.gates[self.offsets[s]:self.offsets[s + 1]]

    def subset(self, idx: np.ndarray) -> "SeqList":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths()[idx]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        g = np.concatenate([self.word(int(s)) for s in idx]) if len(idx) else np.zeros(0, np.uint8)
        lab = self.labels[idx] if self.labels is not None else None
        return SeqList(off, np.ascontiguousarray(g.astype(np.uint8)), lab)


def from_words(words: Sequence[Sequence[int]], labels=None) -> SeqList:
    lens = np.array([len(w) for w in words], dtype=np.int64)
    off = np.zeros(len(words) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    flat = np.fromiter(itertools.chain.from_iterable(words), dtype=np.uint8, count=int(off[-1]))
    return SeqList(off, flat, None if labels is None else np.asarray(labels))


def structured_list(preps, meas, germs, powers) -> SeqList:
    """Bare ``F_q F_p`` for all (p, q), then ``F_q g^l F_p`` for each germ, power, p, q.

    Words are in time order: ``F_p`` acts first.
    """
    words, labels = [], []
    for ip, fp in enumerate(preps):
        for iq, fq in enumerate(meas):
            words.append(tuple(fp) + tuple(fq))
            labels.append((ip, iq, -1, 0))
    for ig, g in enumerate(germs):
        for l in powers:
            gl = tuple(g) * l
            for ip, fp in enumerate(preps):
                for iq, fq in enumerate(meas):
                    words.append(tuple(fp) + gl + tuple(fq))
                    labels.append((ip, iq, ig, l))
    return from_words(words, labels)


def random_list(S: int, K: int, lmin: int, lmax: int, rng: np.random.Generator) -> SeqList:
    lens = rng.integers(lmin, lmax + 1, size=S).astype(np.int64)
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    g = rng.integers(0, K, size=int(off[-1]), dtype=np.uint8)
    return SeqList(off, g, None)


# ---------------------------------------------------------------------------
# The black box: outcome statistics emulated in Hilbert space
# ---------------------------------------------------------------------------
def _device_probs_words(gs: GateSet, sl: SeqList, idx: np.ndarray) -> np.ndarray:
    """Outcome distribution of the emulated device for the sequences ``idx``.

    The device applies the coherent unitaries to the state vector ``|0..0>``
    and the global depolarizing channel after every gate; since the latter
    commutes with unitaries, ``p = 1/d + (1-lam)^L (|<m|U_L..U_1|0>|^2 - 1/d)``
    (Eq. singletDepolarizingChannelSymmetricMixture).  Sequences are advanced
    together, one time step at a time.
    """
    d = 2 ** gs.n_qubits
    lens = sl.lengths()[idx]
    psi = np.zeros((len(idx), d), dtype=np.complex128)
    psi[:, 0] = 1.0
    order = np.argsort(-lens, kind="stable")
    Ls = lens[order]
    starts = sl.offsets[idx][order]
    U = gs.unitaries
    for t in range(int(Ls.max()) if len(Ls) else 0):
        active = int(np.searchsorted(-Ls, -t, side="left"))  # sequences with L > t
        active = int(np.sum(Ls > t))
        g = sl.gates[starts[:active] + t]
        psi[order[:active]] = np.einsum("sab,sb->sa", U[g], psi[order[:active]])
    pc = np.abs(psi) ** 2
    f = (1.0 - gs.lam) ** lens.astype(np.float64)
    return 1.0 / d + f[:, None] * (pc - 1.0 / d)


def device_probs_structured(gs: GateSet, preps, meas, germs, powers, sl: SeqList) -> np.ndarray:
    """Same emulation, using the fiducial/germ structure to multiply unitaries once."""
    d = 2 ** gs.n_qubits
    U = gs.unitaries

    def word_u(w):
        m = np.eye(d, dtype=np.complex128)
        for k in w:
            m = U[k] @ m
        return m

    Up = [word_u(w) for w in preps]
    Uq = [word_u(w) for w in meas]
    out = np.empty((sl.S, d))
    lens = sl.lengths().astype(np.float64)
    lab = sl.labels
    e0 = np.zeros(d, dtype=np.complex128)
    e0[0] = 1
    cache: Dict[Tuple[int, int], np.ndarray] = {}
    for s in range(sl.S):
        ip, iq, ig, l = lab[s]
        if ig < 0:
            M = Uq[iq] @ Up[ip]
        else:
            key = (int(ig), int(l))
            if key not in cache:
                gu = word_u(germs[ig])
                cache[key] = np.linalg.matrix_power(gu, int(l))
            M = Uq[iq] @ cache[key] @ Up[ip]
        amp = M @ e0
        out[s] = np.abs(amp) ** 2
    f = (1.0 - gs.lam) ** lens
    return 1.0 / d + f[:, None] * (out - 1.0 / d)


def sample_counts(p: np.ndarray, n_shots: int, rng: np.random.Generator) -> np.ndarray:
    p = np.clip(p, 0.0, None)
    p = p / p.sum(axis=1, keepdims=True)
    return rng.multinomial(n_shots, p).astype(np.int32)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
MASTER_SEEDS = {"c1": 2008134901, "c2": 2008134902, "c3": 2008134903, "c4": 2008134904, "c5": 2008134905}
LAMBDA = 1e-3
SIGMA = 0.01
N_SHOTS = 1000


@dataclasses.dataclass
class Workload:
    name: str
    truth: GateSet     # generates the counts
    model: GateSet     # the evaluation point (over-rotations redrawn, same lambda)
    seqs: SeqList
    counts: np.ndarray  # int32 [S, M]

    @property
    def n_qubits(self) -> int:
        return self.model.n_qubits


def _streams(name: str, n: int = 6):
    ss = np.random.SeedSequence(MASTER_SEEDS[name])
    return [np.random.default_rng(s) for s in ss.spawn(n)]


_STRUCTURED = {
    # kind, fiducial alphabet, number of fiducials, germ spec, powers
    "c1": ("1q", (1, 2), 6, [(3, 1)], [1, 2, 4, 8, 16, 32, 64]),
    "c2": ("2q", (1, 2, 3, 4), 11, [(2, 3), (3, 3)], [1, 2, 4, 8, 16, 32, 64, 128, 256]),
    "c4": ("3q", (1, 2), 16, [(2, 20), (3, 73)], [1, 2, 4, 8, 16, 32, 64, 128]),
}


def structured_workload(name: str) -> Workload:
    """C1 (1 qubit), C2 (2 qubits) or C4 (3 qubits): fiducial x germ-power x fiducial lists."""
    kind, alpha, nf, spec, powers = _STRUCTURED[name]
    r_rot, r_germ, r_cnt, r_pert, _, _ = _streams(name)
    truth = noisy_gateset(kind, LAMBDA, SIGMA, r_rot)
    model = noisy_gateset(kind, LAMBDA, SIGMA, r_pert)
    fids = shortlex_words(alpha, nf)
    germs = random_germs(truth.K, spec, r_germ)
    sl = structured_list(fids, fids, germs, powers)
    p = device_probs_structured(truth, fids, fids, germs, powers, sl)
    counts = sample_counts(p, N_SHOTS, r_cnt)
    return Workload(name, truth, model, sl, counts)


def random_workload(kind: str, S: int, lmax: int, seed: int, lmin: int = 1) -> Workload:
    """Random words over the gate set of ``kind``, lengths uniform in ``lmin..lmax``."""
    ss = np.random.SeedSequence(seed)
    r_rot, r_seq, r_cnt, r_pert = [np.random.default_rng(s) for s in ss.spawn(4)]
    truth = noisy_gateset(kind, LAMBDA, SIGMA, r_rot)
    model = noisy_gateset(kind, LAMBDA, SIGMA, r_pert)
    sl = random_list(S, truth.K, lmin, lmax, r_seq)
    p = _device_probs_words(truth, sl, np.arange(S))
    counts = sample_counts(p, N_SHOTS, r_cnt)
    return Workload(f"random-{kind}-S{S}-L{lmax}-seed{seed}", truth, model, sl, counts)


def c3_plan(n_sets: int = 512, seed: Optional[int] = None):
    """Uneven batch: per gate set (kind, S, seed).  70% one-qubit, 30% two-qubit
    (a seeded permutation), ``S ~ U{500..20000}``, lengths ``U{1..1024}``."""
    rng = np.random.default_rng(np.random.SeedSequence(MASTER_SEEDS["c3"] if seed is None else seed).spawn(5)[4])
    n1 = int(round(0.7 * n_sets))
    kinds = np.array(["1q"] * n1 + ["2q"] * (n_sets - n1))
    kinds = kinds[rng.permutation(n_sets)]
    S = rng.integers(500, 20001, size=n_sets)
    seeds = rng.integers(1, 2 ** 62, size=n_sets)
    return [(str(k), int(s), int(sd)) for k, s, sd in zip(kinds, S, seeds)]


def uneven_request(kind: str, S: int, seed: int, lmax: int = 1024, emulate: bool = False) -> Workload:
    """One gate set of the uneven batch: random words with lengths ``U{1..lmax}``.

    With ``emulate`` the counts are drawn from the emulated device (the
    state-vector black box, slow at full size); otherwise from the uniform
    distribution over outcomes, which leaves the cost of an evaluation
    unchanged (only zero counts are skipped, and they are as rare)."""
    ss = np.random.SeedSequence(seed)
    r_rot, r_seq, r_cnt, r_pert = [np.random.default_rng(x) for x in ss.spawn(4)]
    truth = noisy_gateset(kind, LAMBDA, SIGMA, r_rot)
    model = noisy_gateset(kind, LAMBDA, SIGMA, r_pert)
    sl = random_list(S, truth.K, 1, lmax, r_seq)
    if emulate:
        p = _device_probs_words(truth, sl, np.arange(S))
    else:
        p = np.full((S, truth.M), 1.0 / truth.M)
    counts = sample_counts(p, N_SHOTS, r_cnt)
    return Workload(f"uneven-{kind}-S{S}-seed{seed}", truth, model, sl, counts)


@dataclasses.dataclass
class FitRequestData:
    """A fit request of the serving workload: random words, counts, and the
    gate sets of its optimizer iterations."""
    kind: str
    seqs: SeqList
    counts: np.ndarray
    iterates: List[GateSet]

    @property
    def n_qubits(self) -> int:
        return self.iterates[0].n_qubits


def serving_trace(rate: float, n_requests: int, seed: Optional[int] = None, smin: int = 1000,
                  smax: int = 100000):
    """Poisson arrivals at ``rate`` per second: (arrival time, kind, S, seed)
    with kinds one/two/three qubits in 60/30/10 proportion and S log-uniform
    in [smin, smax]."""
    rng = np.random.default_rng(np.random.SeedSequence(MASTER_SEEDS["c5"] if seed is None else seed).spawn(6)[5])
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.choice(np.array(["1q", "2q", "3q"]), size=n_requests, p=[0.6, 0.3, 0.1])
    S = np.exp(rng.uniform(np.log(smin), np.log(smax), size=n_requests)).astype(np.int64)
    seeds = rng.integers(1, 2 ** 62, size=n_requests)
    return [(float(a), str(k), int(s), int(sd)) for a, k, s, sd in zip(t, kinds, S, seeds)]


def serving_request(kind: str, S: int, seed: int, n_iter: int = 20) -> FitRequestData:
    """Random words with lengths U{1..256} (one and two qubits) or U{1..128}
    (three qubits); counts ~ Multinomial(1000, uniform) (the cost of an
    evaluation does not depend on their values); iterate k has the
    over-rotation angles delta_true + (1 - k / n_iter) * delta_pert about
    fixed axes, a CPTP schedule ending next to the truth."""
    ss = np.random.SeedSequence(seed)
    r_rot, r_seq, r_cnt, r_pert = [np.random.default_rng(x) for x in ss.spawn(4)]
    _, Us, n = ideal_unitaries(kind)
    D = 4 ** n
    axes = [random_axis(r_rot, D) for _ in Us]
    d_true = r_rot.normal(0.0, SIGMA, size=len(Us))
    d_pert = r_pert.normal(0.0, SIGMA, size=len(Us))
    lmax = 128 if kind == "3q" else 256
    sl = random_list(S, len(Us), 1, lmax, r_seq)
    M = 2 ** n
    counts = sample_counts(np.full((S, M), 1.0 / M), N_SHOTS, r_cnt)
    its = [gateset_from_rotations(kind, LAMBDA, axes, d_true + (1.0 - k / n_iter) * d_pert) for k in range(n_iter)]
    return FitRequestData(kind, sl, counts, its)


def pack_params(gs: GateSet) -> np.ndarray:
    """Full parameter vector in gradient layout ``[rho (D) | E (M*D) | G (K*D*D)]``."""
    return np.concatenate([gs.rho.ravel(), gs.effects.ravel(), gs.gates.ravel()])


def unpack_params(theta: np.ndarray, n_qubits: int, M: int, K: int):
    D = 4 ** n_qubits
    rho = theta[:D]
    E = theta[D:D + M * D].reshape(M, D)
    G = theta[D + M * D:].reshape(K, D, D)
    return rho, E, G


def param_point(mode: str, gs: GateSet, seed: int, scale: float = 0.03) -> np.ndarray:
    """A seeded parameter vector of an estimation mode (layouts of gst_param_*).

    full: the gate set's own parameters.  tp: rho[1:], the first M - 1 effects
    and rows 1.. of the gates of a trace-preserving set with a complete POVM
    (as given).  cptp: the state parameter e_0 plus N(0, scale^2 / 100) entries
    (|0..0> nearly), the first M - 1 effects of the set, and per gate a
    Hamiltonian part h ~ N(0, scale^2) and a dissipator factor with diagonal
    scale (1 + |N(0, 1)|) and entries below it ~ N(0, (0.3 scale)^2), about the
    ideal gates as targets."""
    D, M, K = gs.D, gs.M, gs.K
    if mode == "full":
        return pack_params(gs)
    if mode == "tp":
        return np.concatenate([gs.rho[1:], gs.effects[:M - 1].ravel(), gs.gates[:, 1:, :].ravel()])
    assert mode == "cptp"
    rng = np.random.default_rng(seed)
    A = rng.normal(size=D) * scale * 0.1
    A[0] = 1.0
    m = D - 1
    parts = [A, gs.effects[:M - 1].ravel()]
    for _ in range(K):
        parts += [rng.normal(size=m) * scale, scale * (1.0 + np.abs(rng.normal(size=m))),
                  rng.normal(size=m * (m - 1)) * scale * 0.3]
    return np.concatenate(parts)


def ideal_targets(kind: str) -> np.ndarray:
    """Transfer matrices of the ideal gates of ``kind`` (the CPTP targets)."""
    _, Us, _ = ideal_unitaries(kind)
    return np.ascontiguousarray(np.array([ptm_from_unitary(U) for U in Us]))


# ---------------------------------------------------------------------------
# The fit (Sec. 6.3.1-6.3.2): LGST sequences and iterative MLGST stages
# ---------------------------------------------------------------------------
# Informationally complete product fiducials over (Gii, Gxi, Gix, Gyi, Giy, Gcz):
# per qubit {empty, X(pi/2), Y(pi/2), X(pi/2) X(pi/2)} (|0>, a Y and an X
# eigenstate, |1>); the 16 combinations prepare, 11 of them measure (with four
# outcomes each), as many as the thesis's list uses.
FIT_PREP_FIDUCIALS_2Q = [a + b for a in ((), (1,), (3,), (1, 1)) for b in ((), (2,), (4,), (2, 2))]
FIT_MEAS_FIDUCIALS_2Q = [(), (2,), (4,), (1,), (1, 2), (1, 4), (3,), (3, 2), (3, 4), (1, 1), (2, 2)]
FIT_MAX_LENGTHS = (1, 2, 4, 8, 16, 32)


@dataclasses.dataclass
class FitWorkload:
    truth: GateSet            # generates the counts
    target: GateSet           # the ideal gates (CPTP targets, gauge optimization)
    prep_fids: List[Tuple[int, ...]]
    meas_fids: List[Tuple[int, ...]]
    germs: List[Tuple[int, ...]]
    max_lengths: Tuple[int, ...]
    seqs: SeqList             # every sequence: LGST words first, then by stage
    counts: np.ndarray        # int32 [S, M]
    stage_end: List[int]      # stage s fits sequences [0, stage_end[s])


def fit_words(prep_fids, meas_fids, germs, max_lengths, K):
    """LGST words F_q F_p and F_q G_k F_p (time order: F_p first), then for each
    maximum length L the words F_q g^p F_p with p = floor(L / |g|) >= 1 not
    listed before; returns the words and the end of each stage (stage 0 = LGST)."""
    words, seen, ends = [], set(), []

    def add(w):
        if w not in seen:
            seen.add(w)
            words.append(w)

    for fp in prep_fids:
        for fq in meas_fids:
            add(tuple(fp) + tuple(fq))
    for k in range(K):
        for fp in prep_fids:
            for fq in meas_fids:
                add(tuple(fp) + (k,) + tuple(fq))
    ends.append(len(words))
    for L in max_lengths:
        for g in germs:
            p = L // len(g)
            if p < 1:
                continue
            for fp in prep_fids:
                for fq in meas_fids:
                    add(tuple(fp) + tuple(g) * p + tuple(fq))
        ends.append(len(words))
    return words, ends


def fit_workload() -> FitWorkload:
    """The two-qubit fit: the C2 truth and germs, the informationally complete
    fiducials above, maximum lengths 1..32 (at most 38 gates per sequence),
    counts ~ Multinomial(1000) from the emulated device."""
    kind = "2q"
    r_rot, r_germ, r_cnt, _, _, _ = _streams("c2")
    truth = noisy_gateset(kind, LAMBDA, SIGMA, r_rot)
    germs = random_germs(truth.K, _STRUCTURED["c2"][3], r_germ)
    words, ends = fit_words(FIT_PREP_FIDUCIALS_2Q, FIT_MEAS_FIDUCIALS_2Q, germs, FIT_MAX_LENGTHS, truth.K)
    sl = from_words(words)
    p = _device_probs_words(truth, sl, np.arange(sl.S))
    counts = sample_counts(p, N_SHOTS, np.random.default_rng(np.random.SeedSequence(MASTER_SEEDS["c2"] + 100)))
    names, Us, n = ideal_unitaries(kind)
    G = np.ascontiguousarray(np.array([ptm_from_unitary(U) for U in Us]))
    target = GateSet(n, names, truth.rho.copy(), truth.effects.copy(), G, np.array(Us), 0.0)
    return FitWorkload(truth, target, list(FIT_PREP_FIDUCIALS_2Q), list(FIT_MEAS_FIDUCIALS_2Q), germs,
                       FIT_MAX_LENGTHS, sl, counts, ends)
