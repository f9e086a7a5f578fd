"""ctypes binding of ``gst_oracle.c`` (test infrastructure only).

Argument marshalling only: every number is computed by the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gst_oracle.c")
_LIB = os.path.join(_HERE, "libgst_oracle.so")
_lib = None


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle returned {code}: {msg}")
        self.code = code


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64 plus FMA, no fast-math, no contraction)."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_int64
        lib.oracle_probs.argtypes = [I, I, I, P, P, P, L, P, P, P]
        lib.oracle_probs_extended.argtypes = [I, I, I, P, P, P, L, P, P, P]
        lib.oracle_loglik.argtypes = [I, I, I, P, P, P, L, P, P, P, P, P, P, P]
        lib.oracle_vjp.argtypes = [I, I, I, P, P, P, L, P, P, P, P]
        lib.oracle_tv_distance.argtypes = [L, I, P, P, P]
        for f in (lib.oracle_probs, lib.oracle_probs_extended, lib.oracle_loglik, lib.oracle_vjp):
            f.restype = I
        _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _common(rho, E, G, offsets, gates):
    rho = _c(rho, np.float64)
    E = _c(E, np.float64)
    G = _c(G, np.float64)
    offsets = _c(offsets, np.int64)
    gates = _c(gates, np.uint8)
    D = rho.shape[0]
    M = E.shape[0]
    K = G.shape[0]
    if E.shape != (M, D) or G.shape != (K, D, D):
        raise ValueError("shape mismatch")
    if gates.size == 0:
        gates = np.zeros(1, np.uint8)
    return rho, E, G, offsets, gates, D, M, K


_MSG = {-1: "invalid argument", -2: "gate index out of range", -3: "probability <= 0 with count > 0"}


def probs(rho, E, G, offsets, gates) -> np.ndarray:
    rho, E, G, offsets, gates, D, M, K = _common(rho, E, G, offsets, gates)
    S = len(offsets) - 1
    out = np.empty((S, M), np.float64)
    rc = _load().oracle_probs(D, M, K, _ptr(rho), _ptr(E), _ptr(G), S, _ptr(offsets), _ptr(gates), _ptr(out))
    if rc:
        raise OracleError(rc, _MSG.get(rc, "?"))
    return out


def probs_extended(rho, E, G, offsets, gates) -> np.ndarray:
    rho, E, G, offsets, gates, D, M, K = _common(rho, E, G, offsets, gates)
    S = len(offsets) - 1
    out = np.empty((S, M), np.float64)
    rc = _load().oracle_probs_extended(D, M, K, _ptr(rho), _ptr(E), _ptr(G), S, _ptr(offsets), _ptr(gates), _ptr(out))
    if rc:
        raise OracleError(rc, _MSG.get(rc, "?"))
    return out


def loglik(rho, E, G, offsets, gates, counts, want_grad: bool = True, raise_nonpos: bool = True
           ) -> Tuple[float, np.ndarray, Optional[np.ndarray], int, int]:
    """Returns ``(objective, probs, grad or None, n_nonpos, status)``."""
    rho, E, G, offsets, gates, D, M, K = _common(rho, E, G, offsets, gates)
    S = len(offsets) - 1
    counts = _c(counts, np.int32).reshape(S, M)
    p = np.empty((S, M), np.float64)
    obj = np.zeros(1, np.float64)
    nbad = np.zeros(1, np.int64)
    grad = np.empty(D + M * D + K * D * D, np.float64) if want_grad else None
    rc = _load().oracle_loglik(D, M, K, _ptr(rho), _ptr(E), _ptr(G), S, _ptr(offsets), _ptr(gates),
                               _ptr(counts), _ptr(p), _ptr(obj), _ptr(grad), _ptr(nbad))
    if rc and not (rc == -3 and not raise_nonpos):
        raise OracleError(rc, _MSG.get(rc, "?"))
    return float(obj[0]), p, grad, int(nbad[0]), int(rc)


def vjp(rho, E, G, offsets, gates, W) -> np.ndarray:
    rho, E, G, offsets, gates, D, M, K = _common(rho, E, G, offsets, gates)
    S = len(offsets) - 1
    W = _c(W, np.float64).reshape(S, M)
    grad = np.empty(D + M * D + K * D * D, np.float64)
    rc = _load().oracle_vjp(D, M, K, _ptr(rho), _ptr(E), _ptr(G), S, _ptr(offsets), _ptr(gates), _ptr(W), _ptr(grad))
    if rc:
        raise OracleError(rc, _MSG.get(rc, "?"))
    return grad


def tv_distance(p, q) -> np.ndarray:
    """Statistical distance 1/2 sum_J |p_J - q_J| over the last axis (Eq. statisticaldistance)."""
    p = _c(p, np.float64)
    q = _c(q, np.float64)
    assert p.shape == q.shape and p.ndim >= 1
    m = p.shape[-1]
    out = np.empty(p.shape[:-1], np.float64)
    rc = _load().oracle_tv_distance(p.size // m, m, _ptr(p), _ptr(q), _ptr(out))
    if rc:
        raise OracleError(rc, _MSG.get(rc, "?"))
    return out


def predict(rho, E, G, preps, gates, r_max: int) -> np.ndarray:
    """Predictions of repeated gate applications, Eq. GSTPrediction: the plain
    probabilities of the words prep + [s] * r (time order) for every preparation
    word, gate s and r = 0..r_max, as an array [n_prep, n_gates, r_max + 1, M]."""
    words = [list(w) + [int(s)] * r for w in preps for s in gates for r in range(r_max + 1)]
    off = np.zeros(len(words) + 1, np.int64)
    for x, w in enumerate(words):
        off[x + 1] = off[x] + len(w)
    flat = np.fromiter((g for w in words for g in w), np.uint8, count=int(off[-1]))
    p = probs(rho, E, G, off, flat)
    return p.reshape(len(preps), len(gates), r_max + 1, -1)
