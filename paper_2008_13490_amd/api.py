"""Python front end of the HIP library: torch tensors in, torch tensors out.

Argument marshalling only (``_lib`` holds the ctypes declarations).  Every
probability, objective and gradient is computed by the kernels in
``libgst.so``; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib

_DEV = torch.device("cuda")


def _require_cuda(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    return t.contiguous()


@dataclasses.dataclass
class DeviceGateSet:
    """theta = (rho [D], effects [M, D], gates [K, D, D]) as float64 device tensors."""
    n_qubits: int
    rho: torch.Tensor
    effects: torch.Tensor
    gates: torch.Tensor

    @property
    def D(self):
        return 4 ** self.n_qubits

    @property
    def M(self):
        return self.effects.shape[0]

    @property
    def K(self):
        return self.gates.shape[0]

    def n_params(self):
        return self.D + self.M * self.D + self.K * self.D * self.D

    @staticmethod
    def from_numpy(n_qubits, rho, effects, gates, device=None):
        dev = device or _DEV
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
        return DeviceGateSet(n_qubits, f(rho), f(effects), f(gates))

    def as_struct(self) -> _lib.GstGateset:
        D = self.D
        rho = _require_cuda(self.rho, torch.float64, "rho")
        E = _require_cuda(self.effects, torch.float64, "effects")
        G = _require_cuda(self.gates, torch.float64, "gates")
        if rho.shape != (D,) or E.dim() != 2 or E.shape[1] != D or G.dim() != 3 or G.shape[1:] != (D, D):
            raise ValueError("gate set shapes do not match n_qubits")
        self._keep = (rho, E, G)
        return _lib.GstGateset(self.n_qubits, G.shape[0], E.shape[0], rho.data_ptr(), E.data_ptr(), G.data_ptr())


@dataclasses.dataclass
class DeviceSeqs:
    """CSR sequence list on the device: offsets int64 [S+1], gate indices uint8 (time order)."""
    offsets: torch.Tensor
    gates: torch.Tensor
    max_len: int

    @property
    def S(self):
        return self.offsets.shape[0] - 1

    @staticmethod
    def from_numpy(offsets, gates, device=None):
        dev = device or _DEV
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        g = np.ascontiguousarray(gates, dtype=np.uint8)
        if g.size == 0:
            g = np.zeros(1, np.uint8)
        ml = int(np.diff(off).max()) if len(off) > 1 else 0
        return DeviceSeqs(torch.as_tensor(off, device=dev), torch.as_tensor(g, device=dev), ml)

    def as_struct(self) -> _lib.GstSeqlist:
        off = _require_cuda(self.offsets, torch.int64, "offsets")
        g = _require_cuda(self.gates, torch.uint8, "gates")
        self._keep = (off, g)
        return _lib.GstSeqlist(off.shape[0] - 1, off.data_ptr(), g.data_ptr(), int(self.max_len))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One ``gst_ctx`` bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        self.lib = _lib.load()
        torch.cuda.set_device(device)
        self.stream = stream or torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _lib.check(self.lib.gst_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream)))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gst_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        return torch.device("cuda", self.device)

    def sync(self, raise_on_error: bool = True) -> Tuple[int, int, int]:
        """Wait for the context's work; returns (status, n_bad_index, n_nonpos)."""
        d = _lib.GstDiag()
        rc = self.lib.gst_sync(self.handle, ctypes.byref(d))
        if raise_on_error and rc not in (_lib.GST_OK,):
            _lib.check(rc)
        return rc, d.n_bad_index, d.n_nonpos

    def probs(self, gs: DeviceGateSet, seqs: DeviceSeqs, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = out if out is not None else torch.empty((seqs.S, gs.M), dtype=torch.float64, device=self._dev())
        _lib.check(self.lib.gst_probs(self.handle, ctypes.byref(gs.as_struct()), ctypes.byref(seqs.as_struct()),
                                      _ptr(out)))
        return out

    def loglik(self, gs: DeviceGateSet, seqs: DeviceSeqs, counts: torch.Tensor, want_probs: bool = False,
               want_grad: bool = True):
        """Returns (objective [1], probs [S, M] or None, grad [P] or None), all on the device."""
        counts = _require_cuda(counts, torch.int32, "counts")
        obj = torch.empty(1, dtype=torch.float64, device=self._dev())
        p = torch.empty((seqs.S, gs.M), dtype=torch.float64, device=self._dev()) if want_probs else None
        g = torch.empty(gs.n_params(), dtype=torch.float64, device=self._dev()) if want_grad else None
        _lib.check(self.lib.gst_loglik(self.handle, ctypes.byref(gs.as_struct()), ctypes.byref(seqs.as_struct()),
                                       _ptr(counts), _ptr(p), _ptr(obj), _ptr(g)))
        return obj, p, g

    def loglik_noalloc(self, gs: DeviceGateSet, seqs: DeviceSeqs, counts: torch.Tensor, out):
        """``gst_loglik_noalloc`` into preallocated outputs (objective [1], probs [S, M]
        or None, grad [P] or None): the call allocates nothing."""
        counts = _require_cuda(counts, torch.int32, "counts")
        obj, p, g = out
        _lib.check(self.lib.gst_loglik_noalloc(self.handle, ctypes.byref(gs.as_struct()),
                                               ctypes.byref(seqs.as_struct()), _ptr(counts), _ptr(p), _ptr(obj),
                                               _ptr(g)))
        return obj, p, g

    def vjp(self, gs: DeviceGateSet, seqs: DeviceSeqs, w: torch.Tensor) -> torch.Tensor:
        w = _require_cuda(w, torch.float64, "w")
        g = torch.empty(gs.n_params(), dtype=torch.float64, device=self._dev())
        _lib.check(self.lib.gst_vjp(self.handle, ctypes.byref(gs.as_struct()), ctypes.byref(seqs.as_struct()),
                                    _ptr(w), _ptr(g)))
        return g


class Request:
    """A resident request (``gst_req``): sequences and counts live on the device,
    the sharing plan is built once, and each evaluation takes a new gate set."""

    def __init__(self, ctx: Context, n_qubits: int, n_gates: int, n_outcomes: int, offsets, gates, counts=None):
        self.ctx = ctx
        self.lib = ctx.lib
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        g = np.ascontiguousarray(gates, dtype=np.uint8)
        if g.size == 0:
            g = np.zeros(1, np.uint8)
        ml = int(np.diff(off).max()) if len(off) > 1 else 0
        sl = _lib.GstSeqlist(len(off) - 1, off.ctypes.data, g.ctypes.data, ml)
        c = None
        if counts is not None:
            c = np.ascontiguousarray(counts, dtype=np.int32)
        h = ctypes.c_void_p()
        _lib.check(self.lib.gst_req_create_host(ctx.handle, n_qubits, n_gates, n_outcomes, ctypes.byref(sl),
                                                None if c is None else c.ctypes.data, ctypes.byref(h)))
        self.handle = h
        self.has_counts = counts is not None
        self.S = len(off) - 1
        self.M = n_outcomes
        self.n_params = 4 ** n_qubits * (1 + n_outcomes) + n_gates * 16 ** n_qubits

    @classmethod
    def from_device(cls, ctx: Context, n_qubits: int, n_gates: int, n_outcomes: int, seqs: "DeviceSeqs",
                    counts: Optional[torch.Tensor] = None) -> "Request":
        """A request from a sequence list and counts already on the device (``gst_req_create``)."""
        self = cls.__new__(cls)
        self.ctx, self.lib = ctx, ctx.lib
        if counts is not None:
            counts = _require_cuda(counts, torch.int32, "counts")
        h = ctypes.c_void_p()
        _lib.check(self.lib.gst_req_create(ctx.handle, n_qubits, n_gates, n_outcomes, ctypes.byref(seqs.as_struct()),
                                           _ptr(counts), ctypes.byref(h)))
        self.handle = h
        self.has_counts = counts is not None
        self.S = seqs.S
        self.M = n_outcomes
        self.n_params = 4 ** n_qubits * (1 + n_outcomes) + n_gates * 16 ** n_qubits
        return self

    def plan_info(self) -> dict:
        v = (ctypes.c_int64 * 16)()
        _lib.check(self.lib.gst_req_plan_info(self.handle, v, 16))
        keys = ["plan_used", "sum_len", "trie_nodes", "trunks", "trunk_steps", "item_steps", "levels", "inj_slots",
                "chain_steps", "chain_max", "jump_trunks", "fill_tasks", "grouped", "tiles", "chains", "rows"]
        return dict(zip(keys, [int(x) for x in v]))

    def footprint(self) -> int:
        b = ctypes.c_size_t()
        _lib.check(self.lib.gst_req_footprint(self.handle, ctypes.byref(b)))
        return b.value

    def eval(self, gs: DeviceGateSet, want_probs=False, want_grad=True, out=None):
        dev = self.ctx._dev()
        obj, p, g = out if out is not None else (
            torch.empty(1, dtype=torch.float64, device=dev),
            torch.empty((self.S, self.M), dtype=torch.float64, device=dev) if want_probs else None,
            torch.empty(self.n_params, dtype=torch.float64, device=dev) if want_grad else None)
        _lib.check(self.lib.gst_req_eval(self.handle, ctypes.byref(gs.as_struct()), _ptr(p), _ptr(obj), _ptr(g)))
        return obj, p, g

    def probs(self, gs: DeviceGateSet, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        p = out if out is not None else torch.empty((self.S, self.M), dtype=torch.float64, device=self.ctx._dev())
        _lib.check(self.lib.gst_req_probs(self.handle, ctypes.byref(gs.as_struct()), _ptr(p)))
        return p

    def vjp(self, gs: DeviceGateSet, w: torch.Tensor) -> torch.Tensor:
        w = _require_cuda(w, torch.float64, "w")
        g = torch.empty(self.n_params, dtype=torch.float64, device=self.ctx._dev())
        _lib.check(self.lib.gst_req_vjp(self.handle, ctypes.byref(gs.as_struct()), _ptr(w), _ptr(g)))
        return g

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gst_req_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several resident requests evaluated together (``gst_batch``).

    ``thetas`` are DeviceGateSets whose tensors stay allocated (their contents
    may change between runs); outputs are allocated here per request."""

    def __init__(self, ctx: Context, reqs, thetas, want_probs=False, want_grad=True, capture_graph=False):
        self.ctx, self.lib = ctx, ctx.lib
        n = len(reqs)
        dev = ctx._dev()
        self.reqs, self.thetas = list(reqs), list(thetas)
        self.obj = [torch.empty(1, dtype=torch.float64, device=dev) if r.has_counts else None for r in reqs]
        self.probs = [torch.empty((r.S, r.M), dtype=torch.float64, device=dev) if want_probs else None for r in reqs]
        self.grad = [torch.empty(r.n_params, dtype=torch.float64, device=dev) if want_grad and r.has_counts else None
                     for r in reqs]
        gs = (_lib.GstGateset * max(n, 1))(*[t.as_struct() for t in self.thetas])
        ptrs = lambda ts: (ctypes.c_void_p * max(n, 1))(*[None if t is None else t.data_ptr() for t in ts])
        h = ctypes.c_void_p()
        rq = (ctypes.c_void_p * max(n, 1))(*[r.handle.value for r in reqs])
        _lib.check(self.lib.gst_batch_create(ctx.handle, n, rq, gs, ptrs(self.probs), ptrs(self.obj), ptrs(self.grad),
                                             1 if capture_graph else 0, ctypes.byref(h)))
        self.handle = h

    def run(self):
        _lib.check(self.lib.gst_batch_run(self.handle))

    def nonpos(self):
        v = (ctypes.c_int64 * max(len(self.reqs), 1))()
        _lib.check(self.lib.gst_batch_nonpos(self.handle, v))
        return [int(x) for x in v[:len(self.reqs)]]

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gst_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_set(ctx: Context, n_qubits: int, seqs_per_tile: int = 0, blocks_per_cu: int = 0):
    """Tile policy for requests created afterwards on ``ctx`` (``gst_tune_set``)."""
    _lib.check(ctx.lib.gst_tune_set(ctx.handle, n_qubits, seqs_per_tile, blocks_per_cu))


class Predictor:
    """Predictions of repeated gate applications (``gst_predict``) for fixed
    preparation words (time order), gate indices and r_max: the host arrays are
    marshalled once; each call evaluates a gate set into a tensor
    ``[len(preps), len(gates), r_max + 1, M]`` of <<E_m| G_s^r G_prep |rho>>."""

    def __init__(self, ctx: Context, preps, gates, r_max: int):
        import numpy as np
        self.ctx = ctx
        self.n_prep = len(preps)
        off = np.zeros(len(preps) + 1, np.int64)
        for x, w in enumerate(preps):
            off[x + 1] = off[x] + len(w)
        self._off = off
        self._words = np.ascontiguousarray(np.concatenate([np.asarray(w, np.uint8) for w in preps])
                                           if off[-1] > 0 else np.zeros(1, np.uint8))
        self._gates = np.ascontiguousarray(np.asarray(gates, np.int32))
        self.r_max = int(r_max)

    def shape(self, M: int):
        return (self.n_prep, len(self._gates), self.r_max + 1, M)

    def __call__(self, gs: "DeviceGateSet", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        shape = self.shape(gs.M)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=self.ctx._dev())
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == shape):
            raise ValueError(f"out must be a contiguous float64 device tensor of shape {shape}")
        _lib.check(self.ctx.lib.gst_predict(self.ctx.handle, ctypes.byref(gs.as_struct()), self.n_prep,
                                            self._off.ctypes.data, self._words.ctypes.data, len(self._gates),
                                            self._gates.ctypes.data, self.r_max, _ptr(out)))
        return out


def predict(ctx: Context, gs: "DeviceGateSet", preps, gates, r_max: int,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """One-off ``Predictor(ctx, preps, gates, r_max)(gs, out)``."""
    return Predictor(ctx, preps, gates, r_max)(gs, out)


def tv_distance(ctx: Context, p: torch.Tensor, q: torch.Tensor,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Statistical distance 1/2 sum_m |p - q| over the last axis (``gst_tv_distance``)."""
    assert p.shape == q.shape and p.dtype == torch.float64 and q.dtype == torch.float64
    m = p.shape[-1]
    p2, q2 = p.contiguous(), q.contiguous()
    if out is None:
        out = torch.empty(p.shape[:-1], dtype=torch.float64, device=p.device)
    assert out.shape == p.shape[:-1] and out.is_contiguous() and out.dtype == torch.float64
    _lib.check(ctx.lib.gst_tv_distance(ctx.handle, _ptr(p2), _ptr(q2), p2.numel() // m, m, _ptr(out)))
    return out


class Parameterization:
    """Estimation mode of a fit (``gst_param_*``): ``"full"``, ``"tp"`` or
    ``"cptp"``.  ``forward(theta)`` gives the gate set of a parameter vector;
    ``backward(theta, grad_full)`` the gradient with respect to theta from the
    gradient with respect to the full parameters ([rho | effects | gates]).
    ``targets`` (CPTP): the fixed gates G0, a float64 device tensor [K, D, D]."""

    MODES = {"full": 0, "tp": 1, "cptp": 2}

    def __init__(self, ctx: Context, mode: str, n_qubits: int, n_outcomes: int, n_gates: int,
                 targets: Optional[torch.Tensor] = None):
        self.ctx, self.mode = ctx, self.MODES[mode]
        self.n_qubits, self.M, self.K = n_qubits, n_outcomes, n_gates
        self.D = 4 ** n_qubits
        cnt = ctypes.c_int64(0)
        _lib.check(ctx.lib.gst_param_count(self.mode, n_qubits, n_outcomes, n_gates, ctypes.byref(cnt)))
        self.count = int(cnt.value)
        self.targets = None if targets is None else _require_cuda(targets, torch.float64, "targets")
        if self.targets is not None and tuple(self.targets.shape) != (n_gates, self.D, self.D):
            raise ValueError("targets must be [K, D, D]")

    def _theta(self, theta: torch.Tensor) -> torch.Tensor:
        theta = _require_cuda(theta, torch.float64, "theta")
        if tuple(theta.shape) != (self.count,):
            raise ValueError(f"theta must have {self.count} entries")
        return theta

    def forward(self, theta: torch.Tensor, out: Optional["DeviceGateSet"] = None) -> "DeviceGateSet":
        theta = self._theta(theta)
        if out is None:
            dev = theta.device
            out = DeviceGateSet(self.n_qubits, torch.empty(self.D, dtype=torch.float64, device=dev),
                                torch.empty((self.M, self.D), dtype=torch.float64, device=dev),
                                torch.empty((self.K, self.D, self.D), dtype=torch.float64, device=dev))
        for t in (out.rho, out.effects, out.gates):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError("out tensors must be contiguous float64 device tensors")
        _lib.check(self.ctx.lib.gst_param_forward(self.ctx.handle, self.mode, self.n_qubits, self.M, self.K,
                                                  _ptr(theta), _ptr(self.targets), _ptr(out.rho),
                                                  _ptr(out.effects), _ptr(out.gates)))
        return out

    def backward(self, theta: torch.Tensor, grad_full: torch.Tensor,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        theta = self._theta(theta)
        grad_full = _require_cuda(grad_full, torch.float64, "grad_full")
        if out is None:
            out = torch.empty(self.count, dtype=torch.float64, device=theta.device)
        _lib.check(self.ctx.lib.gst_param_backward(self.ctx.handle, self.mode, self.n_qubits, self.M, self.K,
                                                   _ptr(theta), _ptr(self.targets), _ptr(grad_full), _ptr(out)))
        return out


def _csr_words(words):
    import numpy as np
    off = np.zeros(len(words) + 1, np.int64)
    for i, w in enumerate(words):
        off[i + 1] = off[i] + len(w)
    flat = np.array([int(g) for w in words for g in w] or [0], np.uint8)
    return off, flat


def lgst(n_qubits: int, n_outcomes: int, n_gates: int, offsets, gates, counts, prep_fids, meas_fids):
    """Linear-inversion estimates (``gst_lgst``) from a host sequence list with
    counts and the fiducial words; returns numpy (rho [D], effects [M, D],
    gates [K, D, D]) in the gauge of the truncated singular vectors."""
    import numpy as np
    lib = _lib.load()
    D = 4 ** n_qubits
    off = np.ascontiguousarray(offsets, np.int64)
    g = np.ascontiguousarray(gates, np.uint8) if len(gates) else np.zeros(1, np.uint8)
    cnt = np.ascontiguousarray(counts, np.int32)
    po, pg = _csr_words(prep_fids)
    mo, mg = _csr_words(meas_fids)
    rho, E, G = np.zeros(D), np.zeros((n_outcomes, D)), np.zeros((n_gates, D, D))
    _lib.check(lib.gst_lgst(n_qubits, n_outcomes, n_gates, len(off) - 1, off.ctypes.data, g.ctypes.data,
                            cnt.ctypes.data, len(prep_fids), po.ctypes.data, pg.ctypes.data, len(meas_fids),
                            mo.ctypes.data, mg.ctypes.data, rho.ctypes.data, E.ctypes.data, G.ctypes.data))
    return rho, E, G


def gauge_optimize(n_qubits: int, rho, E, G, target_rho, target_E, target_G, spam_weight: float = 1.0,
                   gtol: float = 1e-12):
    """Gauge optimization toward the targets (``gst_gauge_optimize``) on copies of
    the host arrays; returns (rho, E, G, X, objective)."""
    import numpy as np
    lib = _lib.load()
    rho, E, G = (np.array(a, np.float64, copy=True, order="C") for a in (rho, E, G))
    tr, tE, tG = (np.ascontiguousarray(a, np.float64) for a in (target_rho, target_E, target_G))
    D = rho.shape[0]
    X = np.zeros((D, D))
    obj = ctypes.c_double(0.0)
    _lib.check(lib.gst_gauge_optimize(n_qubits, E.shape[0], G.shape[0], rho.ctypes.data, E.ctypes.data,
                                      G.ctypes.data, tr.ctypes.data, tE.ctypes.data, tG.ctypes.data,
                                      float(spam_weight), float(gtol), X.ctypes.data, ctypes.byref(obj)))
    return rho, E, G, X, obj.value


def mlgst(ctx: Context, stages, mode: str, theta0, targets: Optional[torch.Tensor] = None, max_iter: int = 500,
          gtol: float = 1e-9, memory: int = 10):
    """Iterative MLGST on the GPU (``gst_mlgst``): ``stages`` are ``Request``s of
    growing lists; returns (theta, [report dict per stage])."""
    import numpy as np
    th = np.array(theta0, np.float64, copy=True, order="C")
    arr = (ctypes.c_void_p * len(stages))(*[r.handle.value for r in stages])
    reps = (_lib.GstFitReport * len(stages))()
    opt = _lib.GstFitOptions(int(max_iter), float(gtol), int(memory))
    tg = None if targets is None else _require_cuda(targets, torch.float64, "targets")
    _lib.check(ctx.lib.gst_mlgst(ctx.handle, len(stages), arr, Parameterization.MODES[mode], _ptr(tg),
                                 th.ctypes.data, ctypes.byref(opt), reps))
    out = [dict(iterations=r.iterations, evaluations=r.evaluations, status=r.status, objective=r.objective,
                grad_max=r.grad_max, shrink=r.shrink) for r in reps]
    return th, out


def contract_tp(rho, E, G):
    """TP parameters of an estimate: the entries TP leaves free (rho[1:], the first
    M - 1 effects, rows 1.. of every gate), in the layout of ``gst_param_*``."""
    import numpy as np
    return np.concatenate([np.asarray(rho)[1:], np.asarray(E)[:-1].ravel(), np.asarray(G)[:, 1:, :].ravel()])


def avg_gate_fidelity(n_qubits: int, gates, targets):
    """Average gate fidelity of each transfer matrix against its unitary target's
    transfer matrix (``gst_avg_gate_fidelity``); numpy [K]."""
    import numpy as np
    lib = _lib.load()
    G = np.ascontiguousarray(gates, np.float64)
    T = np.ascontiguousarray(targets, np.float64)
    K = G.shape[0]
    out = np.zeros(K)
    _lib.check(lib.gst_avg_gate_fidelity(n_qubits, K, G.ctypes.data, T.ctypes.data, out.ctypes.data))
    return out


def diamond_unitary(U, V) -> float:
    """Diamond distance of the channels of two unitaries (``gst_diamond_unitary``)."""
    import numpy as np
    lib = _lib.load()
    u = np.ascontiguousarray(np.asarray(U, np.complex128)).view(np.float64)
    v = np.ascontiguousarray(np.asarray(V, np.complex128)).view(np.float64)
    out = ctypes.c_double(0.0)
    _lib.check(lib.gst_diamond_unitary(np.asarray(U).shape[0], u.ctypes.data, v.ctypes.data, ctypes.byref(out)))
    return out.value


def hamiltonian_decomposition(n_qubits: int, G):
    """(h [D], angle |h|, gamma) of a transfer matrix (``gst_hamiltonian_decomposition``)."""
    import numpy as np
    lib = _lib.load()
    g = np.ascontiguousarray(G, np.float64)
    h = np.zeros(4 ** n_qubits)
    ang, gam = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _lib.check(lib.gst_hamiltonian_decomposition(n_qubits, g.ctypes.data, h.ctypes.data, ctypes.byref(ang),
                                                 ctypes.byref(gam)))
    return h, ang.value, gam.value


def max_gates(n_qubits: int) -> int:
    """Largest gate count the library takes for ``n_qubits`` (``gst_max_gates``)."""
    return int(_lib.load().gst_max_gates(int(n_qubits)))


def hamiltonian_decomposition_target(n_qubits: int, G, U):
    """(h [D], angle |h|, gamma): h minimizing ||G - exp(L^H(h))||_F from the target
    unitary U's Hamiltonian (``gst_hamiltonian_decomposition_target``)."""
    import numpy as np
    lib = _lib.load()
    g = np.ascontiguousarray(G, np.float64)
    u = np.ascontiguousarray(np.asarray(U, np.complex128)).view(np.float64)
    h = np.zeros(4 ** n_qubits)
    ang, gam = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _lib.check(lib.gst_hamiltonian_decomposition_target(n_qubits, g.ctypes.data, u.ctypes.data, h.ctypes.data,
                                                        ctypes.byref(ang), ctypes.byref(gam)))
    return h, ang.value, gam.value


def set_plan_jump(ctx: Context, reps: int):
    """Germ-power jump repetitions of the sharing plans of requests created
    afterwards on ``ctx`` (``gst_set_plan_jump``; 0 = off, bit-identical
    probabilities)."""
    _lib.check(ctx.lib.gst_set_plan_jump(ctx.handle, int(reps)))


def profile_only(ctx: Context, family: Optional[str] = None):
    """Record kernel events for one family only (None = all)."""
    _lib.check(ctx.lib.gst_profile_only(ctx.handle, None if family is None else family.encode()))


def profile_enable(ctx: Context, on: bool = True):
    _lib.check(ctx.lib.gst_profile_enable(ctx.handle, 1 if on else 0))


def profile_read(ctx: Context, family: str):
    """(total_ms, launches) of one kernel family since profiling was enabled."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _lib.check(ctx.lib.gst_profile_read(ctx.handle, family.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def split_grad(g: torch.Tensor, n_qubits: int, M: int, K: int):
    """Gradient layout [rho (D) | E (M*D) | G (K*D*D)] -> (d_rho, d_E, d_G) views."""
    D = 4 ** n_qubits
    return g[:D], g[D:D + M * D].view(M, D), g[D + M * D:].view(K, D, D)
