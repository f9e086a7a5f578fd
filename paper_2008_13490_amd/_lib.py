"""ctypes binding of ``libgst.so`` (argument marshalling only).

Every number is computed by the HIP library; this module converts torch
tensors on the GPU into the plain device pointers and sizes of the C ABI
(``include/gst.h``) and raises on error codes.  PyTorch provides device memory
and the stream.  There is no fallback: if the library is missing, importing
the functions raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgst.so")

GST_OK, GST_EINVAL, GST_EINDEX, GST_ENONPOS, GST_ENOMEM, GST_EDEVICE, GST_EBUSY = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "GST_OK", -1: "GST_EINVAL", -2: "GST_EINDEX", -3: "GST_ENONPOS", -4: "GST_ENOMEM",
          -5: "GST_EDEVICE", -6: "GST_EBUSY"}

EXPORTED = [
    "gst_max_gates", "gst_create", "gst_destroy", "gst_sync", "gst_probs", "gst_loglik", "gst_vjp",
    "gst_loglik_noalloc",
    "gst_req_create_host", "gst_req_create", "gst_req_footprint", "gst_req_eval", "gst_req_probs", "gst_req_vjp",
    "gst_req_destroy", "gst_req_plan_info", "gst_batch_create", "gst_batch_run", "gst_batch_nonpos",
    "gst_batch_destroy", "gst_tune_set", "gst_set_plan_jump", "gst_predict", "gst_tv_distance",
    "gst_param_count", "gst_param_forward", "gst_param_backward", "gst_lgst", "gst_gauge_optimize", "gst_mlgst",
    "gst_avg_gate_fidelity", "gst_diamond_unitary", "gst_hamiltonian_decomposition",
    "gst_hamiltonian_decomposition_target",
    "gst_profile_enable", "gst_profile_only",
    "gst_profile_read", "gst_last_error",
]


class GSTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class GstGateset(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int), ("n_gates", ctypes.c_int), ("n_outcomes", ctypes.c_int),
                ("rho", ctypes.c_void_p), ("effects", ctypes.c_void_p), ("gates", ctypes.c_void_p)]


class GstSeqlist(ctypes.Structure):
    _fields_ = [("n_seq", ctypes.c_int64), ("offsets", ctypes.c_void_p), ("gate_idx", ctypes.c_void_p),
                ("max_len", ctypes.c_int64)]


class GstDiag(ctypes.Structure):
    _fields_ = [("n_bad_index", ctypes.c_int64), ("n_nonpos", ctypes.c_int64)]


class GstFitOptions(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("gtol", ctypes.c_double), ("memory", ctypes.c_int)]


class GstFitReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("evaluations", ctypes.c_int), ("status", ctypes.c_int),
                ("objective", ctypes.c_double), ("grad_max", ctypes.c_double), ("shrink", ctypes.c_double)]


_lib = None
_lock = threading.Lock()


def load():
    """Load ``libgst.so``; torch is imported first so that the library binds to the
    same HIP runtime as torch."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (one HIP runtime per process)
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2008_13490_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        lib.gst_max_gates.argtypes = [I]
        lib.gst_create.argtypes = [ctypes.POINTER(P), I, P]
        lib.gst_destroy.argtypes = [P]
        lib.gst_sync.argtypes = [P, ctypes.POINTER(GstDiag)]
        lib.gst_probs.argtypes = [P, ctypes.POINTER(GstGateset), ctypes.POINTER(GstSeqlist), P]
        lib.gst_loglik.argtypes = [P, ctypes.POINTER(GstGateset), ctypes.POINTER(GstSeqlist), P, P, P, P]
        if hasattr(lib, "gst_loglik_noalloc"):
            lib.gst_loglik_noalloc.argtypes = [P, ctypes.POINTER(GstGateset), ctypes.POINTER(GstSeqlist), P, P, P, P]
            lib.gst_loglik_noalloc.restype = I
        lib.gst_vjp.argtypes = [P, ctypes.POINTER(GstGateset), ctypes.POINTER(GstSeqlist), P, P]
        lib.gst_last_error.argtypes = []
        lib.gst_last_error.restype = ctypes.c_char_p
        for name in ("gst_max_gates", "gst_create", "gst_destroy", "gst_sync", "gst_probs", "gst_loglik", "gst_vjp"):
            getattr(lib, name).restype = I
        lib.gst_profile_enable.argtypes = [P, I]
        lib.gst_profile_read.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]
        lib.gst_profile_enable.restype = I
        lib.gst_profile_only.argtypes = [P, ctypes.c_char_p]
        lib.gst_profile_only.restype = I
        lib.gst_tune_set.argtypes = [P, I, I, I]
        lib.gst_tune_set.restype = I
        lib.gst_set_plan_jump.argtypes = [P, I]
        lib.gst_set_plan_jump.restype = I
        lib.gst_predict.argtypes = [P, ctypes.POINTER(GstGateset), I, P, P, I, P, I, P]
        lib.gst_predict.restype = I
        lib.gst_tv_distance.argtypes = [P, P, P, I64, I, P]
        lib.gst_tv_distance.restype = I
        lib.gst_param_count.argtypes = [I, I, I, I, ctypes.POINTER(I64)]
        lib.gst_param_forward.argtypes = [P, I, I, I, I, P, P, P, P, P]
        lib.gst_param_backward.argtypes = [P, I, I, I, I, P, P, P, P]
        for name in ("gst_param_count", "gst_param_forward", "gst_param_backward"):
            getattr(lib, name).restype = I
        lib.gst_lgst.argtypes = [I, I, I, I64, P, P, P, I, P, P, I, P, P, P, P, P]
        lib.gst_gauge_optimize.argtypes = [I, I, I, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double, P, P]
        lib.gst_mlgst.argtypes = [P, I, P, I, P, P, ctypes.POINTER(GstFitOptions), P]
        for name in ("gst_lgst", "gst_gauge_optimize", "gst_mlgst"):
            getattr(lib, name).restype = I
        lib.gst_avg_gate_fidelity.argtypes = [I, I, P, P, P]
        lib.gst_diamond_unitary.argtypes = [I, P, P, P]
        lib.gst_hamiltonian_decomposition.argtypes = [I, P, P, P, P]
        lib.gst_hamiltonian_decomposition_target.argtypes = [I, P, P, P, P, P]
        for name in ("gst_avg_gate_fidelity", "gst_diamond_unitary", "gst_hamiltonian_decomposition",
                     "gst_hamiltonian_decomposition_target"):
            getattr(lib, name).restype = I
        lib.gst_profile_read.restype = I
        if hasattr(lib, "gst_req_create_host"):
            lib.gst_req_create_host.argtypes = [P, I, I, I, ctypes.POINTER(GstSeqlist), P, ctypes.POINTER(P)]
            lib.gst_req_create.argtypes = [P, I, I, I, ctypes.POINTER(GstSeqlist), P, ctypes.POINTER(P)]
            lib.gst_req_create.restype = I
            lib.gst_req_footprint.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
            lib.gst_req_eval.argtypes = [P, ctypes.POINTER(GstGateset), P, P, P]
            lib.gst_req_vjp.argtypes = [P, ctypes.POINTER(GstGateset), P, P]
            lib.gst_req_probs.argtypes = [P, ctypes.POINTER(GstGateset), P]
            lib.gst_req_probs.restype = I
            lib.gst_req_destroy.argtypes = [P]
            lib.gst_req_plan_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), I]
            lib.gst_req_plan_info.restype = I
            for name in ("gst_req_create_host", "gst_req_footprint", "gst_req_eval", "gst_req_vjp", "gst_req_destroy"):
                getattr(lib, name).restype = I
        if hasattr(lib, "gst_batch_create"):
            PP = ctypes.POINTER(ctypes.c_void_p)
            lib.gst_batch_create.argtypes = [P, I, PP, ctypes.POINTER(GstGateset), PP, PP, PP, I, ctypes.POINTER(P)]
            lib.gst_batch_run.argtypes = [P]
            lib.gst_batch_nonpos.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
            lib.gst_batch_destroy.argtypes = [P]
            for name in ("gst_batch_create", "gst_batch_run", "gst_batch_nonpos", "gst_batch_destroy"):
                getattr(lib, name).restype = I
        _lib = lib
        return lib


def check(rc: int):
    if rc != GST_OK:
        msg = _lib.gst_last_error().decode() if _lib is not None else ""
        raise GSTError(rc, msg)
    return rc
