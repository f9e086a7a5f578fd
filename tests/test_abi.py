"""CPU checks of the C ABI: the library loads and exports every function include/gst.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gst.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gst_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = declared_functions()
    for f in ["gst_create", "gst_destroy", "gst_probs", "gst_loglik", "gst_vjp", "gst_sync",
              "gst_req_create_host", "gst_req_create", "gst_req_eval", "gst_req_footprint", "gst_req_destroy", "gst_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2008_13490_amd", "libgst.so")
    if not os.path.exists(lib_path):
        pytest.skip("libgst.so not built")
    lib = ctypes.CDLL(lib_path)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing
    lib.gst_max_gates.restype = ctypes.c_int
    # the documented gate-count caps (larger K is refused with GST_EINVAL)
    assert [lib.gst_max_gates(n) for n in (0, 1, 2, 3, 4, 7)] == [0, 8, 8, 5, 0, 0]
    lib.gst_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.gst_last_error(), bytes)


def test_python_binding_lists_exports():
    from paper_2008_13490_amd import _lib
    assert set(declared_functions()) <= set(_lib.EXPORTED)
