"""The CPTP generator's structure tables of the library (host C++, built here
with g++) against the oracle's transfer matrices of the Hamiltonian and
dissipator maps, which the oracle builds from explicit Pauli matrices: the
tables' entries, and the sparsity they rely on (P_k P_b is a multiple of P_a
only for k = a^b)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from oracle import params as PR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_13490_amd", "csrc")


@pytest.fixture(scope="module")
def tablib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tab") / "libtabprobe.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(ROOT, "tests", "param_probe.cpp"), os.path.join(CSRC, "gst_param_tables.cpp"),
                    "-o", out], check=True)
    lib = ctypes.CDLL(out)
    lib.probe_param_tables.argtypes = [ctypes.c_int] + [ctypes.c_void_p] * 3
    return lib


@pytest.mark.parametrize("n", [1, 2])
def test_tables_match_oracle_bases(tablib, n):
    D = 4 ** n
    y = np.zeros((D, D))
    zr = np.zeros((D, D, D))
    zi = np.zeros((D, D, D))
    tablib.probe_param_tables(n, y.ctypes.data, zr.ctypes.data, zi.ctypes.data)
    ham, Z = PR._generator_bases(n)   # ham[k-1][a][b], Z[j-1][k-1][a][b]
    for a in range(D):
        for b in range(D):
            for k in range(1, D):
                want = y[a, b] if k == (a ^ b) else 0.0
                assert ham[k - 1, a, b] == want, (a, b, k)
            for j in range(1, D):
                for k in range(1, D):
                    want = zr[j, a, b] + 1j * zi[j, a, b] if k == (a ^ b ^ j) else 0.0
                    assert abs(Z[j - 1, k - 1, a, b] - want) <= 1e-15, (a, b, j, k)
    # every entry is a small multiple of 1/2
    assert np.all(2 * y == np.round(2 * y)) and np.all(2 * zr == np.round(2 * zr))
