"""Host dense linear algebra used by the Rayleigh-Ritz step (paper_1806_10284_amd/csrc/pcx_dense.cpp),
compiled here with g++ and checked against numpy.linalg.eigh."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1806_10284_amd", "csrc", "pcx_dense.cpp")


@pytest.fixture(scope="module")
def dense(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("dense") / "libpcx_dense.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-fPIC", "-shared", SRC, "-o", out], check=True)
    lib = ctypes.CDLL(out)
    lib.pcxd_herm_eig.restype = ctypes.c_int
    lib.pcxd_herm_eig.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def _eig(lib, A):
    k = A.shape[0]
    a = np.ascontiguousarray(A.astype(np.complex128))
    w = np.zeros(k)
    v = np.zeros((k, k), dtype=np.complex128)
    assert lib.pcxd_herm_eig(k, a.ctypes.data, w.ctypes.data, v.ctypes.data) == 0
    return w, v


@pytest.mark.parametrize("k", [1, 2, 3, 5, 16, 45, 96])
def test_herm_eig_random(dense, k):
    rng = np.random.default_rng(k)
    M = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    A = M + M.conj().T
    w, V = _eig(dense, A)
    wr = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(w, wr, atol=1e-12 * np.abs(wr).max())
    assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-12
    assert np.abs(A @ V - V * w[None, :]).max() < 1e-11 * np.abs(wr).max()


def test_herm_eig_degenerate_and_graded(dense):
    # repeated eigenvalues and a wide dynamic range, as in a Rayleigh-Ritz pencil near convergence
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20)))
    lam = np.array([2.08, 2.08, 11.5, 11.5, 11.96] + list(np.geomspace(15, 3e4, 15)))
    A = (Q * lam) @ Q.conj().T
    w, V = _eig(dense, A)
    np.testing.assert_allclose(w, np.sort(lam), rtol=1e-12, atol=1e-10)
    assert np.abs(A @ V - V * w[None, :]).max() < 1e-9
