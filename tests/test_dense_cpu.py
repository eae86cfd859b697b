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
    lib.pcxd_herm_eig_cols.restype = ctypes.c_int
    lib.pcxd_herm_eig_cols.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.pcxd_rayleigh_ritz.restype = ctypes.c_int
    lib.pcxd_rayleigh_ritz.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p]
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


@pytest.mark.parametrize("k,ncols", [(36, 12), (45, 1), (24, 0), (7, 7)])
def test_herm_eig_lowest_columns(dense, k, ncols):
    """Only the eigenvectors of the ncols lowest eigenvalues: equal to the leading columns of the
    full decomposition up to a phase, and eigenvectors of A."""
    rng = np.random.default_rng(100 + k)
    M = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
    A = np.ascontiguousarray(M + M.conj().T)
    w = np.zeros(k)
    v = np.zeros((k, max(ncols, 1)), dtype=np.complex128)
    assert dense.pcxd_herm_eig_cols(k, A.ctypes.data, ncols, w.ctypes.data, v.ctypes.data) == 0
    wr, Vr = np.linalg.eigh(A)
    np.testing.assert_allclose(w, wr, atol=1e-12 * np.abs(wr).max())
    if ncols == 0:
        return
    V = v[:, :ncols]
    assert np.abs(V.conj().T @ V - np.eye(ncols)).max() < 1e-12
    assert np.abs(A @ V - V * wr[None, :ncols]).max() < 1e-11 * np.abs(wr).max()
    # simple eigenvalues (random matrix): the columns agree with eigh's up to a unit phase
    ov = np.abs(np.einsum("ij,ij->j", Vr[:, :ncols].conj(), V))
    np.testing.assert_allclose(ov, 1.0, atol=1e-10)


@pytest.mark.parametrize("k,want", [(36, 12), (24, 8), (6, 2)])
def test_rayleigh_ritz_pencil(dense, k, want):
    """Lowest pairs of (GA, GB) with GB = S^H S, GA = S^H D S (as in the Rayleigh-Ritz step):
    theta against scipy's generalized eigh, C^H GB C = I and GA C = GB C diag(theta)."""
    scipy_linalg = pytest.importorskip("scipy.linalg")
    rng = np.random.default_rng(7 * k + want)
    n = 4 * k
    S = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    S[:, 1] *= 1e3          # badly scaled columns: the routine scales to unit norm first
    D = 1.0 + 10 * np.abs(rng.standard_normal(n))
    GB = np.ascontiguousarray(S.conj().T @ S)
    GA = np.ascontiguousarray(S.conj().T @ (D[:, None] * S))
    theta = np.zeros(want)
    c = np.zeros((k, want), dtype=np.complex128)
    assert dense.pcxd_rayleigh_ritz(k, GA.ctypes.data, GB.ctypes.data, want, theta.ctypes.data, c.ctypes.data) == 0
    ref = scipy_linalg.eigh(GA, GB, eigvals_only=True)[:want]
    np.testing.assert_allclose(theta, ref, rtol=1e-11)
    assert np.abs(c.conj().T @ GB @ c - np.eye(want)).max() < 1e-10
    r = GA @ c - (GB @ c) * theta[None, :]
    assert np.abs(r).max() < 1e-9 * np.abs(GA @ c).max()
