"""The paper's printed matrices and spectra, transcribed as written (used as pins).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* ``k1_matrix``, ``k2_matrix``, ``k3_matrix``: K_1 (eq. K1), K_2 (eq. K2 with
  the general J_2 of eq. J2) and K_3 (eq. K3 with the four general categories
  of J_3, eqs. acuteJ3 / obtuseJ3, built from J_1 of eq. J1, rho_4, rho_5,
  psi_1 and psi_2 of Section 3.1).
* ``paper_thetas``: the eigenvalue exponents of Theorems 4.1, 4.2, 4.3
  (cos alpha - cos beta cos gamma >= 0) and 4.4 (< 0), as fractions of a turn.

These are independent of ``curl`` (which applies the quasi-periodic condition
directly) and of ``spectral`` (which indexes the Fourier basis by the lattice
in grid units); the tests check that all three agree.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry


def _e(x):
    return np.exp(2j * np.pi * x)


def _antidiag(top_right: np.ndarray, bottom_left: np.ndarray) -> np.ndarray:
    """[[0, X], [Y, 0]] with X (p x p) in the top-right and Y (q x q) bottom-left."""
    p = top_right.shape[0]
    q = bottom_left.shape[0]
    out = np.zeros((p + q, p + q), dtype=np.complex128)
    out[:p, q:] = top_right
    out[p:, :q] = bottom_left
    return out


def _shift_block(k1: float, top: int, size: int) -> np.ndarray:
    """[[0, e^{-i 2pi k1} I_top], [I_{size-top}, 0]] (size x size)."""
    return _antidiag(_e(-k1) * np.eye(top), np.eye(size - top))


def j2_matrix(geom: Geometry, kappa) -> np.ndarray:
    """eq. (J2): J_2 = e^{i 2pi rho1 k.a1} [[0, e^{-i 2pi k.a1} I_m1], [I_{n1-m1}, 0]]."""
    n1 = geom.n[0]
    m1 = geom.m[0]
    rho1 = geom.rho[0]
    return _e(rho1 * kappa[0]) * _shift_block(kappa[0], m1, n1)


def j1_matrix(geom: Geometry, kappa) -> np.ndarray:
    """eq. (J1): J_1 = e^{i 2pi rho2 k.a1} [[0, e^{-i 2pi k.a1} I_m2], [I_{n1-m2}, 0]]."""
    n1 = geom.n[0]
    m2 = geom.m[1]
    rho2 = geom.rho[1]
    return _e(rho2 * kappa[0]) * _shift_block(kappa[0], m2, n1)


def case_bits(geom: Geometry):
    """rho_4, rho_5, psi_1, psi_2 of Section 3.1 (from the corrected angles)."""
    n1 = geom.n[0]
    m1, m2, _ = geom.m
    rho1, rho2, rho3 = geom.rho
    cg, cb, ca = geom.cos_angles
    rho4 = int(math.ceil(cg * cb * (cg * cb - ca)))
    rho5 = int(math.ceil(cb))
    psi1 = 1 if (rho3 == 0 and (rho2 * n1 - m2) - (rho1 * n1 - m1) > 0) else 0
    psi2 = 1 if (rho3 == 1 and (rho1 * n1 - m1) + (rho2 * n1 - m2) > 0) else 0
    return rho4, rho5, psi1, psi2


def j3_matrix(geom: Geometry, kappa) -> np.ndarray:
    """J_3 by the four general categories (1)-(4) of Section 3.1.

    Reading: the text assigns m1 + m2 = n1 (with cos alpha - cos gamma cos beta < 0)
    to category (3); the quasi-periodic condition gives the matrix of category (4)
    there (the two differ by the phase exp(-i 2 pi k.a1)), so the boundary case
    is taken with (4).
    """
    n1, n2, _ = geom.n
    m1, m2, m3 = geom.m
    rho1, rho2, rho3 = geom.rho
    k1, k2 = kappa[0], kappa[1]
    rho4, rho5, psi1, psi2 = case_bits(geom)
    J1 = j1_matrix(geom, kappa)
    if rho3 == 0:
        if m1 <= m2:
            inner = _shift_block(k1, m2 - m1, n1)
            ph = _e(-(k2 + rho1 * rho4 * k1 - psi1 * k1))
        else:
            inner = _shift_block(k1, n1 - m1 + m2, n1)
            ph = _e(-(k2 - rho2 * rho4 * k1 - psi1 * k1))
        top = ph * np.kron(np.eye(m3), inner)
        bot = np.kron(np.eye(n2 - m3), J1)
    else:
        top = _e(-k2) * np.kron(np.eye(m3), J1)
        if m1 + m2 < n1:
            inner = _shift_block(k1, m1 + m2, n1)
            ph = _e((rho1 * rho4 + psi2) * k1)
        else:
            inner = _shift_block(k1, m1 + m2 - n1, n1)
            ph = _e(-(rho5 * rho4 - psi2) * k1)
        bot = ph * np.kron(np.eye(n2 - m3), inner)
    return _e(rho3 * k2) * _antidiag(top, bot)


def _bidiag_blocks(nb: int, bs: int, wrap: np.ndarray, h: float) -> np.ndarray:
    """(1/h) [[-I, I], [-I, I], ..., [wrap, ..., -I]] with nb blocks of size bs."""
    N = nb * bs
    M = np.zeros((N, N), dtype=np.complex128)
    eye = np.eye(bs)
    for b in range(nb):
        M[b * bs:(b + 1) * bs, b * bs:(b + 1) * bs] = -eye
        if b + 1 < nb:
            M[b * bs:(b + 1) * bs, (b + 1) * bs:(b + 2) * bs] += eye
        else:
            M[b * bs:(b + 1) * bs, 0:bs] += wrap
    return M / h


def k1_matrix(geom: Geometry, kappa) -> np.ndarray:
    """eq. (K1)."""
    return _bidiag_blocks(geom.n[0], 1, np.array([[_e(kappa[0])]]), geom.delta[0])


def k2_matrix(geom: Geometry, kappa) -> np.ndarray:
    """eq. (K2) with J_2 of eq. (J2)."""
    n1, n2, _ = geom.n
    return _bidiag_blocks(n2, n1, _e(kappa[1]) * j2_matrix(geom, kappa), geom.delta[1])


def k3_matrix(geom: Geometry, kappa) -> np.ndarray:
    """eq. (K3) with J_3 by the general categories."""
    n1, n2, n3 = geom.n
    return _bidiag_blocks(n3, n1 * n2, _e(kappa[2]) * j3_matrix(geom, kappa), geom.delta[2])


def paper_derivatives(geom: Geometry, kappa):
    """C_1 = I (x) I (x) K_1, C_2 = I (x) K_2, C_3 = K_3 (Section 3.1), dense."""
    n1, n2, n3 = geom.n
    C1 = np.kron(np.eye(n2 * n3), k1_matrix(geom, kappa))
    C2 = np.kron(np.eye(n3), k2_matrix(geom, kappa))
    C3 = k3_matrix(geom, kappa)
    return C1, C2, C3


def paper_thetas(geom: Geometry, kappa):
    """Eigenvalue exponents of Theorems 4.1-4.4, in turns (theta / (i 2 pi)).

    Returns (tx[i], ty[i, j], tz[i, j, k]) for i, j, k = 0..n-1 such that the
    eigenvalues of K_1, K_2, K_3 are (exp(i 2 pi t) - 1) / delta.

    Reading: Theorem 4.3 applies when cos alpha - cos beta cos gamma >= 0
    (rho3 = 0) and Theorem 4.4 when it is < 0 (rho3 = 1); the restatement in
    Section 4.2 swaps these labels and is not used.
    """
    n1, n2, n3 = geom.n
    m1, m2, m3 = geom.m
    rho1, rho2, rho3 = geom.rho
    k1, k2, k3 = kappa
    i = np.arange(n1)[:, None, None].astype(np.float64)
    j = np.arange(n2)[None, :, None].astype(np.float64)
    k = np.arange(n3)[None, None, :].astype(np.float64)
    # Theorem 4.1
    tx = (i + k1) / n1
    # Theorem 4.2: k.a2^ with a2^ = a2 - (m1/n1) a1 + rho1 a1
    ka2h = k2 - (m1 / n1) * k1 + rho1 * k1
    ty = (j - (m1 / n1) * i + ka2h) / n2
    if rho3 == 0:
        # Theorem 4.3
        ka3h = (k3 - (m3 / n2) * k2 - ((n2 - m3) / n2) * (m1 / n1) * k1
                + ((m1 - m2) / n1) * k1 + rho3 * k2 - (m3 / n2) * rho1 * k1 + rho2 * k1)
        tz = (k - (m3 / n2) * j - ((n2 - m3) / n2) * (m1 / n1) * i
              + ((m1 - m2) / n1) * i + ka3h) / n3
    else:
        # Theorem 4.4
        ka3h = (k3 - (m3 / n2) * k2 - ((n2 - m3) / n2) * (m1 / n1) * k1
                - (m2 / n1) * k1 + rho3 * k2 - (m3 / n2) * rho1 * k1 + rho1 * k1 + rho2 * k1)
        tz = (k - (m3 / n2) * j - ((n2 - m3) / n2) * (m1 / n1) * i
              - (m2 / n1) * i + ka3h) / n3
    shape = (n1, n2, n3)
    return (np.broadcast_to(tx, shape).copy(), np.broadcast_to(ty, shape).copy(),
            np.broadcast_to(tz, shape).copy())
