"""Derivative of a GEP eigenvalue with respect to the diagonal of B.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not in the paper: standard first-order perturbation of a simple eigenvalue of
the Hermitian-definite pencil (A, B).  With lambda = x^* A x / x^* B x and
dA = 0, d lambda / d B_pp = -lambda |x_p|^2 / (x^* B x).

With x = B^{-1} Q_r Sigma_r y (Theorem 5.2) one has x^* B x = lambda ||y||^2,
so the same quantity is -|x_p|^2 / ||y||^2.  A voxel permittivity that is
broadcast to the three Yee edges owned by grid point p receives the sum over
the three components.
"""
from __future__ import annotations

import numpy as np

from .solve import dense_gep


def dlambda_dB(lam: float, x: np.ndarray, eps_yee: np.ndarray) -> np.ndarray:
    """Per Yee point derivative, shape (3, n)."""
    b = np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    xBx = float(np.real(np.vdot(x, b * x)))
    g = -lam * np.abs(x) ** 2 / xBx
    return g.reshape(3, -1)


def fd_dlambda_dB(geom, kappa, eps_yee, band: int, comp: int, point: int, h: float):
    """Central finite difference of the band-th positive eigenvalue (dense solve)."""
    e = np.array(eps_yee, dtype=np.float64, copy=True).reshape(3, -1)
    e[comp, point] += h
    lp = dense_gep(geom, kappa, e, band + 1)[0][band]
    e[comp, point] -= 2 * h
    lm = dense_gep(geom, kappa, e, band + 1)[0][band]
    return (lp - lm) / (2 * h)
