"""Explicit sparse Yee discretisation of the curl (paper Section 3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

C_1, C_2, C_3 are the forward differences of Section 3.1 (the matrices K_1,
K_2 = [.. J_2 ..], K_3 = [.. J_3 ..]).  Instead of transcribing the sixteen J_3
cases we apply the quasi-periodic condition (eq. quasi_periodic) directly:
when the neighbour p + e_d leaves the box [0,n1) x [0,n2) x [0,n3), we subtract
lattice vectors (in grid units L1 = (n1,0,0), L2 = (s1,n2,0), L3 = (s2,s3,n3))
until it is back inside, multiplying by exp(+i 2 pi kappa_l) for every L_l
subtracted (and exp(-i 2 pi kappa_l) for every L_l added).  The paper's listed
J_2 / J_3 matrices are transcribed separately in ``paper_forms`` and compared
entry by entry in the tests.

Vector layout (Section 3, vec()): field component e_l has n = n1 n2 n3 entries
with the x index a fastest, then y index b, then z index c:
    index(a, b, c) = a + n1 * (b + n2 * c).
E_1 lives at (a+1/2, b, c), E_2 at (a, b+1/2, c), E_3 at (a, b, c+1/2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Geometry, lattice_rows_grid_units


def _wrap(q: np.ndarray, rows: np.ndarray, n, kappa):
    """Reduce integer grid points q (N x 3) into the box; return (q', phase)."""
    n1, n2, n3 = n
    q = q.copy()
    phase = np.ones(q.shape[0], dtype=np.complex128)
    # z first (only L3 has a z component), then y (L2), then x (L1)
    for axis, l in ((2, 2), (1, 1), (0, 0)):
        size = n[axis]
        t = np.floor_divide(q[:, axis], size)          # how many L_l to subtract
        q -= t[:, None] * rows[l][None, :]
        phase *= np.exp(2j * np.pi * kappa[l] * t)
    assert np.all((q >= 0) & (q < np.array([n1, n2, n3])))
    return q, phase


def derivative_matrices(geom: Geometry, kappa):
    """Sparse C_1, C_2, C_3 (each n x n, complex128): (C_d f)(p) = (f(p+e_d) - f(p)) / delta_d."""
    n1, n2, n3 = geom.n
    n = n1 * n2 * n3
    kappa = np.asarray(kappa, dtype=np.float64)
    rows = lattice_rows_grid_units(geom)
    c, b, a = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    p = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1).astype(np.int64)
    pidx = p[:, 0] + n1 * (p[:, 1] + n2 * p[:, 2])
    mats = []
    for d in range(3):
        q = p.copy()
        q[:, d] += 1
        q, ph = _wrap(q, rows, geom.n, kappa)
        qidx = q[:, 0] + n1 * (q[:, 1] + n2 * q[:, 2])
        inv = 1.0 / geom.delta[d]
        data = np.concatenate([np.full(n, -inv, dtype=np.complex128), ph * inv])
        ri = np.concatenate([pidx, pidx])
        ci = np.concatenate([pidx, qidx])
        mats.append(sp.csr_matrix((data, (ri, ci)), shape=(n, n)))
    return mats


def curl_matrix(geom: Geometry, kappa):
    """C = [[0, -C3, C2], [C3, 0, -C1], [-C2, C1, 0]] (Section 3, 3n x 3n)."""
    C1, C2, C3 = derivative_matrices(geom, kappa)
    return sp.bmat([[None, -C3, C2], [C3, None, -C1], [-C2, C1, None]], format="csr")


def gradient_matrix(geom: Geometry, kappa):
    """G = [C1; C2; C3] (3n x n): the discrete gradient.  C G = 0 since the C_d commute."""
    C1, C2, C3 = derivative_matrices(geom, kappa)
    return sp.vstack([C1, C2, C3], format="csr")


def double_curl(geom: Geometry, kappa):
    """A = C* C (Section 3, the discrete curl-curl)."""
    C = curl_matrix(geom, kappa)
    return (C.conj().T @ C).tocsr()


def mass_matrix(eps_yee):
    """B = diag(eps_1, eps_2, eps_3) sampled at the Yee points (Section 3).

    ``eps_yee`` has shape (3, n) in the e-layout (index a + n1 (b + n2 c))."""
    eps_yee = np.asarray(eps_yee, dtype=np.float64)
    return sp.diags(eps_yee.reshape(-1).astype(np.complex128), format="csr")
