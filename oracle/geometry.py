"""Lattice normalisation and grid offsets (paper Section 2.2, eq. (transvec)).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Given the user's primitive vectors (columns of ``avec``) and the grid
n1 x n2 x n3, the paper rotates the lattice so that a1 lies on the x axis and
a2 in the xy plane, then rounds the x offsets of a2, a3 and the y offset of a3
to whole grid cells (integers m1, m2, m3, with round-half-up) and corrects the
angles gamma, beta, alpha so that the rotated vectors end on grid points.

Readings (where the text is ambiguous):
  * The case bits rho1, rho2, rho3 are the indicators of the second case
    ("obtuse") used when computing m1, m2, m3.  Equivalently the signed grid
    offsets of the corrected vectors are s = m - rho * n.
  * The m3 case split uses ">= 0" for Case I (the text gives "0 <" and "< 0";
    rho3 = 0 for a value >= 0 in Section 3.1).
  * A rounding argument within 1e-9 of an integer is snapped to it before the
    floor/ceil, so that exact lattices are not perturbed by float noise.
  * Admissibility: the paper requires that the rotated vectors fall inside the
    new primitive cell, which is what makes 0 <= m1, m2 <= n1 and 0 <= m3 <= n2.
    We check exactly that (|a2_x|, |a3_x| <= l1 and |a3_y| < l2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SNAP = 1e-9


class LatticeError(ValueError):
    pass


def round_half_up(x: float) -> int:
    """Round as in the m1/m2/m3 definitions: floor when frac < 1/2, else ceil."""
    r = round(x)
    if abs(x - r) < SNAP:
        return int(r)
    f = math.floor(x)
    return int(f) if (x - f) < 0.5 else int(math.ceil(x))


@dataclass
class Geometry:
    n: tuple            # (n1, n2, n3)
    m: tuple            # (m1, m2, m3)
    rho: tuple          # (rho1, rho2, rho3) case indicators
    shift: tuple        # (s1, s2, s3) = signed grid offsets of a2_x, a3_x, a3_y
    delta: tuple        # (dx, dy, dz)
    avec_rot: np.ndarray  # 3x3, columns a1, a2, a3 after rotation + correction
    cos_angles: tuple   # corrected (cos gamma, cos beta, cos alpha)

    @property
    def npts(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


def lattice_geometry(avec, n1: int, n2: int, n3: int) -> Geometry:
    """Section 2.2: corrected, rotated lattice vectors and the integers m, rho."""
    avec = np.asarray(avec, dtype=np.float64)
    if avec.shape != (3, 3):
        raise LatticeError("avec must be 3x3 (columns are the lattice vectors)")
    if min(n1, n2, n3) < 1:
        raise LatticeError("grid sizes must be positive")
    a1, a2, a3 = avec[:, 0], avec[:, 1], avec[:, 2]
    L1, L2, L3 = (float(np.linalg.norm(v)) for v in (a1, a2, a3))
    if min(L1, L2, L3) <= 0:
        raise LatticeError("zero lattice vector")
    cg_p = float(a1 @ a2) / (L1 * L2)      # cos theta_gamma'
    cb_p = float(a1 @ a3) / (L1 * L3)      # cos theta_beta'
    ca_p = float(a2 @ a3) / (L2 * L3)      # cos theta_alpha'
    vol = float(np.linalg.det(avec))
    if abs(vol) < 1e-12 * L1 * L2 * L3:
        raise LatticeError("lattice vectors are linearly dependent")

    dx = L1 / n1
    # m1 and the corrected gamma (Case I: gamma' <= pi/2, Case II otherwise)
    if cg_p >= 0.0:
        rho1 = 0
        m1 = round_half_up(L2 * cg_p / dx)
        cg = m1 * dx / L2
    else:
        rho1 = 1
        m1 = round_half_up((L1 + L2 * cg_p) / dx)
        cg = (m1 * dx - L1) / L2
    if abs(cg) > 1.0:
        raise LatticeError("a2 does not fit in the primitive cell along x")
    sg = math.sqrt(1.0 - cg * cg)
    if sg <= 0.0:
        raise LatticeError("a2 is parallel to a1 after correction")
    l2 = L2 * sg
    dy = l2 / n2

    # m2 and the corrected beta
    if cb_p >= 0.0:
        rho2 = 0
        m2 = round_half_up(L3 * cb_p / dx)
        cb = m2 * dx / L3
    else:
        rho2 = 1
        m2 = round_half_up((L1 + L3 * cb_p) / dx)
        cb = (m2 * dx - L1) / L3
    if abs(cb) > 1.0:
        raise LatticeError("a3 does not fit in the primitive cell along x")

    # m3 and the corrected alpha (uses the corrected gamma and beta)
    d_p = ca_p - cg * cb
    if d_p >= 0.0:
        rho3 = 0
        m3 = round_half_up(L3 * d_p / (dy * sg))
        ca = m3 * dy * sg / L3 + cg * cb
    else:
        rho3 = 1
        m3 = round_half_up((L2 * sg * sg + L3 * d_p) / (dy * sg))
        ca = (m3 * dy * sg - L2 * sg * sg) / L3 + cg * cb

    if not (0 <= m1 <= n1 and 0 <= m2 <= n1 and 0 <= m3 <= n2):
        raise LatticeError(f"lattice violates the primitive-cell condition (m={m1},{m2},{m3})")

    disc = 1.0 - cg * cg - cb * cb - ca * ca + 2.0 * cg * cb * ca
    if disc <= 0.0:
        raise LatticeError("corrected lattice is degenerate")
    l3 = L3 * math.sqrt(disc) / sg
    dz = l3 / n3
    avec_rot = np.array([
        [L1, L2 * cg, L3 * cb],
        [0.0, L2 * sg, L3 * (ca - cg * cb) / sg],
        [0.0, 0.0, l3],
    ])
    s1 = m1 - rho1 * n1
    s2 = m2 - rho2 * n1
    s3 = m3 - rho3 * n2
    if abs(s3) >= n2:
        raise LatticeError("a3 does not fit in the primitive cell along y")
    return Geometry(n=(n1, n2, n3), m=(m1, m2, m3), rho=(rho1, rho2, rho3),
                    shift=(s1, s2, s3), delta=(dx, dy, dz), avec_rot=avec_rot,
                    cos_angles=(cg, cb, ca))


def kappa_from_bloch(avec, kvec) -> np.ndarray:
    """kappa_l = k . a_l where the Bloch wave vector is 2 pi k (Section 1.2).

    ``kvec`` is the Bloch vector 2 pi k in the user's Cartesian frame, so
    kappa_l = kvec . a~_l / (2 pi), evaluated with the user's vectors (the
    phases are unchanged by the rotation).
    """
    avec = np.asarray(avec, dtype=np.float64)
    kvec = np.asarray(kvec, dtype=np.float64)
    out = np.empty(3)
    for l in range(3):
        a = avec[:, l]
        out[l] = (a[0] * kvec[0] + a[1] * kvec[1] + a[2] * kvec[2]) / (2.0 * math.pi)
    return out


def omega_matrix(avec, geom: Geometry) -> np.ndarray:
    """Section 2.3: Omega = [a1 a2 a3]^{-T} [a~1 a~2 a~3]^T, written as the defining product
    (B B~^{-1} with B = 2 pi [a]^{-T}, B~ = 2 pi [a~]^{-T}), so that the reciprocal vectors of the
    corrected lattice are Omega times those of the user's lattice."""
    B_new = 2.0 * math.pi * np.linalg.inv(np.asarray(geom.avec_rot, dtype=np.float64)).T
    B_old = 2.0 * math.pi * np.linalg.inv(np.asarray(avec, dtype=np.float64)).T
    return B_new @ np.linalg.inv(B_old)


def lattice_rows_grid_units(geom: Geometry) -> np.ndarray:
    """The corrected lattice vectors in grid units, as rows:
    L1 = (n1, 0, 0), L2 = (s1, n2, 0), L3 = (s2, s3, n3)."""
    n1, n2, n3 = geom.n
    s1, s2, s3 = geom.shift
    return np.array([[n1, 0, 0], [s1, n2, 0], [s2, s3, n3]], dtype=np.int64)
