"""Singular value decomposition of C and the nullspace-free operator A_r
(paper Section 5.1, Theorem 5.1; Section 5.2, Theorem 5.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Per Fourier mode nu the curl acts as the cross product with
Lambda = (Lambda_1, Lambda_2, Lambda_3), so Q_r Sigma_r = (I_3 (x) T) W with a
3 x 2 matrix W(nu) = [Pi_1 Lambda_q^{1/2}, Pi_2 Lambda_q^{1/2}] (eqs.
range_basis1, range_basis2):
    W[:, 0] = (Lambda_q 1 - Lambda conj(Lambda_s)) / Lambda_p
    W[:, 1] = Lambda_q^{1/2} (1 x conj(Lambda)) / Lambda_p
with Lambda_q = sum |Lambda_d|^2, Lambda_s = sum Lambda_d and
Lambda_p^2 = 3 Lambda_q - |Lambda_s|^2 = sum_{a<b} |Lambda_a - Lambda_b|^2.

Readings:
  * Lambda_p is printed as (Lambda_1+Lambda_2+Lambda_3)(...)^*, which would
    not normalise Pi_1, Pi_2; the value that does is the one above.
  * When Lambda is (nearly) parallel to the all-ones vector the paper's
    construction degenerates (Lambda_p -> 0).  For Lambda_p^2 < TAU Lambda_q we
    replace the all-ones vector by the unit vector e_m, m = the first index with
    |Lambda_m|^2 <= (1 + 1e-8) min_l |Lambda_l|^2 (ties within rounding go to the
    lowest index); this is another orthonormal basis of the same
    2-dimensional range space, so A_r's eigenvalues are unchanged.
  * A mode with Lambda_q = 0 (only at kappa in Z^3, one mode) has no range
    space: W = 0 there (the Gamma-point mask; A_r then has the two extra zero
    eigenvalues, which the eigensolver excludes).

A_r y = Sigma_r Q_r^* B^{-1} Q_r Sigma_r y = W^H (I_3 (x) T^*) B^{-1} (I_3 (x) T) W y
(eq. NFSEP).  The 2n-vector y is stored as [y_1; y_2], each block in the
Fourier layout (i slowest, k fastest).
"""
from __future__ import annotations

import numpy as np

from .spectral import Spectrum, T_apply, Tstar_apply

TAU = 1e-3


def mixing(lam: np.ndarray) -> np.ndarray:
    """W per mode: lam (3, ...) -> W (3, 2, ...) complex."""
    L1, L2, L3 = lam[0], lam[1], lam[2]
    Lq = (np.abs(L1) ** 2 + np.abs(L2) ** 2 + np.abs(L3) ** 2)
    Lp2 = np.abs(L1 - L2) ** 2 + np.abs(L1 - L3) ** 2 + np.abs(L2 - L3) ** 2
    Ls = L1 + L2 + L3
    W = np.zeros((3, 2) + lam.shape[1:], dtype=np.complex128)
    masked = Lq == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        good = (~masked) & (Lp2 >= TAU * Lq)
        Lp = np.sqrt(Lp2)
        sq = np.sqrt(Lq)
        # paper basis (reference vector = all ones)
        for l in range(3):
            col1 = (Lq - lam[l] * np.conj(Ls)) / Lp
            W[l, 0] = np.where(good, col1, 0.0)
        cr = np.conj(lam)
        cross = np.stack([cr[2] - cr[1], cr[0] - cr[2], cr[1] - cr[0]])   # 1 x conj(Lambda)
        for l in range(3):
            W[l, 1] = np.where(good, sq * cross[l] / Lp, 0.0)
        # fallback basis (reference vector = e_m)
        bad = (~masked) & (~good)
        if np.any(bad):
            a2 = np.abs(lam) ** 2
            mn = a2.min(axis=0)
            m = np.argmax(a2 <= mn * (1.0 + 1e-8), axis=0)
            for mm in range(3):
                sel = bad & (m == mm)
                if not np.any(sel):
                    continue
                lm = lam[mm]
                den = np.sqrt(Lq - a2[mm])
                e = np.zeros(3)
                e[mm] = 1.0
                for l in range(3):
                    col1 = (Lq * e[l] - lam[l] * np.conj(lm)) / den
                    W[l, 0] = np.where(sel, col1, W[l, 0])
                # e_m x conj(Lambda)
                ex = [e[1] * cr[2] - e[2] * cr[1], e[2] * cr[0] - e[0] * cr[2], e[0] * cr[1] - e[1] * cr[0]]
                for l in range(3):
                    W[l, 1] = np.where(sel, sq * ex[l] / den, W[l, 1])
    return W


def split_y(spec: Spectrum, y: np.ndarray):
    n1, n2, n3 = spec.n
    y = np.asarray(y).reshape(2, n1, n2, n3)
    return y[0], y[1]


def QS_apply(spec: Spectrum, y: np.ndarray) -> np.ndarray:
    """u = Q_r Sigma_r y = (I_3 (x) T)(W y): 2n -> 3n (e-layout per component)."""
    W = mixing(spec.lam)
    y1, y2 = split_y(spec, y)
    out = []
    for l in range(3):
        ul = W[l, 0] * y1 + W[l, 1] * y2
        out.append(T_apply(spec, ul))
    return np.concatenate(out)


def QS_adjoint(spec: Spectrum, u: np.ndarray) -> np.ndarray:
    """z = Sigma_r Q_r^* u = W^H (I_3 (x) T^*) u: 3n -> 2n."""
    n = spec.npts
    W = mixing(spec.lam)
    v = [Tstar_apply(spec, u[l * n:(l + 1) * n]) for l in range(3)]
    z1 = sum(np.conj(W[l, 0]) * v[l] for l in range(3))
    z2 = sum(np.conj(W[l, 1]) * v[l] for l in range(3))
    return np.concatenate([z1.reshape(-1), z2.reshape(-1)])


def hfield_mixing(lam: np.ndarray) -> np.ndarray:
    """V per mode (3, 2, ...): the columns Lambda x W[:, c] / Lambda_q.

    The curl acts per mode as the cross product with Lambda, so C Q_r Sigma_r = (I_3 (x) T)(Lambda x W)
    and, from C = P_r Sigma_r Q_r^* (Theorem 5.1), P_r = C Q_r Sigma_r^{-1} = (I_3 (x) T) V with
    V = (Lambda x W) / Lambda_q: the left singular vectors that belong to this package's Q_r (the
    paper's P_r = [P_2, P_1] for its own basis).  Zero on the masked mode."""
    W = mixing(lam)
    Lq = np.sum(np.abs(lam) ** 2, axis=0)
    inv = np.where(Lq > 0, 1.0 / np.where(Lq > 0, Lq, 1.0), 0.0)
    V = np.zeros_like(W)
    for c in range(2):
        w = W[:, c]
        V[0, c] = (lam[1] * w[2] - lam[2] * w[1]) * inv
        V[1, c] = (lam[2] * w[0] - lam[0] * w[2]) * inv
        V[2, c] = (lam[0] * w[1] - lam[1] * w[0]) * inv
    return V


def P_apply(spec: Spectrum, y: np.ndarray) -> np.ndarray:
    """h = P_r y = (I_3 (x) T)(V y): 2n -> 3n, the magnetic field of an NFSEP vector."""
    V = hfield_mixing(spec.lam)
    y1, y2 = split_y(spec, y)
    return np.concatenate([T_apply(spec, V[l, 0] * y1 + V[l, 1] * y2) for l in range(3)])


def P_adjoint(spec: Spectrum, h: np.ndarray) -> np.ndarray:
    """P_r^* h = V^H (I_3 (x) T^*) h: 3n -> 2n."""
    n = spec.npts
    V = hfield_mixing(spec.lam)
    v = [Tstar_apply(spec, h[l * n:(l + 1) * n]) for l in range(3)]
    z1 = sum(np.conj(V[l, 0]) * v[l] for l in range(3))
    z2 = sum(np.conj(V[l, 1]) * v[l] for l in range(3))
    return np.concatenate([z1.reshape(-1), z2.reshape(-1)])


def Ar_apply(spec: Spectrum, eps_yee: np.ndarray, y: np.ndarray) -> np.ndarray:
    """A_r y (eq. NFSEP) with B = diag(eps_yee) (eps_yee shape (3, n))."""
    u = QS_apply(spec, y)
    u = u / np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    return QS_adjoint(spec, u)


def eigvec_from_y(spec: Spectrum, eps_yee: np.ndarray, y: np.ndarray) -> np.ndarray:
    """x = B^{-1} Q_r Sigma_r y (Theorem 5.2), e-layout, 3n."""
    return QS_apply(spec, y) / np.asarray(eps_yee, dtype=np.float64).reshape(-1)


def Ar_dense(spec: Spectrum, eps_yee: np.ndarray) -> np.ndarray:
    """Dense 2n x 2n A_r (tiny grids only), column by column."""
    N = 2 * spec.npts
    out = np.empty((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for col in range(N):
        e[:] = 0
        e[col] = 1
        out[:, col] = Ar_apply(spec, eps_yee, e)
    return out


def preconditioner_diag(spec: Spectrum) -> np.ndarray:
    """Lambda_q^{-1} per mode (0 where masked), 2n: the Sigma_r^{-2} scaling."""
    Lq = np.sum(np.abs(spec.lam) ** 2, axis=0)
    with np.errstate(divide="ignore"):
        d = np.where(Lq > 0, 1.0 / np.where(Lq > 0, Lq, 1.0), 0.0)
    return np.concatenate([d.reshape(-1), d.reshape(-1)])
