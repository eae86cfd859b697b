"""The Fourier basis T that diagonalises C_1, C_2, C_3 (paper Section 4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Columns of T (eq. T) are plane waves that satisfy the quasi-periodic condition
(eq. quasi_periodic): a plane wave exp(i g . p) on the integer grid picks up the
phase exp(i 2 pi kappa_l) over each lattice vector L_l (grid units) exactly
when g . L_l = 2 pi (kappa_l + nu_l) for integers nu_l.  With the lattice rows
M = [[n1,0,0],[s1,n2,0],[s2,s3,n3]] this is g = 2 pi M^{-1} (kappa + nu); a
complete set of distinct waves is nu = (i, j, k) in [0,n1) x [0,n2) x [0,n3).
In turns (g = 2 pi t):
    t_x(i)       = (kappa1 + i) / n1
    t_y(i, j)    = (kappa2 + j - s1 t_x) / n2
    t_z(i, j, k) = (kappa3 + k - s2 t_x - s3 t_y) / n3
and the eigenvalue of C_d on the wave is Lambda_d = (exp(i g_d) - 1) / delta_d
(Theorems 4.1-4.4).  Reading: the paper fixes T only up to the order of its
columns; this index map differs from the one printed in Theorems 4.2-4.4 by a
re-indexing j -> j + rho1 i (and the like), which the tests check as a
permutation of the same set of eigenvalue triples.

Column order (Section 4.2, eq. T): nu index = (i * n2 + j) * n3 + k (i slowest).
Row order: the e-layout a + n1 (b + n2 c).

``T_apply`` / ``Tstar_apply`` follow Algorithms 5.2 / 5.1: DFTs along the
three axes with diagonal twiddles in between; numpy.fft is the 1-D DFT.
The normalisation is n^{-1/2} (T is unitary; the 1/n printed in the
algorithms is read as n^{-1/2}).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import Geometry


@dataclass
class Spectrum:
    n: tuple
    shift: tuple
    delta: tuple
    kappa: np.ndarray
    tx: np.ndarray   # (n1,)          turns
    ty: np.ndarray   # (n1, n2)       turns
    tz: np.ndarray   # (n1, n2, n3)   turns
    lam: np.ndarray  # (3, n1, n2, n3) complex: Lambda_1, Lambda_2, Lambda_3

    @property
    def npts(self):
        return self.n[0] * self.n[1] * self.n[2]


def _turn_exp_minus_one(t):
    """exp(i 2 pi t) - 1 without cancellation: -2 sin^2(pi t) + i sin(2 pi t).
    The turn is first reduced to [-1/2, 1/2] (exact), so a whole turn gives exactly 0."""
    t = t - np.round(t)
    s = np.sin(np.pi * t)
    return -2.0 * s * s + 1j * np.sin(2.0 * np.pi * t)


def spectrum(geom: Geometry, kappa) -> Spectrum:
    n1, n2, n3 = geom.n
    s1, s2, s3 = geom.shift
    kappa = np.asarray(kappa, dtype=np.float64)
    i = np.arange(n1, dtype=np.float64)
    j = np.arange(n2, dtype=np.float64)
    k = np.arange(n3, dtype=np.float64)
    tx = (kappa[0] + i) / n1
    ty = (kappa[1] + j[None, :] - s1 * tx[:, None]) / n2
    tz = (kappa[2] + k[None, None, :] - s2 * tx[:, None, None] - s3 * ty[:, :, None]) / n3
    shape = (n1, n2, n3)
    lam = np.empty((3,) + shape, dtype=np.complex128)
    lam[0] = np.broadcast_to(_turn_exp_minus_one(tx)[:, None, None], shape) / geom.delta[0]
    lam[1] = np.broadcast_to(_turn_exp_minus_one(ty)[:, :, None], shape) / geom.delta[1]
    lam[2] = _turn_exp_minus_one(tz) / geom.delta[2]
    return Spectrum(n=geom.n, shift=geom.shift, delta=geom.delta, kappa=kappa,
                    tx=tx, ty=ty, tz=tz, lam=lam)


def T_dense(spec: Spectrum) -> np.ndarray:
    """T[p, nu] = n^{-1/2} exp(i g(nu) . p), dense n x n (for small grids)."""
    n1, n2, n3 = spec.n
    n = spec.npts
    c, b, a = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    a = a.ravel().astype(np.float64)
    b = b.ravel().astype(np.float64)
    c = c.ravel().astype(np.float64)
    shape = (n1, n2, n3)
    tx = np.broadcast_to(spec.tx[:, None, None], shape).ravel()
    ty = np.broadcast_to(spec.ty[:, :, None], shape).ravel()
    tz = spec.tz.ravel()
    phase = np.outer(a, tx) + np.outer(b, ty) + np.outer(c, tz)
    phase -= np.floor(phase)
    return np.exp(2j * np.pi * phase) / np.sqrt(n)


def _twiddles(spec: Spectrum):
    """Per-axis twiddle phases (turns) between the DFT passes of Algorithms 5.1/5.2:
    phi1 (scalar), phi2[i], phi3[i, j], so that
    t_x a = i a / n1 + a phi1, t_y b = j b / n2 + b phi2[i], t_z c = k c / n3 + c phi3[i, j]."""
    n1, n2, n3 = spec.n
    s1, s2, s3 = spec.shift
    kap = spec.kappa
    phi1 = kap[0] / n1
    phi2 = (kap[1] - s1 * spec.tx) / n2
    phi3 = (kap[2] - s2 * spec.tx[:, None] - s3 * spec.ty) / n3
    return phi1, phi2, phi3


def _cis_turns(x):
    x = x - np.floor(x)
    return np.exp(2j * np.pi * x)


def T_apply(spec: Spectrum, q: np.ndarray) -> np.ndarray:
    """T q by Algorithm 5.2.  q: (n1, n2, n3) Fourier layout -> (n,) e-layout."""
    n1, n2, n3 = spec.n
    phi1, phi2, phi3 = _twiddles(spec)
    a = np.arange(n1)
    b = np.arange(n2)
    c = np.arange(n3)
    X = np.fft.ifft(q, axis=2) * n3                                   # z: k -> c
    X = X * _cis_turns(c[None, None, :] * phi3[:, :, None])
    X = np.fft.ifft(X, axis=1) * n2                                   # y: j -> b
    X = X * _cis_turns(b[None, :, None] * phi2[:, None, None])
    X = np.fft.ifft(X, axis=0) * n1                                   # x: i -> a
    X = X * _cis_turns(a * phi1)[:, None, None]
    X = X / np.sqrt(spec.npts)
    return X.transpose(2, 1, 0).reshape(-1)                           # [c][b][a]


def Tstar_apply(spec: Spectrum, p: np.ndarray) -> np.ndarray:
    """T* p by Algorithm 5.1.  p: (n,) e-layout -> (n1, n2, n3) Fourier layout."""
    n1, n2, n3 = spec.n
    phi1, phi2, phi3 = _twiddles(spec)
    a = np.arange(n1)
    b = np.arange(n2)
    c = np.arange(n3)
    X = p.reshape(n3, n2, n1).transpose(2, 1, 0)                      # [a][b][c]
    X = X * np.conj(_cis_turns(a * phi1))[:, None, None]
    X = np.fft.fft(X, axis=0)                                         # x: a -> i
    X = X * np.conj(_cis_turns(b[None, :, None] * phi2[:, None, None]))
    X = np.fft.fft(X, axis=1)                                         # y: b -> j
    X = X * np.conj(_cis_turns(c[None, None, :] * phi3[:, :, None]))
    X = np.fft.fft(X, axis=2)                                         # z: c -> k
    return X / np.sqrt(spec.npts)
