"""Smallest positive eigenvalues of A x = lambda B x (eq. GEP), plain definitions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

``dense_gep``  : scipy.linalg.eigh on the explicit C*C and B; all 3n eigenvalues.
``sparse_gep`` : shift-invert Lanczos (scipy eigsh) on the penalised pencil
                 (C*C + gamma (B G)(B G)^*, B) with G = [C1; C2; C3].
  The penalty leaves every eigenpair with G^* B x = 0 (the discrete
  divergence-free condition, eq. divergence_free) unchanged and moves the
  gradient (null-space) modes to >= gamma * eps_min * min Lambda_q; gamma is
  chosen so that they land far above the wanted band.  At kappa in Z^3 three
  more zero modes remain; they are removed by the positivity threshold.
``nfsep_dense``: eigenvalues of the dense 2n x 2n A_r (Theorem 5.2), tiny grids.

Positive threshold (reading of "smallest positive eigenvalues"): lambda > tol
with tol = 1e-9 * max(|lambda|) estimate; eigenvalues are counted with
multiplicity.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .curl import curl_matrix, gradient_matrix, mass_matrix
from .geometry import Geometry
from .nfsep import Ar_dense
from .spectral import spectrum


def _positive(w, tol_scale):
    tol = 1e-9 * tol_scale
    return w > tol


def dense_gep(geom: Geometry, kappa, eps_yee, nev: int):
    """Returns (lam[nev], X[3n, nev]) with X B-orthonormal."""
    C = curl_matrix(geom, kappa).toarray()
    A = C.conj().T @ C
    b = np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    w, V = sla.eigh(A, np.diag(b).astype(np.complex128))
    pos = _positive(w, np.max(np.abs(w)))
    w = w[pos][:nev]
    V = V[:, pos][:, :nev]
    return w, V


def all_gep_eigenvalues(geom: Geometry, kappa, eps_yee):
    C = curl_matrix(geom, kappa).toarray()
    A = C.conj().T @ C
    b = np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    return sla.eigh(A, np.diag(b).astype(np.complex128), eigvals_only=True)


def sparse_gep(geom: Geometry, kappa, eps_yee, nev: int, tol: float = 1e-13):
    """Shift-invert Lanczos on the divergence-penalised pencil."""
    spec = spectrum(geom, kappa)
    b = np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    eps_min = float(b.min())
    Lq = np.sort(np.sum(np.abs(spec.lam) ** 2, axis=0).ravel())
    Lq_pos = Lq[Lq > 0]
    # homogeneous eps_min medium bounds lambda_nev from above (eigenvalues decrease as eps grows)
    lam_upper = Lq_pos[min(len(Lq_pos) - 1, (nev + 1) // 2)] / eps_min
    gamma = 20.0 * lam_upper / (eps_min * Lq_pos[0])
    C = curl_matrix(geom, kappa)
    G = gradient_matrix(geom, kappa)
    B = mass_matrix(b)
    BG = B @ G
    A = (C.conj().T @ C + gamma * (BG @ BG.conj().T)).tocsc()
    sigma = -1e-3 * Lq_pos[0] / float(b.max())
    k = min(nev + 4, A.shape[0] - 2)
    w, V = spla.eigsh(A, k=k, M=B.tocsc(), sigma=sigma, which="LM", tol=tol)
    order = np.argsort(w)
    w = w[order]
    V = V[:, order]
    pos = _positive(w, lam_upper)
    w = w[pos][:nev]
    V = V[:, pos][:, :nev]
    if len(w) < nev:
        raise RuntimeError("sparse_gep: not enough positive eigenvalues found")
    return w, V


def nfsep_dense(geom: Geometry, kappa, eps_yee):
    """All eigenvalues of the dense A_r (Theorem 5.2), ascending."""
    spec = spectrum(geom, kappa)
    Ar = Ar_dense(spec, eps_yee)
    return sla.eigvalsh(0.5 * (Ar + Ar.conj().T))


def residuals(geom: Geometry, kappa, eps_yee, lam, X):
    """Relative residuals ||A x - lam B x|| / (lam ||B x||) with the explicit sparse C."""
    C = curl_matrix(geom, kappa)
    b = np.asarray(eps_yee, dtype=np.float64).reshape(-1)
    out = []
    for t in range(len(lam)):
        x = X[:, t]
        r = C.conj().T @ (C @ x) - lam[t] * b * x
        out.append(np.linalg.norm(r) / (abs(lam[t]) * np.linalg.norm(b * x)))
    return np.array(out)
