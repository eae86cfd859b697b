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


def nfsep_inverse_lanczos(spec, eps_yee, nev: int, tol_outer: float = 1e-12, tol_inner: float = 1e-13,
                          seed: int = 1, ncv: int | None = None):
    """The method of Section 5.2 for grids beyond the sparse factorisation: Lanczos on A_r^{-1}.

    A_r = Sigma_r M Sigma_r with M = Q_r^* B^{-1} Q_r Hermitian positive definite and
    cond(M) <= max(eps) / min(eps) (the bound of Section 5.2), so
        A_r^{-1} v = Sigma_r^{-1} M^{-1} Sigma_r^{-1} v,
    each M^{-1} an unpreconditioned conjugate-gradient solve (relative residual tol_inner) whose
    M products are Sigma_r^{-1} A_r Sigma_r^{-1} with the FFT operator of this package.  The largest
    eigenvalues theta of A_r^{-1} (implicitly restarted Lanczos, scipy eigsh, relative accuracy
    tol_outer) give lambda = 1 / theta.  Modes with Lambda_q = 0 (kappa in Z^3) are outside the
    range of Sigma_r and are held at zero.

    Returns (lam[nev] ascending, Y[2n, nev] orthonormal NFSEP eigenvectors, info) with info the
    number of A_r applications and CG iterations.
    """
    from .nfsep import Ar_apply
    n = spec.npts
    Lq = np.sum(np.abs(spec.lam) ** 2, axis=0).reshape(-1)
    live = np.concatenate([Lq, Lq]) > 0
    sig_inv = np.zeros(2 * n)
    sig_inv[live] = 1.0 / np.sqrt(np.concatenate([Lq, Lq])[live])
    info = {"ar_applications": 0, "cg_iterations": 0, "inner_solves": 0}

    def m_apply(v):
        info["ar_applications"] += 1
        return sig_inv * Ar_apply(spec, eps_yee, sig_inv * v)

    M = spla.LinearOperator((2 * n, 2 * n), matvec=m_apply, dtype=np.complex128)

    def cg_count(_xk):
        info["cg_iterations"] += 1

    def ainv_apply(v):
        rhs = sig_inv * np.asarray(v).reshape(-1)
        info["inner_solves"] += 1
        w, flag = spla.cg(M, rhs, rtol=tol_inner, atol=0.0, maxiter=20000, callback=cg_count)
        if flag != 0:
            raise RuntimeError(f"nfsep_inverse_lanczos: CG did not converge (flag {flag})")
        return sig_inv * w

    Ainv = spla.LinearOperator((2 * n, 2 * n), matvec=ainv_apply, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = (rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)) * live
    k = nev
    theta, Y = spla.eigsh(Ainv, k=k, which="LA", tol=tol_outer, v0=v0,
                          ncv=ncv or min(2 * n - 2, max(2 * k + 1, 24)))
    order = np.argsort(-theta)
    theta = theta[order]
    Y = Y[:, order]
    lam = 1.0 / theta
    Y = Y / np.linalg.norm(Y, axis=0)
    return lam, Y, info


def nfsep_residuals(spec, eps_yee, lam, Y):
    """||A_r y - lam y|| / (lam ||y||) per column with the FFT operator."""
    from .nfsep import Ar_apply
    out = []
    for t in range(len(lam)):
        y = Y[:, t]
        r = Ar_apply(spec, eps_yee, y) - lam[t] * y
        out.append(np.linalg.norm(r) / (abs(lam[t]) * np.linalg.norm(y)))
    return np.array(out)
