"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's
own formula: they compare independent routes (the paper's printed matrices,
the explicit sparse operator, dense brute force, closed forms, invariances).
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import scipy.linalg as sla

import pcx_synth as S
from oracle.curl import curl_matrix, derivative_matrices, double_curl, gradient_matrix
from oracle.geometry import LatticeError, kappa_from_bloch, lattice_geometry, round_half_up
from oracle.grad import dlambda_dB, fd_dlambda_dB
from oracle.nfsep import Ar_apply, Ar_dense, QS_adjoint, QS_apply, mixing, preconditioner_diag
from oracle.paper_forms import paper_derivatives, paper_thetas
from oracle.solve import all_gep_eigenvalues, dense_gep, nfsep_dense, sparse_gep
from oracle.spectral import T_apply, T_dense, Tstar_apply, spectrum

from .helpers import random_geometry, sorted_triples

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------- geometry (Section 2.2)

def test_round_half_up():
    # Section 2.2: floor when the fractional part is < 1/2, ceil otherwise
    assert round_half_up(2.49) == 2
    assert round_half_up(2.5) == 3
    assert round_half_up(2.51) == 3
    assert round_half_up(3.0) == 3
    assert round_half_up(3.0 + 1e-12) == 3 and round_half_up(3.0 - 1e-12) == 3


@pytest.mark.parametrize("seed", range(20))
def test_geometry_invariants(seed):
    """eq. (transvec): lengths kept, a1 on x, a2 in xy, vectors end on grid points."""
    rng = np.random.default_rng(seed)
    A, g = random_geometry(rng, 4, 40, ang_lo=60, ang_hi=120)
    R = g.avec_rot
    for l in range(3):
        assert np.isclose(np.linalg.norm(R[:, l]), np.linalg.norm(A[:, l]), rtol=1e-13)
    assert R[1, 0] == 0 and R[2, 0] == 0 and R[2, 1] == 0
    dx, dy, dz = g.delta
    n1, n2, n3 = g.n
    s1, s2, s3 = g.shift
    assert np.isclose(R[0, 0], n1 * dx) and np.isclose(R[1, 1], n2 * dy) and np.isclose(R[2, 2], n3 * dz)
    assert np.isclose(R[0, 1], s1 * dx, atol=1e-13)
    assert np.isclose(R[0, 2], s2 * dx, atol=1e-13)
    assert np.isclose(R[1, 2], s3 * dy, atol=1e-13)
    # each corrected angle is within half a cell of the original
    cos_user = [A[:, 0] @ A[:, 1] / np.linalg.norm(A[:, 0]) / np.linalg.norm(A[:, 1]),
                A[:, 0] @ A[:, 2] / np.linalg.norm(A[:, 0]) / np.linalg.norm(A[:, 2])]
    assert abs(cos_user[0] * np.linalg.norm(A[:, 1]) - g.cos_angles[0] * np.linalg.norm(A[:, 1])) <= dx / 2 + 1e-12
    assert abs(cos_user[1] * np.linalg.norm(A[:, 2]) - g.cos_angles[1] * np.linalg.norm(A[:, 2])) <= dx / 2 + 1e-12


def test_geometry_exact_lattices_unchanged():
    """When the offsets are whole cells no correction happens (Section 2.2, 'theta = theta'')."""
    g = lattice_geometry(S.FCC, 66, 66, 66)       # 66 divisible by 2 and 3: FCC lands on the grid
    assert g.m == (33, 33, 22)
    assert np.allclose(np.degrees(np.arccos(g.cos_angles)), 60.0, atol=1e-10)
    g = lattice_geometry(S.ORTHO, 60, 48, 40)
    assert g.m == (0, 0, 0) and g.shift == (0, 0, 0)
    assert np.allclose(g.delta, (0.025, 0.025, 0.025))


def test_geometry_fcc64_correction():
    """FCC at 64^3: m3 = 64 * 1/3 rounds to 21, so alpha is corrected away from 60 degrees."""
    g = lattice_geometry(S.FCC, 64, 64, 64)
    assert g.m == (32, 32, 21) and g.rho == (0, 0, 0)
    assert abs(np.degrees(np.arccos(g.cos_angles[2])) - 60.0) > 0.1


def test_geometry_rejects_bad_cells():
    with pytest.raises(LatticeError):
        lattice_geometry(np.array([[1, 1, 0], [0, 1e-14, 0], [0, 0, 1.0]]), 4, 4, 4)
    with pytest.raises(LatticeError):        # a2 sticks out of the cell along x
        lattice_geometry(np.array([[1, 2.5, 0], [0, 1, 0], [0, 0, 1.0]]), 4, 4, 4)


def test_kappa_fcc_x_point():
    """G17 reading: X = (2 pi / a)(0,1,0) on the FCC primitive vectors -> kappa = (1/2, 0, 1/2)."""
    kap = kappa_from_bloch(S.FCC, S.FCC_POINTS["X"])
    assert np.allclose(kap, [0.5, 0.0, 0.5], atol=1e-15)


# ---------------------------------------------------------------- Section 3: explicit curl

# first seeds hitting each (rho, split) pattern in a 400-seed sweep, plus a random range
LISTING_SEEDS = sorted(set(range(40)) | {97, 41})


def _listing_geometry(seed):
    rng = np.random.default_rng(1000 + seed)
    while True:
        A, g = random_geometry(rng)
        if g.m[0] < g.n[0] and g.m[1] < g.n[0] and g.m[2] < g.n[1]:
            return rng, g


@pytest.mark.parametrize("seed", LISTING_SEEDS)
def test_wrap_matches_paper_listings(seed):
    """The quasi-periodic wrap equals K1 (eq. K1), K2 with J2 (eq. J2) and K3 with
    the general J3 categories (eqs. acuteJ3/obtuseJ3) entry by entry, for
    0 <= m < n (the listings' case bits are not defined consistently at m = n)."""
    rng, g = _listing_geometry(seed)
    kap = rng.uniform(-0.5, 0.5, 3)
    C = [m.toarray() for m in derivative_matrices(g, kap)]
    P = paper_derivatives(g, kap)
    for d in range(3):
        np.testing.assert_allclose(C[d], P[d], atol=1e-12, rtol=0)


def test_wrap_listing_cases_covered():
    """All eight (rho1, rho2, rho3) patterns and the m1<=m2 / m1+m2<n1 splits occur in the
    sweep: 15 of the 16 combinations (rho = (1,1,1) with m1 + m2 < n1 needs
    |a2_x| + |a3_x| > |a1| and is not drawn)."""
    seen = set()
    for seed in LISTING_SEEDS:
        _, g = _listing_geometry(seed)
        split = (g.m[0] <= g.m[1]) if g.rho[2] == 0 else (g.m[0] + g.m[1] < g.n[0])
        seen.add((g.rho, split))
    assert len({r for r, _ in seen}) == 8
    assert len(seen) == 15


def test_curl_of_gradient_is_zero_and_null_dimension():
    """C G = 0 (the C_d commute); rank(C) = 2n, i.e. null(C*C) has dimension n (Section 5.2)
    and n + 2 at kappa = 0."""
    rng = np.random.default_rng(7)
    A, g = random_geometry(rng, 3, 5)
    for kap, extra in ((rng.uniform(-0.5, 0.5, 3), 0), (np.zeros(3), 2)):
        C = curl_matrix(g, kap).toarray()
        G = gradient_matrix(g, kap).toarray()
        assert np.abs(C @ G).max() < 1e-10
        sv = np.linalg.svd(C, compute_uv=False)
        null = int(np.sum(sv < 1e-9 * sv.max()))
        assert null == g.npts + extra


# ---------------------------------------------------------------- Section 4: spectra and T

@pytest.mark.parametrize("seed", range(30))
def test_theorems_4_1_to_4_4_spectrum(seed):
    """The eigenvalue triples of Theorems 4.1-4.4 (as printed) equal the oracle's, as a set."""
    rng = np.random.default_rng(2000 + seed)
    A, g = random_geometry(rng, 3, 7)
    kap = rng.uniform(-0.5, 0.5, 3)
    spec = spectrum(g, kap)
    shape = g.n
    a = sorted_triples(*paper_thetas(g, kap))
    b = sorted_triples(np.broadcast_to(spec.tx[:, None, None], shape),
                       np.broadcast_to(spec.ty[:, :, None], shape), spec.tz)
    np.testing.assert_allclose(a, b, atol=1e-7)


@pytest.mark.parametrize("seed", range(12))
def test_T_unitary_and_diagonalises(seed):
    """T*T = I and C_l T = T Lambda_l with the explicit sparse C_l (Section 4.2)."""
    rng = np.random.default_rng(3000 + seed)
    A, g = random_geometry(rng, 3, 6)
    kap = rng.uniform(-0.5, 0.5, 3)
    spec = spectrum(g, kap)
    T = T_dense(spec)
    assert np.abs(T.conj().T @ T - np.eye(T.shape[0])).max() < 1e-12
    C = derivative_matrices(g, kap)
    for d in range(3):
        lhs = C[d] @ T
        rhs = T * spec.lam[d].reshape(-1)[None, :]
        assert np.abs(lhs - rhs).max() * g.delta[d] < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_fft_algorithms_match_dense_T(seed):
    """Algorithms 5.2 (T q) and 5.1 (T* p) equal the dense T on random vectors."""
    rng = np.random.default_rng(4000 + seed)
    A, g = random_geometry(rng, 3, 7)
    kap = rng.uniform(-1.5, 1.5, 3)
    spec = spectrum(g, kap)
    T = T_dense(spec)
    q = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    np.testing.assert_allclose(T_apply(spec, q), T @ q.reshape(-1), atol=1e-12)
    p = rng.standard_normal(g.npts) + 1j * rng.standard_normal(g.npts)
    np.testing.assert_allclose(Tstar_apply(spec, p).reshape(-1), T.conj().T @ p, atol=1e-12)


def test_orthorhombic_T_is_numpy_ifftn_with_bloch_phase():
    """Orthorhombic (no shifts): T q = sqrt(n) ifftn(q) times exp(i 2 pi kappa . p / n) -- a textbook FFT."""
    g = lattice_geometry(S.ORTHO, 6, 5, 4)
    kap = np.array([0.3, -0.2, 0.45])
    spec = spectrum(g, kap)
    rng = np.random.default_rng(5)
    q = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    ref = np.fft.ifftn(q) * math.sqrt(g.npts)                 # [a][b][c]
    a, b, c = np.meshgrid(*(np.arange(x) for x in g.n), indexing="ij")
    ref = ref * np.exp(2j * np.pi * (kap[0] * a / 6 + kap[1] * b / 5 + kap[2] * c / 4))
    np.testing.assert_allclose(T_apply(spec, q), ref.transpose(2, 1, 0).reshape(-1), atol=1e-12)


# ---------------------------------------------------------------- Section 5: SVD, NFSEP

@pytest.mark.parametrize("seed", range(6))
def test_mixing_basis_properties(seed):
    """W^H W = Lambda_q I_2, W^H Lambda = 0 and W W^H = Lambda_q I_3 - Lambda Lambda^H
    (the Fourier symbol of C*C, eq. double_eigendecomposition)."""
    rng = np.random.default_rng(5000 + seed)
    A, g = random_geometry(rng, 3, 8)
    kap = rng.uniform(-0.5, 0.5, 3)
    lam = spectrum(g, kap).lam.reshape(3, -1)
    W = mixing(lam)
    Lq = np.sum(np.abs(lam) ** 2, axis=0)
    WhW = np.einsum("lan,lbn->abn", W.conj(), W)
    assert np.abs(WhW - np.eye(2)[:, :, None] * Lq).max() < 1e-12 * Lq.max()
    assert np.abs(np.einsum("lan,ln->an", W.conj(), lam)).max() < 1e-12 * Lq.max()
    WWh = np.einsum("lan,man->lmn", W, W.conj())
    sym = Lq * np.eye(3)[:, :, None] - np.einsum("ln,mn->lmn", lam, lam.conj())
    assert np.abs(WWh - sym).max() < 1e-12 * Lq.max()
    # Lambda_p^2 = 3 Lambda_q - |Lambda_s|^2 (the reading of the garbled definition)
    Ls = lam.sum(axis=0)
    Lp2 = sum(np.abs(lam[a] - lam[b]) ** 2 for a, b in ((0, 1), (0, 2), (1, 2)))
    assert np.abs(Lp2 - (3 * Lq - np.abs(Ls) ** 2)).max() < 1e-12 * Lq.max()


def test_mixing_degenerate_modes():
    """Simple cubic at Gamma: Lambda_1 = Lambda_2 = Lambda_3 on the diagonal modes i=j=k,
    where the paper's basis degenerates; the fallback basis still spans the range."""
    g = lattice_geometry(S.SC, 4, 4, 4)
    lam = spectrum(g, np.zeros(3)).lam.reshape(3, -1)
    W = mixing(lam)
    Lq = np.sum(np.abs(lam) ** 2, axis=0)
    diag_modes = [(i * 4 + i) * 4 + i for i in range(1, 4)]
    for nu in diag_modes:
        assert np.isclose(abs(lam[0, nu] - lam[1, nu]), 0) and Lq[nu] > 0
        G = W[:, :, nu].conj().T @ W[:, :, nu]
        assert np.allclose(G, Lq[nu] * np.eye(2), atol=1e-12)
        assert np.allclose(W[:, :, nu].conj().T @ lam[:, nu], 0, atol=1e-12)
    assert np.all(W[:, :, 0] == 0)          # the masked mode


@pytest.mark.parametrize("seed,gamma", [(0, False), (1, False), (2, False), (3, True), (4, True)])
def test_theorem_5_2_brute_force(seed, gamma):
    """eig(A_r) = the positive eigenvalues of A x = lambda B x (Theorem 5.2), dense."""
    rng = np.random.default_rng(6000 + seed)
    A, g = random_geometry(rng, 3, 5)
    kap = np.zeros(3) if gamma else rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    w = all_gep_eigenvalues(g, kap, eps)
    pos = np.sort(w[w > 1e-9 * w.max()])
    wr = nfsep_dense(g, kap, eps)
    wr = np.sort(wr[wr > 1e-9 * wr.max()])
    assert len(pos) == 2 * g.npts - (2 if gamma else 0)
    np.testing.assert_allclose(wr, pos, rtol=1e-11, atol=1e-11 * pos.max())


def test_homogeneous_closed_form():
    """Homogeneous eps0: the positive eigenvalues are Lambda_q(nu) / eps0, each twice (eq. double_eigendecomposition)."""
    rng = np.random.default_rng(11)
    A, g = random_geometry(rng, 3, 6)
    kap = rng.uniform(-0.5, 0.5, 3)
    lam = spectrum(g, kap).lam
    Lq = np.sum(np.abs(lam) ** 2, axis=0).ravel()
    # closed form written from the symbol: |e^{i g} - 1|^2 = 4 sin^2(g / 2)
    t = (kap[0] + np.arange(g.n[0])) / g.n[0]
    assert np.allclose(np.abs(lam[0, :, 0, 0]) ** 2, 4 * np.sin(np.pi * t) ** 2 / g.delta[0] ** 2)
    w = all_gep_eigenvalues(g, kap, np.full((3, g.npts), 2.5))
    pos = np.sort(w[w > 1e-9 * w.max()])
    np.testing.assert_allclose(pos, np.sort(np.concatenate([Lq, Lq])) / 2.5, rtol=1e-10, atol=1e-10 * pos.max())


def test_conditioning_bound():
    """kappa(Q_r^* B^{-1} Q_r) <= kappa(B^{-1}) (Section 5.2): the spectrum of the
    Sigma_r^{-1} A_r Sigma_r^{-1} lies in [1/eps_max, 1/eps_min]."""
    rng = np.random.default_rng(12)
    A, g = random_geometry(rng, 3, 5)
    kap = rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    spec = spectrum(g, kap)
    Ar = Ar_dense(spec, eps)
    d = np.sqrt(preconditioner_diag(spec))
    K = d[:, None] * Ar * d[None, :]
    ev = np.linalg.eigvalsh(0.5 * (K + K.conj().T))
    assert ev.min() >= 1 / eps.max() - 1e-12 and ev.max() <= 1 / eps.min() + 1e-12


def test_approximate_inverse_preconditioner_spectrum():
    """T = D Sigma_r Q_r^* B Q_r Sigma_r D (D = Lambda_q^{-1}; A_r with eps in place of 1/eps):
    T A_r is similar to (Q_r^* B Q_r)(Q_r^* B^{-1} Q_r), whose eigenvalues lie in
    [1, (M + m)^2 / (4 M m)] for eps in [m, M] (the matrix Kantorovich inequality: for an isometry
    Q, (Q^* B Q)^{-1} <= Q^* B^{-1} Q <= (M + m)^2 / (4 M m) (Q^* B Q)^{-1}); constant eps: T = A_r^{-1}."""
    rng = np.random.default_rng(21)
    A, g = random_geometry(rng, 3, 5)
    kap = rng.uniform(-0.5, 0.5, 3)
    spec = spectrum(g, kap)
    d = preconditioner_diag(spec)
    for eps in (rng.uniform(1.0, 13.0, (3, g.npts)), np.full((3, g.npts), 4.0)):
        Ar = Ar_dense(spec, eps)
        T = d[:, None] * Ar_dense(spec, 1.0 / eps) * d[None, :]
        ev = np.linalg.eigvals(T @ Ar)
        assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max()
        ev = np.sort(ev.real)
        m, M = eps.min(), eps.max()
        kant = (M + m) ** 2 / (4 * M * m)
        assert ev.min() >= 1 - 1e-10 and ev.max() <= kant + 1e-10, (ev.min(), ev.max(), kant)
        if m == M:
            np.testing.assert_allclose(ev, 1.0, atol=1e-10)
    # the bound is attained up to the grid's freedom: for contrast 13 it is far below 13
    assert (14.0 ** 2) / (4 * 13.0) < 3.8


@pytest.mark.parametrize("lat,n", [("fcc", (8, 8, 8)), ("bcc", (6, 8, 5)), ("hex", (8, 8, 10))])
def test_nfsep_identity_with_explicit_curl(lat, n):
    """Q_r Sigma_r (A_r y) = C*C B^{-1} Q_r Sigma_r y with the explicit sparse C (Theorem 5.2's proof)."""
    avec = {"fcc": S.FCC, "bcc": S.BCC, "hex": S.HEX}[lat]
    g = lattice_geometry(avec, *n)
    rng = np.random.default_rng(13)
    kap = rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    spec = spectrum(g, kap)
    y = rng.standard_normal(2 * g.npts) + 1j * rng.standard_normal(2 * g.npts)
    lhs = QS_apply(spec, Ar_apply(spec, eps, y))
    Amat = double_curl(g, kap)
    rhs = Amat @ (QS_apply(spec, y) / eps.reshape(-1))
    np.testing.assert_allclose(lhs, rhs, atol=1e-10 * np.abs(rhs).max())
    # and Sigma_r Q_r^* is the adjoint of Q_r Sigma_r
    u = rng.standard_normal(3 * g.npts) + 1j * rng.standard_normal(3 * g.npts)
    assert np.isclose(np.vdot(u, QS_apply(spec, y)), np.vdot(QS_adjoint(spec, u), y), rtol=1e-12)


# ---------------------------------------------------------------- solvers, invariances, gradient

def test_sparse_and_dense_solvers_agree():
    g = lattice_geometry(S.SC, 8, 8, 8)
    rng = np.random.default_rng(14)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    kap = np.array([0.25, 0.0, 0.0])
    wd, Xd = dense_gep(g, kap, eps, 10)
    ws, Xs = sparse_gep(g, kap, eps, 10)
    np.testing.assert_allclose(ws, wd, rtol=1e-10)


def test_invariances():
    """kappa + Z^3 and -kappa (real eps) leave lambda unchanged; eps -> c eps gives lambda / c;
    scaling the lattice by s gives lambda / s^2."""
    rng = np.random.default_rng(15)
    A, g = random_geometry(rng, 3, 5)
    kap = rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    w0 = all_gep_eigenvalues(g, kap, eps)
    w1 = all_gep_eigenvalues(g, kap + np.array([1.0, -2.0, 3.0]), eps)
    w2 = all_gep_eigenvalues(g, -kap, eps)
    w3 = all_gep_eigenvalues(g, kap, 3.0 * eps)
    g2 = lattice_geometry(2.0 * A, *g.n)
    w4 = all_gep_eigenvalues(g2, kap, eps)
    sc = np.abs(w0).max()
    assert np.abs(np.sort(w0) - np.sort(w1)).max() < 1e-10 * sc
    assert np.abs(np.sort(w0) - np.sort(w2)).max() < 1e-10 * sc
    assert np.abs(np.sort(w0) / 3.0 - np.sort(w3)).max() < 1e-10 * sc
    assert np.abs(np.sort(w0) / 4.0 - np.sort(w4)).max() < 1e-10 * sc


def test_gradient_fd_and_sum_rule():
    """d lambda / d B_pp = -lambda |x_p|^2 / x*Bx vs central differences; the sum rule
    sum_p B_pp d lambda / d B_pp = -lambda (lambda is homogeneous of degree -1 in eps)."""
    g = lattice_geometry(S.FCC, 4, 4, 4)
    rng = np.random.default_rng(16)
    kap = np.array([0.31, -0.07, 0.19])
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    w, X = dense_gep(g, kap, eps, 4)
    gaps = np.diff(w)
    band = int(np.argmax(np.minimum(np.r_[np.inf, gaps], np.r_[gaps, np.inf])[:4]))
    grad = dlambda_dB(w[band], X[:, band], eps)
    assert np.isclose(np.sum(eps * grad), -w[band], rtol=1e-10)
    for comp, point in ((0, 3), (1, 17), (2, 40)):
        fd = fd_dlambda_dB(g, kap, eps, band, comp, point, 1e-5)
        assert np.isclose(fd, grad[comp, point], rtol=1e-5, atol=1e-9 * abs(w[band]))


def test_gradient_via_nfsep_vector():
    """x = B^{-1} Q_r Sigma_r y gives x*Bx = lambda ||y||^2, so dlambda/dB_pp = -|x_p|^2 / ||y||^2."""
    from oracle.nfsep import eigvec_from_y
    g = lattice_geometry(S.SC, 4, 4, 3)
    rng = np.random.default_rng(17)
    kap = np.array([0.2, 0.1, -0.3])
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    spec = spectrum(g, kap)
    Ar = Ar_dense(spec, eps)
    ev, V = np.linalg.eigh(0.5 * (Ar + Ar.conj().T))
    y = V[:, 0]
    x = eigvec_from_y(spec, eps, y)
    b = eps.reshape(-1)
    assert np.isclose(np.vdot(x, b * x).real, ev[0] * np.vdot(y, y).real, rtol=1e-10)
    # and x solves the GEP
    Amat = double_curl(g, kap)
    assert np.linalg.norm(Amat @ x - ev[0] * b * x) < 1e-9 * ev[0] * np.linalg.norm(b * x)


@pytest.mark.parametrize("seed,gamma", [(11, False), (12, True)])
def test_inverse_lanczos_matches_dense_gep(seed, gamma):
    """Section 5.2's method in the oracle (Lanczos on A_r^{-1}, CG inner solves on the FFT operator)
    returns the smallest positive eigenvalues of the explicit-curl GEP, with multiplicity, also at
    Gamma where A_r keeps the masked mode's two zero eigenvalues outside Sigma_r's range."""
    from oracle.solve import nfsep_inverse_lanczos, nfsep_residuals
    rng = np.random.default_rng(seed)
    avec, g = random_geometry(rng, nlo=3, nhi=5)
    kap = np.zeros(3) if gamma else rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    nev = 6
    ref, _ = dense_gep(g, kap, eps, nev)
    spec = spectrum(g, kap)
    lam, Y, info = nfsep_inverse_lanczos(spec, eps, nev, ncv=min(2 * 2 * g.npts - 2, 40))
    np.testing.assert_allclose(lam, ref, rtol=1e-10)
    assert nfsep_residuals(spec, eps, lam, Y).max() < 1e-9
    assert info["ar_applications"] == info["cg_iterations"] > 0


def test_inverse_lanczos_matches_config1_golden():
    """At the SC 16^3 workload the inverse-Lanczos oracle equals the stored explicit-curl
    shift-invert eigenvalues (tests/golden/config1_sc16.json) to 1e-10."""
    import json
    import os
    from oracle.solve import nfsep_inverse_lanczos
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config1_sc16.json")))
    g = lattice_geometry(S.SC, 16, 16, 16)
    kap = kappa_from_bloch(S.SC, np.array([np.pi / 2, 0.0, 0.0]))
    eps = S.sample_yee(S.SC, g.n, g.shift, S.sc_sphere_shapes(), 13.0, 1.0)
    lam, _, _ = nfsep_inverse_lanczos(spectrum(g, kap), eps, 10)
    np.testing.assert_allclose(lam, gold["lambda"], rtol=1e-10)


@pytest.mark.parametrize("seed,gamma", [(21, False), (22, True), (23, False)])
def test_svd_of_the_explicit_curl(seed, gamma):
    """Theorem 5.1 with the explicit sparse C (dense SVD at small grids): the singular values are
    sqrt(Lambda_q) of every mode, twice, and n zeros; at kappa in Z^3 (the Gamma-point SVD) the one mode
    with Lambda_q = 0 adds two more zeros (n + 2).  The oracle's left and right singular vectors
    P_r = (I_3 (x) T) V and Q_r = (I_3 (x) T) W Sigma_r^{-1} satisfy C Q_r = P_r Sigma_r and
    C^* P_r = Q_r Sigma_r, and P_r has orthonormal columns."""
    from oracle.curl import curl_matrix
    from oracle.nfsep import P_adjoint, P_apply, QS_apply, QS_adjoint
    rng = np.random.default_rng(seed)
    avec, g = random_geometry(rng, nlo=3, nhi=5)
    kap = np.zeros(3) if gamma else rng.uniform(-0.5, 0.5, 3)
    n = g.npts
    C = curl_matrix(g, kap).toarray()
    sv = np.sort(np.linalg.svd(C, compute_uv=False))
    spec = spectrum(g, kap)
    lq = np.sort(np.sum(np.abs(spec.lam) ** 2, axis=0).reshape(-1))
    nz = n + 2 if gamma else n
    assert np.all(sv[:nz] < 1e-10 * sv[-1])
    ref = np.sort(np.sqrt(np.repeat(lq[lq > 0], 2)))
    np.testing.assert_allclose(sv[nz:], ref, rtol=1e-10)
    # dense P_r and Q_r Sigma_r, column by column
    P = np.stack([P_apply(spec, e) for e in np.eye(2 * n)], axis=1)
    QS = np.stack([QS_apply(spec, e) for e in np.eye(2 * n)], axis=1)
    lq2 = np.concatenate([np.sum(np.abs(spec.lam) ** 2, axis=0).reshape(-1)] * 2)
    live = lq2 > 0
    G = P.conj().T @ P
    np.testing.assert_allclose(G[np.ix_(live, live)], np.eye(live.sum()), atol=1e-12)
    assert not np.any(P[:, ~live])
    # C Q_r Sigma_r = P_r Sigma_r^2 and C^* P_r = Q_r Sigma_r
    np.testing.assert_allclose(C @ QS, P * lq2[None, :], atol=1e-10 * lq2.max())
    np.testing.assert_allclose(C.conj().T @ P, QS, atol=1e-10 * np.sqrt(lq2.max()))
    # the adjoint map
    h = rng.standard_normal(3 * n) + 1j * rng.standard_normal(3 * n)
    np.testing.assert_allclose(P_adjoint(spec, h), P.conj().T @ h, atol=1e-12 * np.abs(h).max())


@pytest.mark.parametrize("seed", [31, 32])
def test_hfield_operator_and_nfsep(seed):
    """The magnetic-field operator C B^{-1} C^* (explicit C) has the same positive eigenvalues as the GEP,
    and P_r^* (C B^{-1} C^*) P_r = A_r (dense, random eps)."""
    from oracle.curl import curl_matrix
    from oracle.nfsep import P_apply
    rng = np.random.default_rng(seed)
    avec, g = random_geometry(rng, nlo=3, nhi=5)
    kap = rng.uniform(-0.5, 0.5, 3)
    eps = rng.uniform(1.0, 13.0, (3, g.npts))
    C = curl_matrix(g, kap).toarray()
    H = C @ np.diag(1.0 / eps.reshape(-1)) @ C.conj().T
    wh = np.linalg.eigvalsh(0.5 * (H + H.conj().T))
    wh = wh[wh > 1e-9 * wh.max()]
    ref, _ = dense_gep(g, kap, eps, len(wh))
    np.testing.assert_allclose(wh, ref, rtol=1e-9)
    spec = spectrum(g, kap)
    n2 = 2 * g.npts
    P = np.stack([P_apply(spec, e) for e in np.eye(n2)], axis=1)
    Ar = Ar_dense(spec, eps)
    np.testing.assert_allclose(P.conj().T @ H @ P, Ar, atol=1e-9 * np.abs(Ar).max())
