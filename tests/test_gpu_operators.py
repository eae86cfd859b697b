"""GPU parity of the operators behind the C ABI against the FP64 oracle, element by element.

Tolerances (normwise and element-wise relative to the largest reference entry):
  FP64: 1e-12 -- a few dozen rounding steps of size 1.1e-16 through three FFT passes;
  FP32: 2e-6  -- the same chain at FP32 rounding (6e-8) times log2(n) <= 21 passes and
                 the mixing coefficients computed in FP64 and rounded once.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import pcx_synth as S
from oracle.curl import double_curl
from oracle.geometry import lattice_geometry
from oracle.nfsep import Ar_apply, QS_adjoint, QS_apply, eigvec_from_y
from oracle.spectral import spectrum

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-6}


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


VARIANTS = {"auto": 0, "generic": 1, "three_plane": 2, "two_plane": 3, "register": 4}


def _setup(avec, n, kappa, eps, nvec=1, seed=0, variant="auto"):
    import torch
    from paper_1806_10284_amd import Plan, pcx_geometry
    g = pcx_geometry(avec, *n)
    og = lattice_geometry(avec, *n)
    assert tuple(g.shift) == tuple(int(s) for s in og.shift)
    plan = Plan(g, max_vectors=max(nvec, 4))
    plan.pcx_plan_set_eps(eps)
    plan.pcx_plan_set_variant(VARIANTS[variant])
    y = S.random_block(seed, 2 * og.npts, nvec)
    return plan, og, spectrum(og, kappa), y


def _to_dev(a, prec):
    import torch
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(dtype=dt, device="cuda").contiguous()


def _cmp(got, ref, prec, what):
    got = got.astype(np.complex128)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max() / scale
    nerr = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= TOL[prec] and nerr <= TOL[prec], f"{what}: max rel {err:.3e}, norm rel {nerr:.3e}"


CASES = [
    # name, lattice, grid, kappa, precisions
    ("sc4", S.SC, (4, 4, 4), (0.25, 0.1, -0.3)),
    ("mixed543", S.triclinic(1), (5, 4, 3), (0.11, -0.37, 0.42)),
    ("fcc8", S.FCC, (8, 8, 8), (0.5, 0.0, 0.5)),
    ("bcc_12_16_20", S.BCC, (12, 16, 20), (0.2, 0.3, -0.1)),
    ("mix_6_10_15", S.triclinic(2), (6, 10, 15), (-0.45, 0.05, 0.33)),
    ("hex_32_32_40", S.HEX, (32, 32, 40), (0.1, -0.2, 0.3)),
    ("ortho_60_48_40", S.ORTHO, (60, 48, 40), (0.3, 0.1, 0.2)),
    ("gamma_sc8", S.SC, (8, 8, 8), (0.0, 0.0, 0.0)),
    ("integer_kappa", S.triclinic(4), (6, 8, 5), (1.0, -1.0, 2.0)),
    # shapes with fixed-size kernels (planes 16x16, 32x32, 40x40; x lines 16, 32, 64)
    ("gamma_sc16", S.SC, (16, 16, 16), (0.0, 0.0, 0.0)),
    ("tri_32_40_40", S.triclinic(6), (32, 40, 40), (0.37, -0.21, 0.08)),
    ("fcc_64_32_32", S.FCC, (64, 32, 32), (0.25, 0.5, -0.125)),
    # large planes take the two-pass plane path: FP64 at 128 x 128 and 100 x 120 (ragged row and
    # column blocks), FP32 at all three (planes above 80 KB of LDS)
    ("split_hex_8_128_128", S.HEX, (8, 128, 128), (0.21, -0.33, 0.4)),
    ("split_ortho_6_100_120", S.ORTHO, (6, 100, 120), (-0.3, 0.45, 0.05)),
    ("split32_sc_4_144_150", S.SC, (4, 144, 150), (0.1, 0.2, -0.35)),
]


@pytest.mark.parametrize("variant", ["auto", "generic"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,avec,n,kappa", CASES)
def test_apply_Ar_parity(name, avec, n, kappa, prec, variant):
    import torch
    rng = np.random.default_rng(sum(map(ord, name)))
    npts = n[0] * n[1] * n[2]
    eps = rng.uniform(1.0, 13.0, (3, npts))
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=3, seed=7, variant=variant)
    say("apply_Ar", name, n, prec, variant)
    z = torch.empty_like(_to_dev(y, prec))
    plan.pcx_apply_Ar(kappa, _to_dev(y, prec), z)
    torch.cuda.synchronize()
    got = z.cpu().numpy().T
    for v in range(3):
        ref = Ar_apply(spec, eps, y[:, v])
        _cmp(got[:, v], ref, prec, f"{name} vec {v}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,avec,n,kappa", [CASES[1], CASES[4], CASES[7], CASES[9], CASES[11], CASES[13]])
def test_apply_precond_parity(name, avec, n, kappa, prec):
    """pcx_apply_precond = D A_r(eps -> 1/eps) D with D = Lambda_q^{-1} (0 on the Gamma mask), in
    place and out of place."""
    import torch
    from oracle.nfsep import preconditioner_diag
    rng = np.random.default_rng(sum(map(ord, name)) + 1)
    npts = n[0] * n[1] * n[2]
    eps = rng.uniform(1.0, 13.0, (3, npts))
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=2, seed=11)
    say("apply_precond", name, n, prec)
    d = preconditioner_diag(spec)
    yd = _to_dev(y, prec)
    z = torch.empty_like(yd)
    plan.pcx_apply_precond(kappa, yd, z)
    plan.pcx_apply_precond(kappa, yd, yd)
    torch.cuda.synchronize()
    got, got2 = z.cpu().numpy().T, yd.cpu().numpy().T
    for v in range(2):
        ref = d * Ar_apply(spec, 1.0 / eps, d * y[:, v])
        _cmp(got[:, v], ref, prec, f"{name} vec {v}")
        _cmp(got2[:, v], ref, prec, f"{name} vec {v} in place")


@pytest.mark.parametrize("variant", ["auto", "register"])
@pytest.mark.parametrize("name,avec,n,kappa", [
    ("fcc_8_64_64", S.FCC, (8, 64, 64), (0.5, 0.0, 0.5)),          # 64 x 64 planes: register kernels
    ("gamma_sc_4_64_64", S.SC, (4, 64, 64), (0.0, 0.0, 0.0)),      # the same, with the Gamma mask
    CASES[1], CASES[7], CASES[10]])                                # other plane kernels: FP32 copies
def test_apply_precond_fp64_op32_parity(name, avec, n, kappa, variant):
    """pcx_apply_precond with PCX_FP64_OP32 (complex128 in and out, the operator between the FP64
    scalings applied in FP32, as in the FP64 phase of the FP32 + refinement solver) against the
    FP64 oracle D A_r(eps -> 1/eps) D at the FP32 tolerance, in place and out of place; on 64 x 64
    planes the register kernels read FP64 and store the scaled FP64 result themselves."""
    import torch
    from oracle.nfsep import preconditioner_diag
    from paper_1806_10284_amd import PCX_FP64_OP32
    if variant == "register" and n[1:] != (64, 64):
        pytest.skip("the register kernels take 64 x 64 planes only")
    rng = np.random.default_rng(sum(map(ord, name)) + 5)
    npts = n[0] * n[1] * n[2]
    eps = rng.uniform(1.0, 13.0, (3, npts))
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=3, seed=13, variant=variant)
    say("apply_precond fp64_op32", name, n, variant)
    d = preconditioner_diag(spec)
    yd = _to_dev(y, "fp64")
    z = torch.empty_like(yd)
    plan.pcx_apply_precond(kappa, yd, z, precision=PCX_FP64_OP32)
    plan.pcx_apply_precond(kappa, yd, yd, precision=PCX_FP64_OP32)
    torch.cuda.synchronize()
    got, got2 = z.cpu().numpy().T, yd.cpu().numpy().T
    for v in range(3):
        ref = d * Ar_apply(spec, 1.0 / eps, d * y[:, v])
        _cmp(got[:, v], ref, "fp32", f"{name} vec {v}")
        _cmp(got2[:, v], ref, "fp32", f"{name} vec {v} in place")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,avec,n,kappa", [CASES[1], CASES[3], CASES[7], CASES[8]])
def test_QS_and_adjoint_and_eigvec(name, avec, n, kappa, prec):
    import torch
    rng = np.random.default_rng(99)
    npts = n[0] * n[1] * n[2]
    eps = rng.uniform(1.0, 13.0, (3, npts))
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=2, seed=3)
    say("QS", name, n, prec)
    yd = _to_dev(y, prec)
    u = torch.empty((2, 3 * npts), dtype=yd.dtype, device="cuda")
    plan.pcx_apply_QS(kappa, yd, u)
    x = torch.empty_like(u)
    plan.pcx_eigvec(kappa, yd, x)
    ur = rng.standard_normal((3 * npts, 2)) + 1j * rng.standard_normal((3 * npts, 2))
    z = torch.empty_like(yd)
    plan.pcx_apply_QS_adjoint(kappa, _to_dev(ur, prec), z)
    torch.cuda.synchronize()
    u, x, z = u.cpu().numpy().T, x.cpu().numpy().T, z.cpu().numpy().T
    for v in range(2):
        _cmp(u[:, v], QS_apply(spec, y[:, v]), prec, "QS")
        _cmp(x[:, v], eigvec_from_y(spec, eps, y[:, v]), prec, "eigvec")
        _cmp(z[:, v], QS_adjoint(spec, ur[:, v]), prec, "QS_adjoint")


@pytest.mark.parametrize("variant", ["auto", "generic", "two_plane", "three_plane", "register"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_Ar_fcc64_full_size(prec, variant):
    """The 64^3 diamond workload: every output entry against the oracle (numpy FFT route)."""
    import torch
    n = (64, 64, 64)
    og = lattice_geometry(S.FCC, *n)
    eps = S.sample_yee(S.FCC, n, og.shift, S.diamond_shapes(), 13.0, 1.0)
    kappa = (0.5, 0.0, 0.5)
    plan, og, spec, y = _setup(S.FCC, n, kappa, eps, nvec=1, seed=11, variant=variant)
    say("apply_Ar fcc64", prec, variant)
    z = torch.empty_like(_to_dev(y, prec))
    plan.pcx_apply_Ar(kappa, _to_dev(y, prec), z)
    torch.cuda.synchronize()
    _cmp(z.cpu().numpy().T[:, 0], Ar_apply(spec, eps, y[:, 0]), prec, "fcc64")


@pytest.mark.parametrize("case", ["fcc_X", "fcc_generic", "fcc_gamma", "bcc_16", "tri_24"])
def test_register_plane_kernels_64(case):
    """The register-resident FP32 kernels for 64 x 64 planes (8 lanes x 8 values per line, plane-major
    block order per XCD, W formed per mode from FP64 per-plane tables) on a 5-vector block: A_r, Q_r Sigma_r and its
    adjoint against the oracle for every vector, also at Gamma (masked mode) and for n1 = 16 and 24
    (two and three planes per XCD)."""
    import torch
    avec, n, kappa = {
        "fcc_X": (S.FCC, (64, 64, 64), (0.5, 0.0, 0.5)),
        "fcc_generic": (S.FCC, (64, 64, 64), (0.13, -0.41, 0.27)),
        "fcc_gamma": (S.FCC, (64, 64, 64), (0.0, 0.0, 0.0)),
        "bcc_16": (S.BCC, (16, 64, 64), (0.31, 0.07, -0.22)),
        "tri_24": (S.triclinic(5), (24, 64, 64), (-0.17, 0.38, 0.44)),
    }[case]
    og = lattice_geometry(avec, *n)
    rng = np.random.default_rng(19)
    eps = rng.uniform(1.0, 13.0, (3, og.npts))
    nv = 5
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=nv, seed=21, variant="register")
    say("register planes", case)
    yd = _to_dev(y, "fp32")
    z = torch.empty_like(yd)
    plan.pcx_apply_Ar(kappa, yd, z)
    u = torch.empty((nv, 3 * og.npts), dtype=yd.dtype, device="cuda")
    plan.pcx_apply_QS(kappa, yd, u)
    ur = S.random_block(22, 3 * og.npts, nv)
    zq = torch.empty_like(yd)
    plan.pcx_apply_QS_adjoint(kappa, _to_dev(ur, "fp32"), zq)
    torch.cuda.synchronize()
    z, u, zq = z.cpu().numpy().T, u.cpu().numpy().T, zq.cpu().numpy().T
    for v in range(nv):
        _cmp(z[:, v], Ar_apply(spec, eps, y[:, v]), "fp32", f"A_r vector {v}")
        _cmp(u[:, v], QS_apply(spec, y[:, v]), "fp32", f"QS vector {v}")
        _cmp(zq[:, v], QS_adjoint(spec, ur[:, v]), "fp32", f"QS adjoint vector {v}")


def test_nfsep_identity_with_explicit_curl_fcc64():
    """Q_r Sigma_r (A_r y) = C*C B^{-1} Q_r Sigma_r y with the oracle's explicit sparse C applied to
    the GPU's own outputs (a property that holds at any size)."""
    import torch
    n = (64, 64, 64)
    og = lattice_geometry(S.FCC, *n)
    eps = S.sample_yee(S.FCC, n, og.shift, S.diamond_shapes(), 13.0, 1.0)
    kappa = (0.5, 0.0, 0.5)
    plan, og, spec, y = _setup(S.FCC, n, kappa, eps, nvec=1, seed=12)
    say("identity fcc64")
    yd = _to_dev(y, "fp64")
    z = torch.empty_like(yd)
    plan.pcx_apply_Ar(kappa, yd, z)
    u = torch.empty((1, 3 * og.npts), dtype=yd.dtype, device="cuda")
    uz = torch.empty_like(u)
    plan.pcx_apply_QS(kappa, yd, u)
    plan.pcx_apply_QS(kappa, z, uz)
    torch.cuda.synchronize()
    u = u.cpu().numpy()[0]
    uz = uz.cpu().numpy()[0]
    A = double_curl(og, kappa)
    rhs = A @ (u / eps.reshape(-1))
    assert np.linalg.norm(uz - rhs) / np.linalg.norm(rhs) < 1e-11


def test_triclinic128_fp64_two_pass_planes():
    """128^3 triclinic in FP64 (its 128 x 128 planes take the two-pass path): every output entry."""
    import torch
    n = (128, 128, 128)
    avec = S.triclinic(5)
    og = lattice_geometry(avec, *n)
    eps = S.voxel_to_yee(S.random_sphere_fill(avec, n, og.shift, seed=5))
    kappa = tuple(S.random_kappas(5, 1)[0])
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=1, seed=14)
    say("apply_Ar tri128 fp64")
    z = torch.empty_like(_to_dev(y, "fp64"))
    plan.pcx_apply_Ar(kappa, _to_dev(y, "fp64"), z)
    torch.cuda.synchronize()
    _cmp(z.cpu().numpy().T[:, 0], Ar_apply(spec, eps, y[:, 0]), "fp64", "tri128 fp64")


def test_triclinic128_fp32_sampled():
    """128^3 triclinic (the largest workload): every output entry of one FP32 matvec."""
    import torch
    n = (128, 128, 128)
    avec = S.triclinic(5)
    og = lattice_geometry(avec, *n)
    eps = S.voxel_to_yee(S.random_sphere_fill(avec, n, og.shift, seed=5))
    kappa = tuple(S.random_kappas(5, 1)[0])
    plan, og, spec, y = _setup(avec, n, kappa, eps, nvec=1, seed=13)
    say("apply_Ar tri128 fp32")
    z = torch.empty_like(_to_dev(y, "fp32"))
    plan.pcx_apply_Ar(kappa, _to_dev(y, "fp32"), z)
    torch.cuda.synchronize()
    _cmp(z.cpu().numpy().T[:, 0], Ar_apply(spec, eps, y[:, 0]), "fp32", "tri128")


def test_errors_from_device_calls():
    import torch
    from paper_1806_10284_amd import Plan, PcxError, pcx_geometry
    g = pcx_geometry(S.SC, 4, 4, 4)
    plan = Plan(g, max_vectors=2)
    y = torch.zeros((1, 128), dtype=torch.complex128, device="cuda")
    with pytest.raises(PcxError):              # eps not set
        plan.pcx_apply_Ar((0.1, 0, 0), y, torch.empty_like(y))
    with pytest.raises(PcxError):
        plan.pcx_plan_set_eps(np.full(3 * 64, -1.0))
    with pytest.raises(PcxError):
        plan.pcx_plan_set_eps(np.full(3 * 64, np.nan))
    plan.pcx_plan_set_eps(np.full(64, 2.0), layout=1)
    y3 = torch.zeros((3, 128), dtype=torch.complex128, device="cuda")
    with pytest.raises(PcxError):              # more vectors than the plan allows
        plan.pcx_apply_Ar((0.1, 0, 0), y3, torch.empty_like(y3))
