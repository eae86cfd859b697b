"""The largest workload: a seeded triclinic lattice (lengths U[0.8, 1.2], angles U[70, 110] deg),
grid 128^3 (n = 2,097,152), random spheres (radii U[0.08, 0.15]) filled to 30 % with eps = 13,
20 bands at 16 seeded wave vectors solved as one batch with FP32 matvecs and FP64 refinement (the
refinement's FP64 planes of 128 x 128 take the two-pass plane path).

Checks: every problem converges (relative residual 1e-9, or the FP64 working-precision floor
1024 eps ||A_r|| for bands below it); for the first wave vector the first eigenvectors, mapped by
pcx_eigvec, satisfy the explicit GEP C*C x = lambda B x of the oracle (sparse Yee curl with Bloch
wraps) within the bound r * sqrt(max Lambda_q) / ||Sigma_r y|| derived in test_gpu_solve, r the
accepted relative residual, and x* B x = lambda.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import pcx_synth as S
from oracle.geometry import lattice_geometry
from oracle.nfsep import preconditioner_diag
from oracle.solve import residuals
from oracle.spectral import spectrum

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def test_triclinic128_batch_fp32_refine():
    import torch
    from paper_1806_10284_amd import PCX_EPS_VOXEL, PCX_MODE_FP32_REFINE, Plan, pcx_geometry, pcx_solve_batch
    n = (128, 128, 128)
    avec = S.triclinic(5)
    geom = pcx_geometry(avec, *n)
    vox = S.random_sphere_fill(avec, n, tuple(geom.shift), seed=5)
    kappas = [tuple(k) for k in S.random_kappas(55, 16)]
    nev, tol = 20, 1e-9
    plan = Plan(geom, max_vectors=32)
    plan.pcx_plan_set_eps(vox, PCX_EPS_VOXEL)
    say("config5 batch: 16 wave vectors, 20 bands, 128^3")
    t0 = time.perf_counter()
    lam, ys, stats = pcx_solve_batch([(plan, kappas)], nev, mode=PCX_MODE_FP32_REFINE, tol=tol, nworkers=2,
                                     want_y=[0])
    el = time.perf_counter() - t0
    say(f"config5: {el:.1f} s, {el / len(kappas):.2f} s per wave vector; iterations "
        f"{[s.iterations for s in stats]}, fp32 {[s.iterations_fp32 for s in stats]}")
    assert all(s.converged == nev for s in stats)
    assert np.all(np.diff(lam, axis=1) >= -1e-12 * lam[:, 1:])
    # eigenvectors of the first wave vector against the explicit GEP
    og = lattice_geometry(avec, *n)
    eps_yee = S.voxel_to_yee(vox)
    k0, m = kappas[0], 2
    y = ys[0][:m].contiguous()
    x = torch.empty((m, 3 * plan.n), dtype=torch.complex128, device="cuda")
    plan.pcx_eigvec(k0, y, x)
    torch.cuda.synchronize()
    X = x.cpu().numpy().T
    Y = y.cpu().numpy().T
    say("config5: explicit-curl residuals of 2 eigenvectors")
    res = residuals(og, k0, eps_yee, lam[0][:m], X)
    d = preconditioner_diag(spectrum(og, k0))
    lq = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    sig_y = np.sqrt(np.einsum("i,ij->j", lq, np.abs(Y) ** 2))
    # the solver accepts relative residual tol, or absolute residual 1024 eps ||A_r|| with
    # ||A_r|| <= max Lambda_q / min eps (bands it cannot resolve further)
    floor = 1024 * np.finfo(np.float64).eps / 2 * lq.max() / eps_yee.min()
    eff = np.maximum(tol, floor / lam[0][:m])
    bound = 1.5 * eff * np.sqrt(lq.max()) / sig_y
    say("config5 residuals", res, "bounds", bound)
    assert np.all(res < bound), (res, bound)
    b = eps_yee.reshape(-1)
    xbx = np.einsum("ij,i,ij->j", X.conj(), b, X).real
    np.testing.assert_allclose(xbx, lam[0][:m], rtol=1e-9)
