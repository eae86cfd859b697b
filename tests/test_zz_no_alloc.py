"""pcx_apply_Ar_noalloc: z = A_r y with every temporary in the library's static device scratch.

Checked through the C ABI against pcx_apply_Ar on the same plan and inputs (FP64 1e-12, FP32 2e-6
relative: the same kernels, except that the fixed-size FP32 adjoint forms the mixing W per mode
instead of reading the plan's table) and against the oracle's A_r, on calls in a row whose
second input is smaller than the first (the scratch keeps the previous call's contents).  The
calls must not change the device's free memory, and a block larger than the scratch is refused
before anything is launched.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import pcx_synth as S
from oracle.geometry import lattice_geometry
from oracle.nfsep import Ar_apply
from oracle.spectral import spectrum

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-6}


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _dev(a, prec):
    import torch
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(dtype=dt, device="cuda").contiguous()


def _case(avec, n, kappa, prec, nvec, seed):
    from paper_1806_10284_amd import Plan, pcx_geometry
    og = lattice_geometry(avec, *n)
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 13.0, (3, og.npts))
    plan = Plan(pcx_geometry(avec, *n), max_vectors=max(nvec, 1))
    plan.pcx_plan_set_eps(eps)
    y = S.random_block(seed, 2 * og.npts, nvec)
    return plan, og, eps, y


def _run(plan, og, eps, y, kappa, prec):
    import torch
    yd = _dev(y, prec)
    z_ref = torch.empty_like(yd)
    plan.pcx_apply_Ar(kappa, yd, z_ref)
    z = torch.full_like(yd, float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.pcx_apply_Ar_noalloc(kappa, yd, z)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    got = z.cpu().numpy().T.astype(np.complex128)
    ref = z_ref.cpu().numpy().T.astype(np.complex128)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= TOL[prec], err
    spec = spectrum(og, kappa)
    o = Ar_apply(spec, eps, y[:, 0])
    err_o = np.abs(got[:, 0] - o).max() / np.abs(o).max()
    assert err_o <= TOL[prec], err_o
    return err, err_o


def test_noalloc_matches_apply_Ar_two_calls_second_smaller():
    cases = [
        # fixed-size FP32 kernels (the adjoint without its W table), 8 vectors at 64^3
        (S.FCC, (64, 64, 64), (0.5, 0.0, 0.5), "fp32", 8, 1),
        # a smaller input right after: ragged triclinic grid, generic kernels, FP64
        (S.triclinic(1), (5, 4, 3), (0.11, -0.37, 0.42), "fp64", 2, 2),
        # FP64 at 64^3, then Gamma on a small grid (masked mode)
        (S.FCC, (64, 64, 64), (0.13, -0.41, 0.27), "fp64", 3, 3),
        (S.SC, (8, 8, 8), (0.0, 0.0, 0.0), "fp32", 1, 4),
    ]
    for avec, n, kappa, prec, nvec, seed in cases:
        say("noalloc", n, kappa, prec, nvec)
        plan, og, eps, y = _case(avec, n, kappa, prec, nvec, seed)
        err, err_o = _run(plan, og, eps, y, kappa, prec)
        say("noalloc", n, prec, "vs pcx_apply_Ar", err, "vs oracle", err_o)


def test_noalloc_refuses_a_block_beyond_the_scratch():
    import torch
    from paper_1806_10284_amd import Plan, pcx_geometry
    from paper_1806_10284_amd._lib import PcxError
    g = pcx_geometry(S.FCC, 64, 64, 64)
    plan = Plan(g, max_vectors=4)
    plan.pcx_plan_set_eps(np.full(3 * plan.n, 2.0))
    # FP64 at 64^3: 12.6 MB of workspace per vector, 10 fit in 128 MiB, 11 do not
    y = torch.zeros((11, 2 * plan.n), dtype=torch.complex128, device="cuda")
    z = torch.empty_like(y)
    say("noalloc refusal, 11 FP64 vectors at 64^3")
    with pytest.raises(PcxError, match="at most 10 vectors"):
        plan.pcx_apply_Ar_noalloc((0.5, 0.0, 0.5), y, z)
    torch.cuda.synchronize()
