"""The Rayleigh-Ritz products of the block eigensolver (Section 5.2) through the C ABI
(pcx_block_gram, pcx_block_combine), against numpy on the same seeded columns.

Widths span every kernel path: the matrix-core Hermitian Gram kernel (up to 48 columns), its
tiled form over pairs of column groups (49-96 columns), the VALU kernels beyond and for the general
product; combinations up to 48 inputs and 32 outputs, up to 96 inputs with outputs in chunks of 32,
and the VALU kernel beyond.  Column length 40010 (ragged against the row chunks, stages and tiles);
an odd length in FP32 (columns not 16-byte aligned, a row pair straddling the end) takes the VALU
Gram kernel, which a case checks too.
Both kernels accumulate in FP64 from inputs in the storage precision, so the reference is the
FP64 product of the stored (for FP32: rounded) values, and the bound is a multiple of the unit
roundoff times |A|^H |B| entry by entry (FP32 outputs of the combination: plus their own rounding).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LEN = 40010


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def _plan():
    import pcx_synth as S
    from paper_1806_10284_amd import Plan, pcx_geometry
    return Plan(pcx_geometry(S.SC, 4, 4, 4), max_vectors=1)


def _cols(rng, k, prec, length=LEN):
    import torch
    a = rng.standard_normal((k, length)) + 1j * rng.standard_normal((k, length))
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    t = torch.from_numpy(a).to(dtype=dt, device="cuda").contiguous()
    return t, t.cpu().numpy().astype(np.complex128)      # the stored values


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ka,half", [(12, False), (36, True), (48, True), (60, False), (60, True), (90, True),
                                     (100, True)])
def test_block_gram_hermitian(ka, half, prec):
    rng = np.random.default_rng(1000 + ka + 7 * half)
    plan = _plan()
    import torch
    a, an = _cols(rng, ka, prec)
    b = bn = None
    if half:
        # A2 = A diag(d) along the columns' length (d real), so A^H A2 is Hermitian, as S^H A_r S is
        d = rng.uniform(0.5, 2.0, LEN)
        b = (a * torch.from_numpy(d).to(device="cuda", dtype=a.real.dtype)).contiguous()
        bn = b.cpu().numpy().astype(np.complex128)
    say("block gram herm", ka, "halves", 2 if half else 1, prec)
    g = plan.pcx_block_gram(a, b, herm=True)
    B = np.concatenate([an, bn]) if half else an
    ref = an.conj() @ B.T
    bound = 64 * 1.1e-16 * (np.abs(an) @ np.abs(B).T) + 1e-300
    # the kernels form the upper triangle of each ka x ka half; the lower one is its mirror and the
    # diagonal is taken real (A2 is rounded to the storage precision, so A^H A2 is Hermitian only
    # to that rounding: the strict upper triangle and the real diagonal are what is compared)
    iu = np.triu_indices(ka, 1)
    for h in range(2 if half else 1):
        sl = slice(h * ka, (h + 1) * ka)
        gh, rh, bh = g[:, sl], ref[:, sl], bound[:, sl]
        err = max(float((np.abs(gh[iu] - rh[iu]) / bh[iu]).max()),
                  float((np.abs(np.diag(gh).real - np.diag(rh).real) / np.diag(bh)).max()))
        say("  half", h, "max error / bound", err)
        assert err <= 1.0
        np.testing.assert_array_equal(gh.T[iu], gh[iu].conj())     # the mirrored lower triangle
        assert np.all(np.diag(gh).imag == 0.0)


def test_block_gram_odd_length_fp32():
    rng = np.random.default_rng(55)
    plan = _plan()
    a, an = _cols(rng, 20, "fp32", length=LEN - 1)
    say("block gram herm 20, odd length, fp32")
    g = plan.pcx_block_gram(a, None, herm=True)
    ref = an.conj() @ an.T
    assert np.all(np.abs(g - ref) <= 64 * 1.1e-16 * (np.abs(an) @ np.abs(an).T))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_block_gram_general(prec):
    rng = np.random.default_rng(77)
    plan = _plan()
    a, an = _cols(rng, 7, prec)
    b, bn = _cols(rng, 13, prec)
    say("block gram general 7 x 13", prec)
    g = plan.pcx_block_gram(a, b, herm=False)
    ref = an.conj() @ bn.T
    assert np.all(np.abs(g - ref) <= 64 * 1.1e-16 * (np.abs(an) @ np.abs(bn).T))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ks,m", [(12, 12), (36, 24), (48, 32), (60, 24), (60, 40), (90, 60), (100, 24)])
def test_block_combine(ks, m, prec):
    import torch
    rng = np.random.default_rng(2000 + ks * 7 + m)
    plan = _plan()
    s, sn = _cols(rng, ks, prec)
    c = rng.standard_normal((ks, m)) + 1j * rng.standard_normal((ks, m))
    y = torch.empty((m, LEN), dtype=s.dtype, device="cuda")
    say("block combine", ks, "->", m, prec)
    plan.pcx_block_combine(s, c, y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.complex128)
    ref = c.T @ sn
    bound = 64 * 1.1e-16 * (np.abs(c).T @ np.abs(sn))
    if prec == "fp32":
        bound = bound + 2.0 ** -23 * np.abs(ref)
    err = np.abs(got - ref) / (bound + 1e-300)
    say("  max error / bound", float(err.max()))
    assert np.all(err <= 1.0)
