"""The single-gyroid workload (Section 6: BCC lattice, level set of the sin-cos sum above 1.1,
eps swept from 3 to 30): the input generator and the properties the GPU sweep is checked
against at full size.

* the gyroid function is periodic on the BCC primitive cell and on no smaller FCC-type cell, and
  odd under inversion (so the fill of f > 1.1 equals that of f < -1.1);
* in vacuum (eps = 1 everywhere) the positive eigenvalues of C*C x = lambda x are the closed-form
  Lambda_q, each twice (the two transverse polarisations), against the explicit sparse curl;
* for B1 <= B2 (entrywise, diagonal) the k-th positive eigenvalue does not increase, and with
  1 <= eps <= eps_max it lies in [lambda_k(vacuum) / eps_max, lambda_k(vacuum)] (Courant-Fischer on
  the pencil; the nullspace of C*C does not depend on B, so positive eigenvalues pair up in
  order).
"""
from __future__ import annotations

import numpy as np

import pcx_synth as S
from oracle.geometry import kappa_from_bloch, lattice_geometry
from oracle.solve import dense_gep
from oracle.spectral import spectrum


def test_gyroid_function_is_bcc_periodic_and_odd():
    rng = np.random.default_rng(5)
    r = rng.uniform(-1.0, 1.0, (4000, 3))
    f = S.gyroid_function(r)
    for i in range(3):
        np.testing.assert_allclose(S.gyroid_function(r + S.BCC[:, i]), f, atol=1e-12)
    # an FCC translation (half a cube face diagonal) is not a symmetry
    assert np.abs(S.gyroid_function(r + S.FCC[:, 0]) - f).max() > 0.5
    np.testing.assert_allclose(S.gyroid_function(-r), -f, atol=1e-12)
    assert np.abs(f).max() <= 1.5 + 1e-12
    frac_hi = np.mean(S.gyroid_function(rng.uniform(0, 1, (200000, 3))) > S.GYROID_LEVEL)
    frac_lo = np.mean(S.gyroid_function(rng.uniform(0, 1, (200000, 3))) < -S.GYROID_LEVEL)
    assert 0.08 < frac_hi < 0.2 and abs(frac_hi - frac_lo) < 0.01


def test_gyroid_yee_sampling():
    n = (16, 16, 16)
    g = lattice_geometry(S.BCC, *n)
    e = S.gyroid_yee(n, g.shift, 13.0)
    assert e.shape == (3, g.npts)
    assert set(np.unique(e)) == {1.0, 13.0}
    # the three Yee sub-grids see nearly the same fill as the continuum level set
    fill = (e > 1.0).mean(axis=1)
    assert np.all(np.abs(fill - fill.mean()) < 0.02) and 0.08 < fill.mean() < 0.2
    # shifting the grid by one primitive vector is the same crystal: sample the first Yee
    # sub-grid at p + n1 e1 (one lattice vector away) directly
    r = S.grid_fractional(n, g.shift, S.YEE_OFFSETS[0]) @ S.BCC.T
    np.testing.assert_array_equal(S.gyroid_function(r + S.BCC[:, 0]) > S.GYROID_LEVEL, e[0] > 1.0)


def _vacuum_positive(geom, kappa, count):
    lq = np.sum(np.abs(spectrum(geom, kappa).lam) ** 2, axis=0).reshape(-1)
    lq = np.sort(lq[lq > 1e-12 * lq.max()])
    return np.repeat(lq, 2)[:count]


def test_vacuum_spectrum_is_doubled_lambda_q():
    n = (6, 6, 6)
    g = lattice_geometry(S.BCC, *n)
    for k in (S.BCC_POINTS["H"], S.BCC_POINTS["P"], np.array([0.4, -1.1, 0.7])):
        kappa = kappa_from_bloch(S.BCC, k)
        ref, _ = dense_gep(g, kappa, np.ones((3, g.npts)), 12)
        np.testing.assert_allclose(ref, _vacuum_positive(g, kappa, 12), rtol=1e-10)


def test_eps_sweep_monotone_and_bracketed():
    n = (6, 6, 6)
    g = lattice_geometry(S.BCC, *n)
    kappa = kappa_from_bloch(S.BCC, S.BCC_POINTS["N"])
    nev = 8
    vac = _vacuum_positive(g, kappa, nev)
    prev = None
    for eps_in in (3.0, 13.0, 30.0):
        lam, _ = dense_gep(g, kappa, S.gyroid_yee(n, g.shift, eps_in), nev)
        assert np.all(lam <= vac * (1 + 1e-10)) and np.all(lam >= vac / eps_in * (1 - 1e-10))
        if prev is not None:
            assert np.all(lam <= prev * (1 + 1e-10))
        prev = lam
