"""Host-only checks of libpcx.so: it loads, exports every symbol include/pcx.h declares,
and its lattice geometry (Section 2.2) matches the oracle's exactly.  No device calls."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

import pcx_synth as S
from oracle.geometry import LatticeError, lattice_geometry

from .helpers import random_lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1806_10284_amd", "libpcx.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libpcx.so not built")


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "pcx.h")).read()
    return sorted(set(re.findall(r"\b(pcx_[a-z_A-Z]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    from paper_1806_10284_amd import _lib
    lib = _lib.load()
    declared = header_symbols()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTED) == declared


def _check_same(avec, n):
    from paper_1806_10284_amd import api
    try:
        og = lattice_geometry(avec, *n)
    except LatticeError:
        with pytest.raises(Exception):
            api.pcx_geometry(avec, *n)
        return None
    g = api.geom_dict(api.pcx_geometry(avec, *n))
    assert g["m"] == og.m and g["rho"] == og.rho and g["shift"] == tuple(int(x) for x in og.shift)
    np.testing.assert_allclose(g["delta"], og.delta, rtol=1e-14)
    np.testing.assert_allclose(g["avec_rot"], og.avec_rot, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(g["cos_angles"], og.cos_angles, rtol=1e-13, atol=1e-15)
    return g


@pytest.mark.parametrize("name,avec,n", [
    ("sc16", S.SC, (16, 16, 16)), ("fcc64", S.FCC, (64, 64, 64)), ("bcc48", S.BCC, (48, 48, 48)),
    ("hex", S.HEX, (32, 32, 40)), ("ortho", S.ORTHO, (60, 48, 40)), ("tri128", S.triclinic(5), (128, 128, 128)),
    ("fcc66", S.FCC, (60, 60, 60)),
])
def test_geometry_matches_oracle_workloads(name, avec, n):
    assert _check_same(avec, n) is not None


@pytest.mark.parametrize("seed", range(40))
def test_geometry_matches_oracle_random(seed):
    rng = np.random.default_rng(500 + seed)
    A = random_lattice(rng)
    n = tuple(int(x) for x in rng.choice([2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16, 20, 24], 3))
    _check_same(A, n)


def test_kappa_from_bloch_matches_oracle():
    from oracle.geometry import kappa_from_bloch
    from paper_1806_10284_amd import api
    for avec in (S.FCC, S.BCC, S.HEX, S.triclinic(3)):
        for k in S.fcc_path(7):
            a = api.pcx_kappa_from_bloch(avec, k)
            b = kappa_from_bloch(avec, k)
            assert np.array_equal(a, b)


def test_geometry_errors():
    from paper_1806_10284_amd import _lib, api
    with pytest.raises(_lib.PcxError) as e:
        api.pcx_geometry(S.SC, 7, 8, 8)          # 7 is not 2,3,5-smooth
    assert e.value.code == _lib.PCX_E_SIZE
    with pytest.raises(_lib.PcxError) as e:
        api.pcx_geometry(S.SC, 512, 8, 8)        # beyond PCX_MAX_N
    assert e.value.code == _lib.PCX_E_SIZE
    with pytest.raises(_lib.PcxError) as e:
        api.pcx_geometry(np.array([[1, 1, 0], [0, 0, 0], [0, 0, 1.0]]), 4, 4, 4)
    assert e.value.code == _lib.PCX_E_LATTICE
    with pytest.raises(_lib.PcxError) as e:
        api.pcx_geometry(S.SC, 0, 4, 4)
    assert e.value.code == _lib.PCX_E_ARG
    with pytest.raises(_lib.PcxError) as e:
        api.pcx_geometry(np.array([[1, 2.5, 0], [0, 1, 0], [0, 0, 1.0]]), 4, 4, 4)
    assert e.value.code == _lib.PCX_E_LATTICE


def test_preconditioner_codes():
    from paper_1806_10284_amd import PCX_PRECOND_DIAG, PCX_PRECOND_INVERSE, PCX_PRECOND_NONE, api
    assert api._precond(True) == PCX_PRECOND_INVERSE and api._precond(False) == PCX_PRECOND_NONE
    assert api._precond(PCX_PRECOND_DIAG) == 1
    with pytest.raises(ValueError):
        api._precond(3)
