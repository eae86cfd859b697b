"""Shared helpers for the tests (random admissible lattices, comparisons)."""
from __future__ import annotations

import numpy as np


def random_lattice(rng, ang_lo=50.0, ang_hi=130.0):
    """A random lattice with |a1| the longest, randomly rotated (columns are vectors)."""
    while True:
        L = rng.uniform(0.8, 1.2, 3)
        L[0] = L.max() + 0.01
        g, b, a = np.radians(rng.uniform(ang_lo, ang_hi, 3))
        cg, cb, ca = np.cos([g, b, a])
        a3y = (ca - cg * cb) / np.sin(g)
        z2 = 1.0 - cb ** 2 - a3y ** 2
        if z2 <= 0.05:
            continue
        A = np.array([
            [L[0], L[1] * cg, L[2] * cb],
            [0.0, L[1] * np.sin(g), L[2] * a3y],
            [0.0, 0.0, L[2] * np.sqrt(z2)],
        ])
        R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        return R @ A


def random_geometry(rng, nlo=3, nhi=6, **kw):
    from oracle.geometry import LatticeError, lattice_geometry
    while True:
        A = random_lattice(rng, **kw)
        n = tuple(int(x) for x in rng.integers(nlo, nhi, 3))
        try:
            return A, lattice_geometry(A, *n)
        except LatticeError:
            continue


def sorted_triples(tx, ty, tz, decimals=8):
    z = np.stack([np.exp(2j * np.pi * np.asarray(t)).ravel() for t in (tx, ty, tz)], axis=1)
    v = np.round(np.concatenate([z.real, z.imag], axis=1), decimals) + 0.0
    return v[np.lexsort(v.T[::-1])]
