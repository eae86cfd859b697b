"""Band structures along a path of Brillouin-zone corner points (Section 6).

Each segment between two consecutive corner points is cut into ``parts`` equal parts (the paper
uses 10), so a path through c corners has (c - 1) * parts + 1 wave vectors; each is one GEP
(Section 5.2), and the wave vectors of every plan (several lattices, or one geometry with several
permittivities) go to the device as one ``pcx_solve_batch`` request.  The horizontal axis of a
band diagram is the arc length of the path in Bloch-vector units, the vertical axis the
frequency omega = sqrt(lambda) / (2 pi).

Only the path construction and the bookkeeping live here; every solve runs in libpcx.so.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import _lib as L
from .api import pcx_kappa_from_bloch, pcx_omega, pcx_solve_batch


def kpath(corners, parts: int = 10):
    """Bloch vectors (Cartesian, (c - 1) * parts + 1 rows) along the polyline through ``corners``,
    each segment cut into ``parts`` equal parts, endpoints included once; and the arc length at each
    point.  A zero-length segment is rejected."""
    c = np.asarray(corners, dtype=np.float64).reshape(-1, 3)
    if c.shape[0] < 2 or parts < 1:
        raise ValueError("a path needs at least two corner points and parts >= 1")
    seg = np.linalg.norm(np.diff(c, axis=0), axis=1)
    if np.any(seg == 0.0):
        raise ValueError("repeated consecutive corner point")
    base = np.concatenate([[0.0], np.cumsum(seg)])
    pts, arc = [c[0]], [0.0]
    for i in range(c.shape[0] - 1):
        for t in range(1, parts + 1):
            u = t / parts
            pts.append(c[i] + u * (c[i + 1] - c[i]))
            arc.append(base[i] + u * seg[i])
    return np.array(pts), np.array(arc)


@dataclass
class BandStructure:
    kvecs: np.ndarray       # (npts, 3) Bloch vectors 2 pi k
    arc: np.ndarray         # (npts,) arc length along the path
    kappas: np.ndarray      # (nplans, npts, 3) phases kappa_l = k . a_l per plan's lattice
    lam: np.ndarray         # (nplans, npts, nev) smallest positive eigenvalues, ascending
    stats: list             # SolveStats per problem, plan-major

    @property
    def omega(self) -> np.ndarray:
        """Frequencies sqrt(lambda) / (2 pi)."""
        return np.sqrt(np.maximum(self.lam, 0.0)) / (2.0 * np.pi)


def band_structure(plans, avecs, corners, nev: int = 10, parts: int = 10, *, mode=L.PCX_MODE_FP32_REFINE,
                   tol: float = 1e-9, nworkers: int = 0, warm_start: bool = False, **solve_kw) -> BandStructure:
    """The ``nev`` smallest positive eigenvalues at every point of ``kpath(corners, parts)`` for each
    plan (its permittivity already set).  ``avecs``: the lattice vectors (columns) of each plan, or
    one 3x3 array shared by all; the Bloch vectors are mapped to each plan's phases with
    ``pcx_kappa_from_bloch``.  By default all problems are solved as one batch; with
    ``warm_start`` each plan's path is walked point by point, every solve starting from the
    previous point's eigenvectors (neighbouring wave vectors have nearby eigenspaces)."""
    plans = list(plans)
    if not plans:
        raise ValueError("no plans")
    av = np.asarray(avecs, dtype=np.float64)
    avs = [av] * len(plans) if av.ndim == 2 else list(av)
    if len(avs) != len(plans):
        raise ValueError("one lattice per plan, or one for all")
    kvecs, arc = kpath(corners, parts)
    kappas = np.array([[pcx_kappa_from_bloch(a, k) for k in kvecs] for a in avs])
    if warm_start:
        lam = np.zeros((len(plans), len(kvecs), nev))
        stats = []
        for q, (p, kap) in enumerate(zip(plans, kappas)):
            y = None
            for t, k in enumerate(kap):
                lam[q, t], y, _, st = p.pcx_solve(tuple(k), nev, mode=mode, tol=tol, want_y=True, y0=y, **solve_kw)
                stats.append(st)
        return BandStructure(kvecs, arc, kappas, lam, stats)
    problems = [(p, [tuple(k) for k in kap]) for p, kap in zip(plans, kappas)]
    lam, _, stats = pcx_solve_batch(problems, nev, mode=mode, tol=tol, nworkers=nworkers, **solve_kw)
    return BandStructure(kvecs, arc, kappas, lam.reshape(len(plans), len(kvecs), nev), stats)


def rotated_bloch_vectors(avec, geom, kvecs) -> np.ndarray:
    """Section 2.3: the Bloch vectors ``kvecs`` (user frame, rows) in the frame of the rotated,
    angle-corrected lattice ``geom``, Omega k; their phases with the corrected vectors equal
    those of ``kvecs`` with the user's vectors."""
    om = pcx_omega(avec, geom)
    return np.asarray(kvecs, dtype=np.float64).reshape(-1, 3) @ om.T
