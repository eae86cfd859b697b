"""Seeded synthetic inputs for the photonic-crystal eigenproblem.

This module generates INPUTS only: lattice vectors, Bloch vectors, permittivity
arrays and random start vectors.  It holds none of the eigensolver's
arithmetic, and both the HIP library's tests/benchmarks and the CPU oracle
consume it.

Permittivity sampling needs to know where a grid point sits inside the unit
cell.  With the corrected lattice vectors written in grid units as rows
L1 = (n1, 0, 0), L2 = (s1, n2, 0), L3 = (s2, s3, n3) (the integer shifts s are
an input here; the caller computes them), a grid point p has fractional
coordinates f with p = f1 L1 + f2 L2 + f3 L3, and it is placed at the Cartesian
point a~ f of the user's lattice vectors a~ (columns of ``avec``).  Shapes are
spheres and finite cylinders ("rods") given in the user's Cartesian frame and
tested with periodic images.

Yee sampling (permittivity on the three edge-centred sub-grids):
    component 1 at (a + 1/2, b, c), component 2 at (a, b + 1/2, c),
    component 3 at (a, b, c + 1/2)
in the e-layout index a + n1 (b + n2 c).  "Voxel" permittivity is sampled at
the grid point (a, b, c) itself and shared by the three edges.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --------------------------------------------------------------------------
# lattices (columns are the primitive vectors, lattice constant a = 1)
# --------------------------------------------------------------------------

SC = np.eye(3)
FCC = 0.5 * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])   # columns (0,.5,.5),(.5,0,.5),(.5,.5,0)
BCC = 0.5 * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])
# hexagonal: a1 = (1,0,0), a2 = (-1/2, sqrt(3)/2, 0), a3 = (0, 0, 1.25)
HEX = np.array([[1.0, -0.5, 0.0], [0.0, math.sqrt(3.0) / 2.0, 0.0], [0.0, 0.0, 1.25]])
ORTHO = np.diag([1.5, 1.2, 1.0])


def triclinic(seed: int):
    """Seeded triclinic lattice: lengths U[0.8, 1.2], angles U[70, 110] degrees,
    the longest vector first; redrawn until the cell is admissible (the third
    vector's y offset stays inside the cell)."""
    rng = np.random.default_rng(seed)
    while True:
        L = np.sort(rng.uniform(0.8, 1.2, 3))[::-1]
        g, b, a = np.radians(rng.uniform(70.0, 110.0, 3))   # gamma(a1,a2) beta(a1,a3) alpha(a2,a3)
        cg, cb, ca = math.cos(g), math.cos(b), math.cos(a)
        sg = math.sin(g)
        a3y = (ca - cg * cb) / sg
        z2 = 1.0 - cb * cb - a3y * a3y
        if z2 <= 0.05:
            continue
        if L[2] * abs(a3y) >= 0.95 * L[1] * sg:
            continue
        avec = np.array([
            [L[0], L[1] * cg, L[2] * cb],
            [0.0, L[1] * sg, L[2] * a3y],
            [0.0, 0.0, L[2] * math.sqrt(z2)],
        ])
        return avec


# --------------------------------------------------------------------------
# Bloch vectors (Cartesian, units of 1/a; the Bloch vector is 2 pi k)
# --------------------------------------------------------------------------

TWO_PI = 2.0 * math.pi
FCC_POINTS = {
    "G": np.array([0.0, 0.0, 0.0]),
    "X": TWO_PI * np.array([0.0, 1.0, 0.0]),
    "W": TWO_PI * np.array([0.5, 1.0, 0.0]),
    "K": TWO_PI * np.array([0.75, 0.75, 0.0]),
    "L": TWO_PI * np.array([0.5, 0.5, 0.5]),
    "U": TWO_PI * np.array([0.25, 1.0, 0.25]),
}


# SC corner points (Cartesian, a = 1)
SC_POINTS = {
    "G": np.array([0.0, 0.0, 0.0]),
    "X": TWO_PI * np.array([0.0, 0.5, 0.0]),
    "M": TWO_PI * np.array([0.5, 0.5, 0.0]),
    "R": TWO_PI * np.array([0.5, 0.5, 0.5]),
}

# BCC corner points (Cartesian, cubic cell side a = 1)
BCC_POINTS = {
    "G": np.array([0.0, 0.0, 0.0]),
    "H": TWO_PI * np.array([0.0, 0.0, 1.0]),
    "N": TWO_PI * np.array([0.0, 0.5, 0.5]),
    "P": TWO_PI * np.array([0.5, 0.5, 0.5]),
}


def _hex_points():
    # reciprocal vectors of HEX (2 pi times the rows of HEX^-1); b1, b2 at 60 degrees
    b = TWO_PI * np.linalg.inv(HEX)
    b1, b2, b3 = b[0], b[1], b[2]
    m, k, a = 0.5 * b1, (b1 + b2) / 3.0, 0.5 * b3
    return {"G": np.zeros(3), "M": m, "K": k, "A": a, "L": m + a, "H": k + a}


def _ortho_points():
    # rectangular Brillouin zone of ORTHO: half reciprocal vectors and their sums
    b = TWO_PI * np.linalg.inv(ORTHO)
    x, y, z = 0.5 * b[0], 0.5 * b[1], 0.5 * b[2]
    return {"G": np.zeros(3), "X": x, "Y": y, "Z": z, "S": x + y, "U": x + z, "T": y + z, "R": x + y + z}


# primitive-orthorhombic corner points (Cartesian) for the lattice ORTHO
ORTHO_POINTS = _ortho_points()
# hexagonal corner points (Cartesian) for the lattice HEX
HEX_POINTS = _hex_points()


def fcc_path(npts: int, labels=("G", "X", "W", "K", "G", "L")) -> np.ndarray:
    """npts Bloch vectors spaced uniformly in arc length along the polyline, endpoints included."""
    corners = np.array([FCC_POINTS[c] for c in labels])
    seg = np.linalg.norm(np.diff(corners, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    s = np.linspace(0.0, cum[-1], npts)
    out = np.empty((npts, 3))
    for t, x in enumerate(s):
        i = min(np.searchsorted(cum, x, side="right") - 1, len(seg) - 1)
        u = (x - cum[i]) / seg[i]
        out[t] = corners[i] + u * (corners[i + 1] - corners[i])
    return out


def random_kappas(seed: int, count: int) -> np.ndarray:
    """Seeded reduced wave vectors kappa in (-1/2, 1/2]^3."""
    rng = np.random.default_rng(seed)
    return 0.5 - rng.uniform(0.0, 1.0, (count, 3))


# --------------------------------------------------------------------------
# grid points -> Cartesian positions in the user's frame
# --------------------------------------------------------------------------

def _grid_rows(n, shift):
    n1, n2, n3 = n
    s1, s2, s3 = shift
    return np.array([[n1, 0, 0], [s1, n2, 0], [s2, s3, n3]], dtype=np.float64)


def grid_fractional(n, shift, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Fractional lattice coordinates (n, 3) of the points (a, b, c) + offset, e-layout order."""
    n1, n2, n3 = n
    c, b, a = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    p = np.stack([a.ravel() + offset[0], b.ravel() + offset[1], c.ravel() + offset[2]], axis=1)
    M = _grid_rows(n, shift)
    return np.linalg.solve(M.T, p.T).T           # p = f M  <=>  M^T f^T = p^T


YEE_OFFSETS = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5))


@dataclass
class Sphere:
    center: np.ndarray
    radius: float


@dataclass
class Rod:
    p0: np.ndarray
    p1: np.ndarray
    radius: float


_IMAGES = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)], dtype=np.float64)


def _inside(avec, frac, shape, chunk=1 << 16) -> np.ndarray:
    """Boolean mask: which fractional points lie in the shape or a periodic image of it."""
    avec = np.asarray(avec, dtype=np.float64)
    inv = np.linalg.inv(avec)
    out = np.zeros(frac.shape[0], dtype=bool)
    if isinstance(shape, Sphere):
        ref = inv @ np.asarray(shape.center, dtype=np.float64)
    else:
        ref = inv @ np.asarray(shape.p0, dtype=np.float64)
        d = np.asarray(shape.p1, dtype=np.float64) - np.asarray(shape.p0, dtype=np.float64)
        dd = float(d @ d)
    # a sphere reaches at most radius * |row l of avec^-1| along fractional coordinate l, so a point
    # whose minimum-image fractional offset exceeds that in some l is outside every image
    half = shape.radius * np.linalg.norm(inv, axis=1) if isinstance(shape, Sphere) else None
    for s in range(0, frac.shape[0], chunk):
        df = frac[s:s + chunk] - ref
        df -= np.round(df)
        if half is not None:
            cand = np.all(np.abs(df) <= half + 1e-12, axis=1)
            if not cand.any():
                continue
            sub = np.zeros(df.shape[0], dtype=bool)
            sub[cand] = _sphere_images(df[cand], avec, shape.radius)
            out[s:s + chunk] = sub
            continue
        best = np.full(df.shape[0], np.inf)
        for img in _IMAGES:
            r = (df + img) @ avec.T            # Cartesian offset from the reference point
            if isinstance(shape, Sphere):
                dist2 = np.einsum("ij,ij->i", r, r)
            else:
                t = np.clip((r @ d) / dd, 0.0, 1.0)
                q = r - t[:, None] * d[None, :]
                dist2 = np.einsum("ij,ij->i", q, q)
            best = np.minimum(best, dist2)
        out[s:s + chunk] = best <= shape.radius ** 2
    return out


def _sphere_images(df, avec, radius):
    best = np.full(df.shape[0], np.inf)
    for img in _IMAGES:
        r = (df + img) @ avec.T
        best = np.minimum(best, np.einsum("ij,ij->i", r, r))
    return best <= radius ** 2


def sample_yee(avec, n, shift, shapes, eps_in: float, eps_out: float) -> np.ndarray:
    """Permittivity (3, n1 n2 n3) at the Yee points: eps_in inside any shape (closed set)."""
    npts = n[0] * n[1] * n[2]
    out = np.full((3, npts), eps_out, dtype=np.float64)
    for comp in range(3):
        frac = grid_fractional(n, shift, YEE_OFFSETS[comp])
        mask = np.zeros(npts, dtype=bool)
        for sh in shapes:
            mask |= _inside(avec, frac, sh)
        out[comp, mask] = eps_in
    return out


def sample_voxel(avec, n, shift, shapes, eps_in: float, eps_out: float) -> np.ndarray:
    """Permittivity (n1 n2 n3,) at the grid points."""
    npts = n[0] * n[1] * n[2]
    frac = grid_fractional(n, shift)
    mask = np.zeros(npts, dtype=bool)
    for sh in shapes:
        mask |= _inside(avec, frac, sh)
    out = np.full(npts, eps_out, dtype=np.float64)
    out[mask] = eps_in
    return out


def voxel_to_yee(eps_voxel: np.ndarray) -> np.ndarray:
    """Broadcast a voxel permittivity to the three Yee edges owned by each grid point."""
    e = np.asarray(eps_voxel, dtype=np.float64).reshape(-1)
    return np.stack([e, e, e])


# --------------------------------------------------------------------------
# the workloads' structures
# --------------------------------------------------------------------------

def sc_sphere_shapes():
    """One sphere r = 0.25 at the cell centre (simple cubic)."""
    return [Sphere(np.array([0.5, 0.5, 0.5]), 0.25)]


def diamond_shapes(r_sphere=0.12, r_rod=0.11):
    """Diamond structure on the FCC lattice: spheres at 0 and (1/4,1/4,1/4) and
    rods from (1/4,1/4,1/4) to its four nearest FCC lattice points."""
    b = np.array([0.25, 0.25, 0.25])
    shapes = [Sphere(np.zeros(3), r_sphere), Sphere(b, r_sphere)]
    for nb in (np.zeros(3), FCC[:, 0], FCC[:, 1], FCC[:, 2]):
        shapes.append(Rod(b, nb.copy(), r_rod))
    return shapes


def blob_shapes(avec, seed: int, count: int = 6):
    """Seeded spheres: centres uniform in the cell, radii U[0.1, 0.2] * V^{1/3}."""
    rng = np.random.default_rng(seed)
    vol = abs(np.linalg.det(avec))
    scale = vol ** (1.0 / 3.0)
    shapes = []
    for _ in range(count):
        f = rng.uniform(0.0, 1.0, 3)
        shapes.append(Sphere(np.asarray(avec) @ f, rng.uniform(0.1, 0.2) * scale))
    return shapes


def random_sphere_fill(avec, n, shift, seed: int, fill: float = 0.3,
                       rmin: float = 0.08, rmax: float = 0.15, eps_in=13.0, eps_out=1.0):
    """Add seeded random spheres until the fraction of eps_in voxels reaches ``fill``."""
    rng = np.random.default_rng(seed)
    npts = n[0] * n[1] * n[2]
    frac = grid_fractional(n, shift)
    mask = np.zeros(npts, dtype=bool)
    while mask.mean() < fill:
        f = rng.uniform(0.0, 1.0, 3)
        mask |= _inside(avec, frac, Sphere(np.asarray(avec) @ f, rng.uniform(rmin, rmax)))
    out = np.full(npts, eps_out)
    out[mask] = eps_in
    return out


GYROID_LEVEL = 1.1
GYROID_EPS_SWEEP = tuple(float(e) for e in np.linspace(3.0, 30.0, 10))   # 3, 6, ..., 30


def gyroid_function(r: np.ndarray) -> np.ndarray:
    """sin(2 pi x) cos(2 pi y) + sin(2 pi y) cos(2 pi z) + sin(2 pi z) cos(2 pi x) at Cartesian
    points r (m, 3), cubic cell side a = 1 (the single-gyroid level set of Section 6)."""
    t = 2.0 * math.pi * np.asarray(r, dtype=np.float64)
    s, c = np.sin(t), np.cos(t)
    return s[:, 0] * c[:, 1] + s[:, 1] * c[:, 2] + s[:, 2] * c[:, 0]


def gyroid_yee(n, shift, eps_in: float, eps_out: float = 1.0, level: float = GYROID_LEVEL,
               avec=None) -> np.ndarray:
    """Single gyroid on the BCC lattice (Section 6): eps_in at the Yee points where the gyroid
    function exceeds ``level``, eps_out elsewhere; (3, n1 n2 n3).  The function is unchanged by
    the BCC translations (each of x, y, z moved by 1/2 flips the sign of every sine and cosine),
    so it is periodic on the primitive cell of ``BCC``."""
    avec = BCC if avec is None else np.asarray(avec, dtype=np.float64)
    npts = n[0] * n[1] * n[2]
    out = np.full((3, npts), eps_out, dtype=np.float64)
    for comp in range(3):
        r = grid_fractional(n, shift, YEE_OFFSETS[comp]) @ avec.T
        out[comp, gyroid_function(r) > level] = eps_in
    return out


def _periodic_gauss(field3d: np.ndarray, sigma_vox: float) -> np.ndarray:
    """Periodic Gaussian blur (sigma in voxels) of a [c][b][a] array, by FFT convolution."""
    out = np.fft.fftn(field3d)
    for ax, size in enumerate(field3d.shape):
        f = np.fft.fftfreq(size)
        g = np.exp(-2.0 * (math.pi * sigma_vox * f) ** 2)
        shp = [1, 1, 1]
        shp[ax] = size
        out *= g.reshape(shp)
    return np.real(np.fft.ifftn(out))


def smooth_diamond_field(avec, n, shift, seed: int, eps_lo=1.0, eps_hi=13.0):
    """Per-voxel eps = lo + (hi - lo) clip(phi, 0, 1), with phi = blurred diamond
    indicator (sigma 1.5 voxels) + 0.15 * blurred seeded noise (sigma 3, unit std)."""
    rng = np.random.default_rng(seed)
    shape3 = (n[2], n[1], n[0])
    ind = sample_voxel(avec, n, shift, diamond_shapes(), 1.0, 0.0).reshape(shape3)
    phi = _periodic_gauss(ind, 1.5)
    noise = _periodic_gauss(rng.standard_normal(shape3), 3.0)
    noise /= noise.std()
    phi = phi + 0.15 * noise
    return eps_lo + (eps_hi - eps_lo) * np.clip(phi, 0.0, 1.0).reshape(-1)


def random_block(seed: int, rows: int, cols: int) -> np.ndarray:
    """Seeded complex Gaussian block (rows x cols), complex128, column-major by column index."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((cols, rows)) + 1j * rng.standard_normal((cols, rows))).T.copy()
