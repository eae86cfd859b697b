"""Path construction of the band-structure driver (Section 6: each segment between corner points cut
into equal parts, 10 in the paper)."""
from __future__ import annotations

import numpy as np
import pytest

import pcx_synth as S
from paper_1806_10284_amd.bands import kpath


def test_kpath_parts_and_arc_length():
    corners = np.array([S.BCC_POINTS[c] for c in "GHNGPH"])
    pts, arc = kpath(corners, 10)
    assert pts.shape == (51, 3) and arc.shape == (51,)
    np.testing.assert_allclose(pts[::10], corners, atol=1e-14)
    seg = np.linalg.norm(np.diff(corners, axis=0), axis=1)
    np.testing.assert_allclose(arc[::10], np.concatenate([[0.0], np.cumsum(seg)]), rtol=1e-14)
    # equal steps inside each segment, and the arc length is the distance walked
    for i in range(5):
        steps = np.linalg.norm(np.diff(pts[10 * i:10 * i + 11], axis=0), axis=1)
        np.testing.assert_allclose(steps, seg[i] / 10, rtol=1e-12)
    np.testing.assert_allclose(np.diff(arc), np.linalg.norm(np.diff(pts, axis=0), axis=1), rtol=1e-12)


def test_kpath_rejects_degenerate_paths():
    with pytest.raises(ValueError):
        kpath([S.SC_POINTS["G"]], 10)
    with pytest.raises(ValueError):
        kpath([S.SC_POINTS["G"], S.SC_POINTS["X"]], 0)
    with pytest.raises(ValueError):
        kpath([S.SC_POINTS["G"], S.SC_POINTS["X"], S.SC_POINTS["X"]], 4)


@pytest.mark.parametrize("name", ["SC", "FCC", "BCC", "HEX", "ORTHO"])
def test_corner_points_lie_on_the_brillouin_zone_boundary(name):
    """Every corner point k != Gamma is as close to some nonzero reciprocal lattice vector G as to
    Gamma (|k - G| = |k|, on the boundary of the first Brillouin zone) and no closer to any."""
    avec = getattr(S, name)
    pts = getattr(S, f"{name}_POINTS")
    B = 2 * np.pi * np.linalg.inv(avec)          # rows: reciprocal vectors, b_i . a_j = 2 pi delta_ij
    rng = np.arange(-2, 3)
    G = np.array([i * B[0] + j * B[1] + k * B[2] for i in rng for j in rng for k in rng
                  if (i, j, k) != (0, 0, 0)])
    for lab, k in pts.items():
        if lab == "G":
            assert np.all(k == 0)
            continue
        d = np.linalg.norm(k - G, axis=1)
        assert d.min() == pytest.approx(np.linalg.norm(k), rel=1e-12), (name, lab)


def test_band_structure_argument_checks():
    """Rejected before anything reaches the device: no plans, or a lattice count that matches
    neither one-for-all nor one-per-plan."""
    from paper_1806_10284_amd.bands import band_structure
    corners = [S.SC_POINTS["G"], S.SC_POINTS["X"]]
    with pytest.raises(ValueError):
        band_structure([], S.SC, corners)
    with pytest.raises(ValueError):
        band_structure([object(), object(), object()], [S.SC, S.FCC], corners)
