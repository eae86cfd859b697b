"""The 14 Bravais lattices with the corner points of their irreducible Brillouin zones.

The paper computes band structures for all 14 lattices (Section 6) along paths through the corner
points of each irreducible Brillouin zone, tabulated in an appendix that is not part of the text.
The tables here follow the standard published convention for high-symmetry points (Setyawan and
Curtarolo, Comput. Mater. Sci. 49 (2010) 299): each point is given by its coordinates f in the
reciprocal basis b_i of the listed primitive vectors a_j (b_i . a_j = 2 pi delta_ij), so the
Cartesian Bloch vector is 2 pi k = sum_i f_i b_i.  For lattices whose point set depends on the
cell shape, one admissible shape is fixed (the variant is named).  Lattice constant a = 1.

Each entry: primitive vectors (columns, user frame), the corner points (Cartesian Bloch vectors)
and a continuous default path through them.  Input definitions only; no solver arithmetic.
"""
from __future__ import annotations

import math

import numpy as np


def _cols(*vs):
    return np.array(vs, dtype=np.float64).T


def _cart(avec, frac):
    """sum_i f_i b_i with the rows of 2 pi avec^-1 as the reciprocal vectors b_i."""
    B = 2.0 * math.pi * np.linalg.inv(avec)
    return {k: np.asarray(f, dtype=np.float64) @ B for k, f in frac.items()}


def _cubic():
    return _cols((1, 0, 0), (0, 1, 0), (0, 0, 1)), {
        "G": (0, 0, 0), "X": (0, 0.5, 0), "M": (0.5, 0.5, 0), "R": (0.5, 0.5, 0.5)}, "GXMGRX"


def _fcc():
    a = _cols((0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))
    return a, {"G": (0, 0, 0), "X": (0.5, 0, 0.5), "W": (0.5, 0.25, 0.75), "K": (0.375, 0.375, 0.75),
               "L": (0.5, 0.5, 0.5), "U": (0.625, 0.25, 0.625)}, "GXWKGLUWLK"


def _bcc():
    a = _cols((-0.5, 0.5, 0.5), (0.5, -0.5, 0.5), (0.5, 0.5, -0.5))
    return a, {"G": (0, 0, 0), "H": (0.5, -0.5, 0.5), "N": (0, 0, 0.5), "P": (0.25, 0.25, 0.25)}, "GHNGPH"


def _tet(c=1.4):
    return _cols((1, 0, 0), (0, 1, 0), (0, 0, c)), {
        "G": (0, 0, 0), "A": (0.5, 0.5, 0.5), "M": (0.5, 0.5, 0), "R": (0, 0.5, 0.5), "X": (0, 0.5, 0),
        "Z": (0, 0, 0.5)}, "GXMGZRAZ"


def _bct2(c=1.6):
    # body-centred tetragonal with c > a (variant BCT2)
    a = _cols((-0.5, 0.5, c / 2), (0.5, -0.5, c / 2), (0.5, 0.5, -c / 2))
    eta = (1 + 1 / c ** 2) / 4
    zeta = 1 / (2 * c ** 2)
    return a, {"G": (0, 0, 0), "N": (0, 0.5, 0), "P": (0.25, 0.25, 0.25), "S": (-eta, eta, eta),
               "S1": (eta, 1 - eta, -eta), "X": (0, 0, 0.5), "Y": (-zeta, zeta, 0.5), "Y1": (0.5, 0.5, -zeta),
               "Z": (0.5, 0.5, -0.5)}, ["G", "X", "Y", "S", "G", "Z", "S1", "N", "P", "Y1", "Z"]


def _orc(a=1.0, b=1.2, c=1.5):
    return _cols((a, 0, 0), (0, b, 0), (0, 0, c)), {
        "G": (0, 0, 0), "X": (0.5, 0, 0), "Y": (0, 0.5, 0), "Z": (0, 0, 0.5), "S": (0.5, 0.5, 0),
        "U": (0.5, 0, 0.5), "T": (0, 0.5, 0.5), "R": (0.5, 0.5, 0.5)}, "GXSYGZURTZ"


def _orcf1(a=1.0, b=1.3, c=1.7):
    # face-centred orthorhombic with 1/a^2 > 1/b^2 + 1/c^2 (variant ORCF1)
    av = _cols((0, b / 2, c / 2), (a / 2, 0, c / 2), (a / 2, b / 2, 0))
    zeta = (1 + a * a / (b * b) - a * a / (c * c)) / 4
    eta = (1 + a * a / (b * b) + a * a / (c * c)) / 4
    return av, {"G": (0, 0, 0), "A": (0.5, 0.5 + zeta, zeta), "A1": (0.5, 0.5 - zeta, 1 - zeta),
                "L": (0.5, 0.5, 0.5), "T": (1, 0.5, 0.5), "X": (0, eta, eta), "X1": (1, 1 - eta, 1 - eta),
                "Y": (0.5, 0, 0.5), "Z": (0.5, 0.5, 0)}, ["G", "Y", "T", "Z", "G", "X", "A1", "Y"]


def _orci(a=1.0, b=1.3, c=1.7):
    av = _cols((-a / 2, b / 2, c / 2), (a / 2, -b / 2, c / 2), (a / 2, b / 2, -c / 2))
    zeta = (1 + a * a / (c * c)) / 4
    eta = (1 + b * b / (c * c)) / 4
    delta = (b * b - a * a) / (4 * c * c)
    mu = (a * a + b * b) / (4 * c * c)
    return av, {"G": (0, 0, 0), "L": (-mu, mu, 0.5 - delta), "L1": (mu, -mu, 0.5 + delta),
                "L2": (0.5 - delta, 0.5 + delta, -mu), "R": (0, 0.5, 0), "S": (0.5, 0, 0), "T": (0, 0, 0.5),
                "W": (0.25, 0.25, 0.25), "X": (-zeta, zeta, zeta), "X1": (zeta, 1 - zeta, -zeta),
                "Y": (eta, -eta, eta), "Y1": (1 - eta, eta, -eta), "Z": (0.5, 0.5, -0.5)}, \
        ["G", "X", "L", "T", "W", "R", "X1", "Z", "G", "Y", "S", "W"]


def _orcc(a=1.0, b=1.4, c=1.2):
    av = _cols((a / 2, -b / 2, 0), (a / 2, b / 2, 0), (0, 0, c))
    zeta = (1 + a * a / (b * b)) / 4
    return av, {"G": (0, 0, 0), "A": (zeta, zeta, 0.5), "A1": (-zeta, 1 - zeta, 0.5), "R": (0, 0.5, 0.5),
                "S": (0, 0.5, 0), "T": (-0.5, 0.5, 0.5), "X": (zeta, zeta, 0), "X1": (-zeta, 1 - zeta, 0),
                "Y": (-0.5, 0.5, 0), "Z": (0, 0, 0.5)}, ["G", "X", "S", "R", "A", "Z", "G", "Y", "X1", "A1", "T", "Y"]


def _hex(c=1.25):
    av = _cols((1, 0, 0), (-0.5, math.sqrt(3) / 2, 0), (0, 0, c))
    # with a2 at 120 degrees from a1, b1 and b2 are 60 degrees apart: M = b1 / 2, K = (b1 + b2) / 3
    return av, {"G": (0, 0, 0), "M": (0.5, 0, 0), "K": (1 / 3, 1 / 3, 0), "A": (0, 0, 0.5),
                "L": (0.5, 0, 0.5), "H": (1 / 3, 1 / 3, 0.5)}, "GMKGALHA"


def _rhl1(alpha_deg=70.0):
    al = math.radians(alpha_deg)
    ch = math.cos(al / 2)
    av = _cols((ch, -math.sin(al / 2), 0), (ch, math.sin(al / 2), 0),
               (math.cos(al) / ch, 0, math.sqrt(1 - math.cos(al) ** 2 / ch ** 2)))
    eta = (1 + 4 * math.cos(al)) / (2 + 4 * math.cos(al))
    nu = 0.75 - eta / 2
    return av, {"G": (0, 0, 0), "B": (eta, 0.5, 1 - eta), "B1": (0.5, 1 - eta, eta - 1), "F": (0.5, 0.5, 0),
                "L": (0.5, 0, 0), "L1": (0, 0, -0.5), "P": (eta, nu, nu), "P1": (1 - nu, 1 - nu, 1 - eta),
                "P2": (nu, nu, eta - 1), "Q": (1 - nu, nu, 0), "X": (nu, 0, -nu), "Z": (0.5, 0.5, 0.5)}, \
        ["G", "L", "B1", "B", "Z", "G", "X", "Q", "F", "P1", "Z"]


def _mcl(b=1.1, c=1.3, alpha_deg=75.0):
    al = math.radians(alpha_deg)
    av = _cols((1, 0, 0), (0, b, 0), (0, c * math.cos(al), c * math.sin(al)))
    eta = (1 - b * math.cos(al) / c) / (2 * math.sin(al) ** 2)
    nu = 0.5 - eta * c * math.cos(al) / b
    return av, {"G": (0, 0, 0), "A": (0.5, 0.5, 0), "C": (0, 0.5, 0.5), "D": (0.5, 0, 0.5),
                "D1": (0.5, 0, -0.5), "E": (0.5, 0.5, 0.5), "H": (0, eta, 1 - nu), "H1": (0, 1 - eta, nu),
                "H2": (0, eta, -nu), "M": (0.5, eta, 1 - nu), "M1": (0.5, 1 - eta, nu), "M2": (0.5, eta, -nu),
                "X": (0, 0.5, 0), "Y": (0, 0, 0.5), "Y1": (0, 0, -0.5), "Z": (0.5, 0, 0)}, \
        ["G", "Y", "H", "C", "E", "M1", "A", "X", "H1"]


def _mclc1(b=1.2, c=1.4, alpha_deg=75.0):
    # base-centred monoclinic whose reciprocal angle k_gamma exceeds 90 degrees (variant MCLC1)
    al = math.radians(alpha_deg)
    av = _cols((0.5, b / 2, 0), (-0.5, b / 2, 0), (0, c * math.cos(al), c * math.sin(al)))
    zeta = (2 - b * math.cos(al) / c) / (4 * math.sin(al) ** 2)
    eta = 0.5 + 2 * zeta * c * math.cos(al) / b
    psi = 0.75 - 1 / (4 * b * b * math.sin(al) ** 2)
    phi = psi + (0.75 - psi) * b * math.cos(al) / c
    return av, {"G": (0, 0, 0), "N": (0.5, 0, 0), "N1": (0, -0.5, 0), "F": (1 - zeta, 1 - zeta, 1 - eta),
                "F1": (zeta, zeta, eta), "F2": (-zeta, -zeta, 1 - eta), "I": (phi, 1 - phi, 0.5),
                "I1": (1 - phi, phi - 1, 0.5), "L": (0.5, 0.5, 0.5), "M": (0.5, 0, 0.5),
                "X": (1 - psi, psi - 1, 0), "X1": (psi, 1 - psi, 0), "X2": (psi - 1, -psi, 0), "Y": (0.5, 0.5, 0),
                "Y1": (-0.5, -0.5, 0), "Z": (0, 0, 0.5)}, ["G", "Y", "F", "L", "I"]


def _tri1a(lengths=(1.0, 1.1, 0.95), angles_deg=(80.0, 76.0, 84.0)):
    # triclinic with every reciprocal angle above 90 degrees (variant TRI1a); angles are
    # (gamma = <a1, a2>, beta = <a1, a3>, alpha = <a2, a3>)
    la, lb, lc = lengths
    g, b, a = (math.radians(x) for x in angles_deg)
    a3y = (math.cos(a) - math.cos(g) * math.cos(b)) / math.sin(g)
    av = _cols((la, 0, 0), (lb * math.cos(g), lb * math.sin(g), 0),
               (lc * math.cos(b), lc * a3y, lc * math.sqrt(1 - math.cos(b) ** 2 - a3y ** 2)))
    return av, {"G": (0, 0, 0), "L": (0.5, 0.5, 0), "M": (0, 0.5, 0.5), "N": (0.5, 0, 0.5),
                "R": (0.5, 0.5, 0.5), "X": (0.5, 0, 0), "Y": (0, 0.5, 0), "Z": (0, 0, 0.5)}, \
        ["X", "G", "Y", "L", "G", "Z", "N", "G", "M", "R", "G"]


_BUILDERS = {
    "CUB": _cubic, "FCC": _fcc, "BCC": _bcc, "TET": _tet, "BCT": _bct2, "ORC": _orc, "ORCF": _orcf1,
    "ORCI": _orci, "ORCC": _orcc, "HEX": _hex, "RHL": _rhl1, "MCL": _mcl, "MCLC": _mclc1, "TRI": _tri1a,
}

BRAVAIS_NAMES = tuple(_BUILDERS)


def bravais(name: str):
    """(avec columns, {label: Cartesian Bloch vector}, [default path labels]) of lattice `name`."""
    avec, frac, path = _BUILDERS[name]()
    return avec, _cart(avec, frac), list(path)


def bravais_fractions(name: str):
    """The corner points as coordinates in the reciprocal basis (for the tests)."""
    _, frac, _ = _BUILDERS[name]()
    return {k: np.asarray(v, dtype=np.float64) for k, v in frac.items()}
