"""Writes the stored expected eigenvalues under tests/golden/ from the FP64 oracle only.

Usage:  python tests/golden/make_golden.py [--dense]

config1_sc16.json : simple cubic a = 1, grid 16^3, kappa = (1/4, 0, 0) (Bloch vector
                    (pi/2, 0, 0)), eps = 13 in the sphere r = 0.25 at the cell centre
                    (sampled at the Yee points), 1 elsewhere; the 10 smallest positive
                    eigenvalues of C*C x = lambda B x.  Sparse shift-invert solve; with
                    --dense also the dense eigh of the 12288 x 12288 pencil, which must agree.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pcx_synth as S  # noqa: E402
from oracle.geometry import kappa_from_bloch, lattice_geometry  # noqa: E402
from oracle.solve import dense_gep, residuals, sparse_gep  # noqa: E402


def config1():
    g = lattice_geometry(S.SC, 16, 16, 16)
    kap = kappa_from_bloch(S.SC, np.array([np.pi / 2, 0.0, 0.0]))
    eps = S.sample_yee(S.SC, g.n, g.shift, S.sc_sphere_shapes(), 13.0, 1.0)
    return g, kap, eps


def main():
    dense = "--dense" in sys.argv
    g, kap, eps = config1()
    t = time.time()
    w, X = sparse_gep(g, kap, eps, 10)
    ts = time.time() - t
    res = residuals(g, kap, eps, w, X)
    out = {"config": "SC 16^3, kappa=(1/4,0,0), sphere r=0.25 eps=13 at Yee points",
           "kappa": list(map(float, kap)), "nev": 10,
           "lambda": [float(x) for x in w], "sparse_seconds": ts,
           "max_rel_residual": float(res.max()),
           "eps_inside_count": [int(np.sum(e > 1)) for e in eps]}
    if dense:
        t = time.time()
        wd, _ = dense_gep(g, kap, eps, 10)
        out["dense_seconds"] = time.time() - t
        out["dense_vs_sparse_max_rel"] = float(np.max(np.abs(wd - w) / wd))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_sc16.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
