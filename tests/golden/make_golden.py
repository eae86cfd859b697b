"""Writes the stored expected eigenvalues under tests/golden/ from the FP64 oracle only.

Usage:  python tests/golden/make_golden.py [config1] [--dense] [fcc_small] [config2]

config1_sc16.json : simple cubic a = 1, grid 16^3, kappa = (1/4, 0, 0) (Bloch vector
                    (pi/2, 0, 0)), eps = 13 in the sphere r = 0.25 at the cell centre
                    (sampled at the Yee points), 1 elsewhere; the 10 smallest positive
                    eigenvalues of C*C x = lambda B x.  Sparse shift-invert solve; with
                    --dense also the dense eigh of the 12288 x 12288 pencil, which must agree.
fcc_diamond_<m>.json : FCC lattice with the diamond structure (spheres r = 0.12a at the two
                    basis sites, rods r = 0.11a to the four nearest neighbours, eps 13 in air,
                    sampled at the Yee points), grid m^3 (the largest the sparse factorisation
                    handles here), X point, 10 bands: sparse shift-invert solve with the explicit
                    curl, cross-checked with the inverse-Lanczos solve on the FFT operator.
config2_fcc64.json : the same structure at 64^3, X point, 10 bands, by the method of Section 5.2
                    (Lanczos on A_r^{-1}, unpreconditioned CG inner solves, tolerances 1e-12 /
                    1e-13), with the FFT residual of every band, the number of A_r applications
                    and the wall time on this host.
"""
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pcx_synth as S  # noqa: E402
from oracle.geometry import kappa_from_bloch, lattice_geometry  # noqa: E402
from oracle.solve import (dense_gep, nfsep_inverse_lanczos, nfsep_residuals, residuals,  # noqa: E402
                          sparse_gep)
from oracle.spectral import spectrum  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FCC_SMALL = 16


def config1():
    g = lattice_geometry(S.SC, 16, 16, 16)
    kap = kappa_from_bloch(S.SC, np.array([np.pi / 2, 0.0, 0.0]))
    eps = S.sample_yee(S.SC, g.n, g.shift, S.sc_sphere_shapes(), 13.0, 1.0)
    return g, kap, eps


def fcc_diamond(m):
    g = lattice_geometry(S.FCC, m, m, m)
    kap = kappa_from_bloch(S.FCC, S.FCC_POINTS["X"])
    eps = S.sample_yee(S.FCC, g.n, g.shift, S.diamond_shapes(), 13.0, 1.0)
    return g, kap, eps


def host_info():
    model = platform.processor() or ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count()}


def write(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def make_config1(dense):
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
    write("config1_sc16.json", out)


def make_fcc_small(m=FCC_SMALL):
    g, kap, eps = fcc_diamond(m)
    t = time.time()
    w, X = sparse_gep(g, kap, eps, 10)
    ts = time.time() - t
    res = residuals(g, kap, eps, w, X)
    spec = spectrum(g, kap)
    t = time.time()
    wl, _, info = nfsep_inverse_lanczos(spec, eps, 10)
    tl = time.time() - t
    out = {"config": f"FCC diamond {m}^3 (spheres r=0.12a, rods r=0.11a, eps 13/1 at Yee points), X point",
           "grid": [m, m, m], "kappa": list(map(float, kap)), "nev": 10,
           "lambda": [float(x) for x in w], "sparse_seconds": ts, "max_rel_residual": float(res.max()),
           "inverse_lanczos_vs_sparse_max_rel": float(np.max(np.abs(wl - w) / w)),
           "inverse_lanczos_seconds": tl, "inverse_lanczos_ar_applications": info["ar_applications"],
           "eps_inside_count": [int(np.sum(e > 1)) for e in eps], "host": host_info()}
    write(f"fcc_diamond_{m}.json", out)


def make_config2():
    g, kap, eps = fcc_diamond(64)
    spec = spectrum(g, kap)
    t = time.time()
    w, Y, info = nfsep_inverse_lanczos(spec, eps, 10)
    tl = time.time() - t
    res = nfsep_residuals(spec, eps, w, Y)
    out = {"config": "FCC diamond 64^3 (spheres r=0.12a, rods r=0.11a, eps 13/1 at Yee points), X point",
           "grid": [64, 64, 64], "kappa": list(map(float, kap)), "nev": 10,
           "method": "Lanczos on A_r^{-1} (scipy eigsh, tol 1e-12), CG inner solves (rtol 1e-13), FFT operator",
           "lambda": [float(x) for x in w], "rel_residual_fft": [float(x) for x in res],
           "seconds": tl, "ar_applications": info["ar_applications"], "cg_iterations": info["cg_iterations"],
           "inner_solves": info["inner_solves"], "threads": "numpy FFT, single-threaded",
           "eps_inside_count": [int(np.sum(e > 1)) for e in eps], "host": host_info()}
    write("config2_fcc64.json", out)


def main():
    args = sys.argv[1:] or ["config1"]
    if "config1" in args or "--dense" in args:
        make_config1("--dense" in args)
    if "fcc_small" in args:
        make_fcc_small()
    if "config2" in args:
        make_config2()


if __name__ == "__main__":
    main()
