#!/usr/bin/env python3
"""Benchmark: nullspace-free matvecs/s, HBM GB/s against the MI355X peak, and seconds per k-point.

Workload: FCC lattice with the diamond structure (dielectric spheres r = 0.12a at the two basis
sites joined by rods r = 0.11a, eps 13 in air), grid 64^3 (n = 262144, A_r of dimension 2n),
one wave vector at the X point, the 10 smallest positive eigenvalues, FP32 matvecs with FP64
refinement (the default mode; --mode fp64 runs the plain FP64 path).  Synthetic, seeded input;
everything is resident on the device before the timed region.

One step = one complete k-point solve (pcx_solve): LOBPCG iterations (A_r block matvecs, the
approximate-inverse preconditioner, FP64 Gram products, host Rayleigh-Ritz), refinement and the
eigenvalues on the host.

Printed (one JSON line): value = single-vector A_r applications per second over the timed solves
(the approximate-inverse preconditioner runs the same kernels with eps in place of 1/eps; its
applications are listed separately under "solve"), s_per_kpoint, the final relative residual of
every band and the bands (if any) accepted at the absolute residual floor; the roofline of the
dominant matvec kernel measured with HIP events on a 32-vector block (working set ~ 450 MB, larger
than the 256 MB last-level cache); and the FP64 CPU oracle's matvec rate on this host's cores,
with its estimated seconds per k-point, as a reference.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--mode fp32_refine|fp64|fp32]
                    [--no-cpu-baseline] [--profile-kernels]
                    [--workload fcc_diamond|gyroid_sweep|gyroid_bands|triclinic128]

--workload gyroid_sweep times the single-gyroid permittivity sweep of Section 6 instead (BCC 64^3,
eps 3..30, one plan per eps, all ten solved as one batch at the N point); its roofline block runs
on the eps = 12 plan.  --workload gyroid_bands solves the same ten plans along G-H-N-G-P-H with 10
parts per segment (510 problems per step; run it with --steps 1 --warmup 0).  --workload
triclinic128 solves the largest configuration, a seeded triclinic lattice at 128^3 with 20 bands at
16 wave vectors as one batch (about 26 s per step; --steps 1 --warmup 0), its roofline block on 8
vectors.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_GRID = (64, 64, 64)
NEV = 10
ROOF_VECTORS = 32
ROOF_WARMUP_S = 0.2      # seconds of back-to-back applications before the roofline timing


def kernel_bytes_per_vector(n: int, fp64: bool) -> dict:
    """Algorithmic HBM bytes per vector for each of the three A_r kernels (complex c, real r):
    plane forward reads y (2c) writes t (3c); x-line reads t (3c) and 1/eps (3r) and writes t (3c);
    plane adjoint reads t (3c) writes z (2c).  Total 16c + 3r per point."""
    c = 16 if fp64 else 8
    r = 8 if fp64 else 4
    return {"plane_fwd": 5 * c * n, "xline": 6 * c * n + 3 * r * n, "plane_adj": 5 * c * n}


KERNEL_SOURCES = ("pcx_fft.hip", "pcx_fixed.hip", "pcx_wave.hip", "pcx_dev.h", "pcx_internal.h")


def kernel_source_hash() -> str:
    """Digest of the matvec kernel sources; counter summaries taken on other sources are not used."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_10284_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# kernel-name prefix in a rocprofv3 trace -> (A_r kernel, precision)
KERNEL_KEYS = [
    ("pcx::k_w64_fwd<float", "plane_fwd_fp32"), ("pcx::k_w64_adj<float", "plane_adj_fp32"),
    ("pcx::k_p2_fwd<float", "plane_fwd_fp32"), ("pcx::k_p2_fwd<double", "plane_fwd_fp64"),
    ("pcx::k_p2_adj<float", "plane_adj_fp32"), ("pcx::k_p2_adj<double", "plane_adj_fp64"),
    ("pcx::k_p3_fwd<float", "plane_fwd_fp32"), ("pcx::k_p3_fwd<double", "plane_fwd_fp64"),
    ("pcx::k_plane_fwd<float", "plane_fwd_fp32"), ("pcx::k_plane_fwd<double", "plane_fwd_fp64"),
    ("pcx::k_p3_adj<float", "plane_adj_fp32"), ("pcx::k_p3_adj<double", "plane_adj_fp64"),
    ("pcx::k_plane_adj<float", "plane_adj_fp32"), ("pcx::k_plane_adj<double", "plane_adj_fp64"),
    ("pcx::k_xl_fixed<float", "xline_fp32"), ("pcx::k_xl_fixed<double", "xline_fp64"),
    ("pcx::k_xline<float", "xline_fp32"), ("pcx::k_xline<double", "xline_fp64"),
]


def summarize_traffic(fetch_csv: str, write_csv: str, out_json: str):
    """Per-dispatch HBM bytes of the A_r kernels from two rocprofv3 --pmc runs of
    `bench.py --profile-kernels` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by
    what the same counter reads for the 512 MiB calibration copy of that run."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        acc = defaultdict(list)
        copy = []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            name = r["Kernel_Name"]
            key = next((k for p, k in KERNEL_KEYS if name.startswith("void " + p) or name.startswith(p)), None)
            if key:
                acc[key].append(v)
            elif "copy" in name.lower() or "elementwise" in name.lower():
                copy.append(v)
        return {k: sum(v) / len(v) for k, v in acc.items()}, (max(copy) if copy else None)

    fetch, fcopy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_kernel(write_csv, "WRITE_SIZE")
    copy_kib = 512 * 1024
    cal_f = copy_kib / fcopy if fcopy else 1.0
    cal_w = copy_kib / wcopy if wcopy else 1.0
    per_f32 = kernel_bytes_per_vector(N_GRID[0] * N_GRID[1] * N_GRID[2], False)
    per_f64 = kernel_bytes_per_vector(N_GRID[0] * N_GRID[1] * N_GRID[2], True)
    kernels = {}
    for key in sorted(set(fetch) & set(write)):
        base, prec = key.rsplit("_", 1)
        alg = (per_f64 if prec == "fp64" else per_f32)[base] * ROOF_VECTORS
        hbm = (fetch[key] * cal_f + write[key] * cal_w) * 1024.0
        kernels[key] = {"hbm_bytes_per_launch": hbm, "fetch_kib": fetch[key], "write_kib": write[key],
                        "algorithmic_bytes_per_launch": alg, "vectors": ROOF_VECTORS}
    out = {"kernel_source_hash": kernel_source_hash(), "calibration": {"fetch": cal_f, "write": cal_w},
           "kernels": kernels, "note": "FCC diamond 64^3, 32-vector block; commands in traffic_fcc64.md"}
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
    return out


# FP32 register kernels with FP64 input / scaled FP64 output: the FP64-phase preconditioner
# (trace summaries only)
MIXED_KEYS = [("pcx::k_w64_fwd<double", "precond_plane_fwd_fp32in64"),
              ("pcx::k_w64_adj<double", "precond_plane_adj_fp32out64")]

# the two passes of the planes that take the two-pass path (trace summaries only)
SPLIT_KEYS = [(f"pcx::{k}<{t}", f"{lab}_{p}") for k, lab in
              (("k_zrow128_fwd", "rows_fwd"), ("k_zpass_fwd", "rows_fwd"), ("k_ypass_fwd", "cols_fwd"),
               ("k_ycol128_adj", "cols_adj"), ("k_ypass_adj", "cols_adj"), ("k_zrow128_adj", "rows_adj"),
               ("k_zpass_adj", "rows_adj"))
              for t, p in (("float", "fp32"), ("double", "fp64"))]


def summarize_trace(trace_csv: str, last: int = 20) -> str:
    """Markdown table of the A_r kernels' dispatch durations in a rocprofv3 --kernel-trace file,
    grouped by vector count (the grid's y extent): calls, mean, and the mean of the last `last`
    dispatches (for the 32-vector roofline block: the applications bench.py times, after its
    sustained warm-up)."""
    import csv
    from collections import defaultdict
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    groups = defaultdict(list)
    for r in rows:
        name = r["Kernel_Name"]
        key = next((k for p, k in KERNEL_KEYS + MIXED_KEYS + SPLIT_KEYS if name.startswith("void " + p) or name.startswith(p)),
                   None)
        if key:
            groups[(key, int(r["Grid_Size_Y"]))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    # the solves: every dispatch before the first plane kernel of the roofline block
    stop = next((k for k, r in enumerate(rows) if r["Kernel_Name"].startswith(("pcx::k_w64_fwd<float", "void pcx::k_w64_fwd<float",
                                                                                 "void pcx::k_p2_fwd", "pcx::k_p2_fwd"))
                 and int(r["Grid_Size_Y"]) == ROOF_VECTORS), len(rows))
    sol = rows[:stop]
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in sol) * 1e-6
    gaps = [(int(b["Start_Timestamp"]) - int(a["End_Timestamp"])) * 1e-3 for a, b in zip(sol, sol[1:])]
    span = (int(sol[-1]["End_Timestamp"]) - int(sol[0]["Start_Timestamp"])) * 1e-6 if sol else 0.0
    head = (f"Before the roofline block: {len(sol)} dispatches, span {span:.1f} ms, kernel time {busy:.1f} ms; "
            f"gaps between consecutive kernels: {sum(g for g in gaps if 20 <= g < 1000) * 1e-3:.1f} ms in "
            f"{sum(1 for g in gaps if 20 <= g < 1000)} gaps of 20 us - 1 ms, "
            f"{sum(g for g in gaps if 0 < g < 20) * 1e-3:.1f} ms below 20 us, "
            f"{sum(g for g in gaps if g >= 1000) * 1e-3:.1f} ms in gaps of 1 ms or more.\n\n")
    lines = ["| A_r kernel | vectors | calls | mean us | mean of last %d us |" % last, "|---|---|---|---|---|"]
    for (key, nv), d in sorted(groups.items(), key=lambda kv: (kv[0][0], -len(kv[1]))):
        if len(d) < 5:
            continue
        tail = d[-last:]
        lines.append(f"| {key} | {nv} | {len(d)} | {sum(d) / len(d):.1f} | {sum(tail) / len(tail):.1f} |")
    return head + "\n".join(lines)


def load_traffic(dominant: str, fp64: bool):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None if it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_fcc64.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    key = f"{dominant}_{'fp64' if fp64 else 'fp32'}"
    ent = d.get("kernels", {}).get(key)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def setup(torch, max_vectors: int):
    import pcx_synth as S
    from paper_1806_10284_amd import Plan, pcx_geometry, pcx_kappa_from_bloch
    g = pcx_geometry(S.FCC, *N_GRID)
    eps = S.sample_yee(S.FCC, N_GRID, tuple(g.shift), S.diamond_shapes(), 13.0, 1.0)
    kappa = pcx_kappa_from_bloch(S.FCC, S.FCC_POINTS["X"])
    plan = Plan(g, max_vectors=max_vectors)
    plan.pcx_plan_set_eps(eps)
    return plan, kappa, eps, g


def roofline_block(torch, plan, kappa, fp64: bool, reps: int, warmup_s: float = ROOF_WARMUP_S,
                   vectors: int = ROOF_VECTORS):
    import pcx_synth as S
    n = plan.n
    dt = torch.complex128 if fp64 else torch.complex64
    y = torch.from_numpy(np.ascontiguousarray(S.random_block(3, 2 * n, vectors).T)).to(dtype=dt, device="cuda")
    z = torch.empty_like(y)
    # sustained warm-up: after the host-side set-up above the GPU has idled, and its clocks take
    # some 30 ms of load to return to their steady state (the first applications run up to 15 %
    # slower); the timed applications then see the clocks a solve runs at
    t_w = time.perf_counter()
    plan.pcx_time_Ar_kernels(kappa, y, z, reps=2)
    while time.perf_counter() - t_w < warmup_s:
        plan.pcx_time_Ar_kernels(kappa, y, z, reps=10)
    ms = plan.pcx_time_Ar_kernels(kappa, y, z, reps=reps)
    names = ["plane_fwd", "xline", "plane_adj"]
    per = kernel_bytes_per_vector(n, fp64)
    out = {}
    for nm, t in zip(names, ms):
        b = per[nm] * vectors
        out[nm] = {"ms": t, "bytes": b, "gbs": b / (t * 1e-3) / 1e9}
    tot_ms = sum(ms)
    tot_b = sum(per.values()) * vectors
    return out, {"ms": tot_ms, "bytes": tot_b, "gbs": tot_b / (tot_ms * 1e-3) / 1e9,
                 "matvecs_per_s": vectors / (tot_ms * 1e-3)}


_CPU_JOB = {}


def _cpu_worker(budget_s: float):
    """One process of the CPU baseline: the oracle's A_r on the stored workload for budget_s."""
    from oracle.nfsep import Ar_apply
    spec, eps, y = _CPU_JOB["spec"], _CPU_JOB["eps"], _CPU_JOB["y"]
    done = 0
    t0 = time.perf_counter()
    while True:
        Ar_apply(spec, eps, y)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            return done, el


def host_info() -> dict:
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    blas = None
    try:
        dep = np.__config__.CONFIG["Build Dependencies"]["blas"]
        blas = f"{dep.get('name')} {dep.get('version')}"
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": cores, "numpy_blas": blas}


def cpu_baseline(avec, grid, eps, kappa, label: str, budget_s: float = 12.0, lanczos_ar: int | None = None):
    """The FP64 oracle on this host's cores, before anything touches the GPU: one process per usable
    core (at most 16, the box's share) applies the oracle's A_r (numpy FFT route, single-threaded per
    process, BLAS threads pinned to 1) to the same workload for budget_s; value = their summed rate.
    The oracle's own eigensolve (Section 5.2's inverse Lanczos, a sequential chain of A_r
    applications) needs `lanczos_ar` applications on this workload (counted when the stored
    oracle eigenvalues were written), so its seconds per k-point are estimated as that count over
    the rate of one process running alone (measured first, for budget_s / 2)."""
    import multiprocessing as mp

    from oracle.geometry import lattice_geometry
    from oracle.spectral import spectrum
    import pcx_synth as S
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    info = host_info()
    procs = max(1, min(16, info["usable_cores"]))
    g = lattice_geometry(avec, *grid)
    _CPU_JOB.update(spec=spectrum(g, kappa), eps=eps, y=S.random_block(4, 2 * g.npts, 1)[:, 0])
    ctx = mp.get_context("fork")
    with ctx.Pool(1) as pool:                 # one process alone: the rate a sequential solve sees
        d1, el1 = pool.map(_cpu_worker, [budget_s / 2])[0]
    with ctx.Pool(procs) as pool:
        runs = pool.map(_cpu_worker, [budget_s] * procs)
    rate = sum(d / el for d, el in runs)
    one = d1 / el1
    out = {"value": rate, "unit": "matvecs/s", "cores": procs, "kind": "oracle",
           "sample": f"{sum(d for d, _ in runs)} FP64 A_r applications of the oracle (numpy FFT) on {label}, "
                     f"{procs} processes x {budget_s:.0f} s (after {d1} by one process alone in {el1:.1f} s)",
           "host": info, "fft": "numpy.fft (pocketfft), one thread per process"}
    if lanczos_ar:
        out["s_per_kpoint_estimate"] = lanczos_ar / one
        out["s_per_kpoint_note"] = (f"oracle inverse Lanczos (CG inner solves) needs {lanczos_ar} sequential A_r "
                                    f"applications on this workload; estimate = count / the rate of one "
                                    f"process alone ({one:.2f} matvecs/s)")
    return out


def cpu_baseline_for(workload: str):
    """The oracle's inputs for the bench workload, from the oracle's own geometry (no GPU library)."""
    import pcx_synth as S
    from oracle.geometry import kappa_from_bloch, lattice_geometry
    if workload == "fcc_diamond":
        g = lattice_geometry(S.FCC, *N_GRID)
        eps = S.sample_yee(S.FCC, N_GRID, tuple(g.shift), S.diamond_shapes(), 13.0, 1.0)
        kappa = kappa_from_bloch(S.FCC, S.FCC_POINTS["X"])
        gold = os.path.join(ROOT, "tests", "golden", "config2_fcc64.json")
        lanczos_ar = json.load(open(gold)).get("ar_applications") if os.path.exists(gold) else None
        return cpu_baseline(S.FCC, N_GRID, eps, kappa, "FCC diamond 64^3 at X", lanczos_ar=lanczos_ar)
    g = lattice_geometry(S.BCC, *N_GRID)
    eps = S.gyroid_yee(N_GRID, tuple(g.shift), 12.0)
    kappa = kappa_from_bloch(S.BCC, S.BCC_POINTS["N"])
    return cpu_baseline(S.BCC, N_GRID, eps, kappa, "BCC gyroid 64^3 (eps 12) at N")


def run_gyroid_sweep(args, torch, mode, cpu):
    """Section 6's permittivity sweep: the single gyroid on the BCC lattice (level set > 1.1, cubic
    cell a), grid 64^3, eps = 3, 6, ..., 30 in air, one plan per eps, the N point, 10 bands.  One
    step = the whole sweep as one pcx_solve_batch call (worker threads with their own streams
    overlap the ten solves).  --workload gyroid_bands: the ten plans along the path G-H-N-G-P-H with
    each segment cut into 10 parts (51 wave vectors, 510 problems per step), the paper's figure of
    band structures against eps."""
    import pcx_synth as S
    from paper_1806_10284_amd import Plan, pcx_geometry, pcx_kappa_from_bloch, pcx_solve_batch
    from paper_1806_10284_amd.bands import band_structure
    bands = args.workload == "gyroid_bands"
    g = pcx_geometry(S.BCC, *N_GRID)
    kappa = pcx_kappa_from_bloch(S.BCC, S.BCC_POINTS["N"])
    plans, epss = [], []
    for e in S.GYROID_EPS_SWEEP:
        eps = S.gyroid_yee(N_GRID, tuple(g.shift), e)
        p = Plan(g, max_vectors=ROOF_VECTORS)
        p.pcx_plan_set_eps(eps)
        plans.append(p)
        epss.append(eps)
    print(f"[bench] setup done: BCC gyroid {N_GRID}, eps {S.GYROID_EPS_SWEEP}, kappa {kappa.tolist()}",
          file=sys.stderr, flush=True)
    problems = [(p, [tuple(kappa)]) for p in plans]
    corners = [S.BCC_POINTS[c] for c in "GHNGPH"]
    nprob = len(problems) * (51 if bands else 1)

    def one_sweep():
        t = time.perf_counter()
        if bands:
            bs = band_structure(plans, S.BCC, corners, NEV, parts=10, mode=mode, tol=1e-10, nworkers=args.workers)
            lam, st = bs.lam.reshape(-1, NEV), bs.stats
        else:
            lam, _, st = pcx_solve_batch(problems, NEV, mode=mode, tol=1e-10, nworkers=args.workers)
        return lam, st, time.perf_counter() - t

    def its(st):
        return [x.iterations for x in st] if not bands else \
            f"mean {np.mean([x.iterations for x in st]):.1f}, max {max(x.iterations for x in st)}"

    for w in range(args.warmup):
        _, st, s_el = one_sweep()
        print(f"[bench] warmup {w}: iterations {its(st)}, {s_el:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    applies = applies32 = matvecs = 0
    iters = []
    for s in range(args.steps):
        lam, st, s_el = one_sweep()
        matvecs += sum(x.matvecs for x in st)
        applies += sum(x.matvecs + x.precond_applies for x in st)
        applies32 += sum(x.matvecs_fp32 + x.precond_applies_fp32 for x in st)
        iters.append(its(st))
        print(f"[bench] step {s}: iterations {iters[-1]}, {s_el:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    q_mid = S.GYROID_EPS_SWEEP.index(12.0)
    kern, tot = roofline_block(torch, plans[q_mid], kappa, args.mode == "fp64", args.reps)
    dominant = max(kern, key=lambda k: kern[k]["ms"])
    dk = kern[dominant]
    print(f"[bench] roofline block: {json.dumps(kern)}", file=sys.stderr, flush=True)
    out = {
        "metric": "nullspace-free matvecs/s + HBM GB/s vs peak; s per k-point, 10 bands at 64^3",
        "value": matvecs / el,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_refine": "f32+f64", "fp64": "f64", "fp32": "f32"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "BCC single gyroid 64^3 (sin-cos level set > 1.1, eps 3..30 in steps of 3 "
                               "in air), one plan per eps batched, "
                               + ("path G-H-N-G-P-H with 10 parts per segment (51 wave vectors), "
                                  if bands else "N point, ") + "10 smallest positive eigenvalues",
                   "grid": list(N_GRID), "nev": NEV, "mode": args.mode, "solver": "lobpcg",
                   "eps": list(S.GYROID_EPS_SWEEP), "kappa": kappa.tolist(), "workers": args.workers or 4},
        "s_per_kpoint": el / args.steps / nprob,
        "solve": {"iterations": iters, "matvecs_per_step": matvecs / args.steps,
                  "operator_applications_per_step": applies / args.steps,
                  "fp32_application_fraction": applies32 / max(applies, 1), "tol": 1e-10,
                  "problems_per_step": nprob,
                  "fp64_fallbacks_last_step": int(sum(x.restarts for x in st)),
                  "lambda_at_N" if not bands else "lambda_at_G":
                      {str(e): [float(x) for x in lam[q * (nprob // len(plans))]]
                       for q, e in enumerate(S.GYROID_EPS_SWEEP)}},
        "block_matvec": {"vectors": ROOF_VECTORS, "precision": "fp64" if args.mode == "fp64" else "fp32",
                         "matvecs_per_s": tot["matvecs_per_s"], "gbs": tot["gbs"],
                         "frac_of_peak": tot["gbs"] / HBM_PEAK_GBS,
                         "kernels": {k: {"ms": v["ms"], "gbs": v["gbs"]} for k, v in kern.items()}},
        # the committed counter data were taken on the FCC diamond workload, not this one
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": dk["bytes"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


TRI_GRID = (128, 128, 128)
TRI_NEV, TRI_TOL, TRI_VECTORS = 20, 1e-9, 8


def run_triclinic128(args, torch, mode):
    """The largest workload: a seeded triclinic lattice (seed 5) at 128^3, random spheres filled to
    30 % with eps = 13, 20 bands at 16 seeded wave vectors, solved as one pcx_solve_batch call (one
    step).  Its planes (128 x 128) take the two-pass plane path; the roofline block is 8 vectors
    (a 1.1 GB FP32 working set, beyond the last-level cache), with the 3-pass algorithmic bytes."""
    import pcx_synth as S
    from paper_1806_10284_amd import PCX_EPS_VOXEL, Plan, pcx_geometry, pcx_solve_batch
    avec = S.triclinic(5)
    g = pcx_geometry(avec, *TRI_GRID)
    vox = S.random_sphere_fill(avec, TRI_GRID, tuple(g.shift), seed=5)
    kappas = [tuple(k) for k in S.random_kappas(55, 16)]
    plan = Plan(g, max_vectors=32)
    plan.pcx_plan_set_eps(vox, PCX_EPS_VOXEL)
    print(f"[bench] setup done: triclinic(5) {TRI_GRID}, {len(kappas)} wave vectors", file=sys.stderr, flush=True)
    workers = args.workers or 2

    def one_batch():
        t = time.perf_counter()
        lam, _, st = pcx_solve_batch([(plan, kappas)], TRI_NEV, mode=mode, tol=TRI_TOL, nworkers=workers)
        return lam, st, time.perf_counter() - t

    for w in range(args.warmup):
        _, st, s_el = one_batch()
        print(f"[bench] warmup {w}: {s_el:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = applies = applies32 = 0
    iters = []
    for s in range(args.steps):
        lam, st, s_el = one_batch()
        matvecs += sum(x.matvecs for x in st)
        applies += sum(x.matvecs + x.precond_applies for x in st)
        applies32 += sum(x.matvecs_fp32 + x.precond_applies_fp32 for x in st)
        iters.append([x.iterations for x in st])
        print(f"[bench] step {s}: iterations {iters[-1]}, {s_el:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern, tot = roofline_block(torch, plan, kappas[0], args.mode == "fp64", args.reps, vectors=TRI_VECTORS)
    dominant = max(kern, key=lambda k: kern[k]["ms"])
    dk = kern[dominant]
    print(f"[bench] roofline block: {json.dumps(kern)}", file=sys.stderr, flush=True)
    out = {
        "metric": "nullspace-free matvecs/s + HBM GB/s vs peak; s per k-point, 20 bands at 128^3",
        "value": matvecs / el,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_refine": "f32+f64", "fp64": "f64", "fp32": "f32"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "triclinic (seed 5) 128^3, random spheres eps 13 filling 30 %, 16 seeded wave "
                               "vectors in one batch, 20 smallest positive eigenvalues",
                   "grid": list(TRI_GRID), "nev": TRI_NEV, "mode": args.mode, "solver": "lobpcg",
                   "workers": workers},
        "s_per_kpoint": el / args.steps / len(kappas),
        "solve": {"iterations": iters, "matvecs_per_step": matvecs / args.steps,
                  "operator_applications_per_step": applies / args.steps,
                  "fp32_application_fraction": applies32 / max(applies, 1), "tol": TRI_TOL,
                  "lambda_first_wave_vector": [float(x) for x in lam[0]]},
        "block_matvec": {"vectors": TRI_VECTORS, "precision": "fp64" if args.mode == "fp64" else "fp32",
                         "matvecs_per_s": tot["matvecs_per_s"], "gbs": tot["gbs"],
                         "frac_of_peak": tot["gbs"] / HBM_PEAK_GBS,
                         "kernels": {k: {"ms": v["ms"], "gbs": v["gbs"]} for k, v in kern.items()}},
        # counters were taken on the FCC diamond workload; the two-pass planes move 236n B (FP32)
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": dk["bytes"]},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="fp32_refine", choices=["fp32_refine", "fp64", "fp32"])
    ap.add_argument("--solver", default="lobpcg", choices=["lobpcg", "lanczos"],
                    help="lanczos: the paper's driver (inverse Lanczos, CG inner solves, FP64; --mode ignored)")
    ap.add_argument("--workload", default="fcc_diamond",
                    choices=["fcc_diamond", "gyroid_sweep", "gyroid_bands", "triclinic128"],
                    help="gyroid_sweep: BCC single gyroid 64^3, eps 3..30 as one batch of 10 plans at N; "
                         "gyroid_bands: the same ten plans along G-H-N-G-P-H, 10 parts per segment; "
                         "triclinic128: a seeded triclinic 128^3, 20 bands at 16 wave vectors in one batch "
                         "(no CPU baseline)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--workers", type=int, default=0,
                    help="batch workloads: worker threads (0: 4 for the gyroid, 2 for triclinic128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only run the 32-vector A_r block (and a calibration copy) for rocprofv3 counters")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic_fcc64.json from two rocprofv3 --pmc counter files and exit")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print the A_r kernels' dispatch durations by vector count from a rocprofv3 trace and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_traffic:
        out = summarize_traffic(*args.summarize_traffic, os.path.join(ROOT, "profiles", "traffic_fcc64.json"))
        print(json.dumps(out, indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this solver is single-device (k-points shard across GPUs "
              "without communication)", file=sys.stderr)
        sys.exit(2)

    if args.solver == "lanczos":
        args.mode = "fp64"
    # the CPU baseline runs first, in forked processes, before anything initialises the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.profile_kernels and args.workload != "triclinic128":
        cpu = cpu_baseline_for(args.workload)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    import torch
    from paper_1806_10284_amd import PCX_MODE_FP32, PCX_MODE_FP32_REFINE, PCX_MODE_FP64
    torch.cuda.set_device(0)
    mode = {"fp32_refine": PCX_MODE_FP32_REFINE, "fp64": PCX_MODE_FP64, "fp32": PCX_MODE_FP32}[args.mode]
    if args.workload != "fcc_diamond":
        if args.solver != "lobpcg" or args.profile_kernels:
            print(f"--workload {args.workload} runs the batched LOBPCG solver only", file=sys.stderr)
            sys.exit(2)
        if args.workload == "triclinic128":
            return run_triclinic128(args, torch, mode)
        return run_gyroid_sweep(args, torch, mode, cpu)
    plan, kappa, eps, g = setup(torch, max_vectors=ROOF_VECTORS)
    print(f"[bench] setup done: FCC diamond {N_GRID}, kappa {kappa.tolist()}", file=sys.stderr, flush=True)

    if args.profile_kernels:
        for fp64 in (False, True):
            kern, _ = roofline_block(torch, plan, kappa, fp64, reps=5)
            print(f"[bench] profiled block matvec fp64={fp64}: {json.dumps(kern)}", file=sys.stderr, flush=True)
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")   # 512 MiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 5 x 512 MiB", file=sys.stderr, flush=True)
        return

    solve_kw = dict(mode=mode, tol=1e-10, want_y=False)

    def one_solve():
        if args.solver == "lanczos":
            # the paper's outer / inner tolerances (1e-12, 1e-13)
            lam, sl = plan.pcx_solve_lanczos(kappa, NEV)
            return lam, {"it": sl["steps"], "it32": 0, "mv": sl["matvecs"], "mv32": 0, "pre": 0, "pre32": 0,
                         "tm": 0.0, "s": sl["seconds"], "res": [float(r) for r in sl["residual"]], "floor": []}
        lam, _, _, st = plan.pcx_solve(kappa, NEV, **solve_kw)
        return lam, {"it": st.iterations, "it32": st.iterations_fp32, "mv": st.matvecs, "mv32": st.matvecs_fp32,
                     "pre": st.precond_applies, "pre32": st.precond_applies_fp32, "tm": st.seconds_matvec,
                     "s": st.seconds, "res": [float(r) for r in st.residual],
                     "floor": [j for j in range(NEV) if (st.floor_mask >> j) & 1]}

    for w in range(args.warmup):
        lam, st = one_solve()
        print(f"[bench] warmup {w}: {st['it']} it, {st['mv']} matvecs, {st['s']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    matvecs = matvecs32 = pre = pre32 = 0
    tm = 0.0
    iters = []
    for s in range(args.steps):
        lam, st = one_solve()
        matvecs += st["mv"]
        matvecs32 += st["mv32"]
        pre += st["pre"]
        pre32 += st["pre32"]
        tm += st["tm"]
        iters.append(st["it"])
        print(f"[bench] step {s}: {st['it']} it ({st['it32']} fp32), {st['mv']} matvecs, "
              f"{st['pre']} preconditioner applications, {st['s']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    # value: applications of A_r itself per second.  The approximate-inverse preconditioner runs the
    # same three kernels with eps in place of 1/eps; its applications are listed under "solve" and
    # counted only in the in-solve bandwidth figure
    applies, applies32 = matvecs + pre, matvecs32 + pre32
    value = matvecs / el
    n = plan.n
    per32 = sum(kernel_bytes_per_vector(n, False).values())
    per64 = sum(kernel_bytes_per_vector(n, True).values())
    solve_gbs = (applies32 * per32 + (applies - applies32) * per64) / el / 1e9

    # per-band agreement of the timed mode with the plain FP64 path (same tolerance)
    per_band = None
    if args.mode != "fp64" or args.solver == "lanczos":
        lam64, _, _, _ = plan.pcx_solve(kappa, NEV, mode=PCX_MODE_FP64, tol=1e-10, want_y=False)
        per_band = [float(abs(a - b) / b) for a, b in zip(lam, lam64)]
        print(f"[bench] per-band |lambda - lambda_fp64| / lambda_fp64: {per_band}", file=sys.stderr, flush=True)

    fp64_roof = args.mode == "fp64"
    kern, tot = roofline_block(torch, plan, kappa, fp64_roof, args.reps)
    dominant = max(kern, key=lambda k: kern[k]["ms"])
    dk = kern[dominant]
    traffic = load_traffic(dominant, fp64_roof)
    print(f"[bench] roofline block: {json.dumps(kern)}", file=sys.stderr, flush=True)


    out = {
        "metric": "nullspace-free matvecs/s + HBM GB/s vs peak; s per k-point, 10 bands at 64^3",
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32_refine": "f32+f64", "fp64": "f64", "fp32": "f32"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "FCC diamond 64^3 (spheres r=0.12a, rods r=0.11a, eps 13/1), X point, "
                               "10 smallest positive eigenvalues",
                   "grid": list(N_GRID), "nev": NEV, "mode": args.mode, "solver": args.solver,
                   "kappa": kappa.tolist()},
        "s_per_kpoint": el / args.steps,
        "solve": {"iterations": iters, "matvecs_per_solve": matvecs / args.steps,
                  "precond_applies_per_solve": pre / args.steps,
                  "operator_applications_per_solve": applies / args.steps,
                  "fp32_application_fraction": applies32 / max(applies, 1),
                  "matvec_time_fraction": tm / el, "matvec_gbs_in_solve": solve_gbs,
                  "tol": solve_kw["tol"], "lambda": [float(x) for x in lam],
                  "final_rel_residual_per_band": st["res"][:NEV],
                  "bands_accepted_at_floor": st["floor"],
                  "rel_diff_vs_fp64_per_band": per_band,
                  "omega_over_2pi": [math.sqrt(max(x, 0)) / (2 * math.pi) for x in lam]},
        "block_matvec": {"vectors": ROOF_VECTORS, "precision": "fp64" if fp64_roof else "fp32",
                         "matvecs_per_s": tot["matvecs_per_s"], "gbs": tot["gbs"],
                         "frac_of_peak": tot["gbs"] / HBM_PEAK_GBS,
                         "kernels": {k: {"ms": v["ms"], "gbs": v["gbs"]} for k, v in kern.items()}},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": dk["bytes"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
