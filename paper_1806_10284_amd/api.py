"""Python binding of the pcx C ABI: the same calls, with torch tensors for device memory.

Every computation runs in libpcx.so (HIP kernels on the current device); this module only
checks shapes/dtypes and passes pointers and the current torch stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _avec9(avec) -> L.c_double9:
    a = np.ascontiguousarray(np.asarray(avec, dtype=np.float64).reshape(3, 3))
    return L.c_double9(*a.reshape(-1).tolist())


def pcx_geometry(avec, n1: int, n2: int, n3: int) -> L.PcxGeom:
    """Section 2.2: corrected, rotated lattice (columns of ``avec`` are the user's vectors)."""
    lib = L.load()
    g = L.PcxGeom()
    L.check(lib.pcx_geometry(_avec9(avec), int(n1), int(n2), int(n3), ctypes.byref(g)))
    return g


def pcx_kappa_from_bloch(avec, kvec) -> np.ndarray:
    lib = L.load()
    out = L.c_double3()
    L.check(lib.pcx_kappa_from_bloch(_avec9(avec), L.c_double3(*[float(x) for x in kvec]), out))
    return np.array(list(out))


def pcx_omega(avec, geom: L.PcxGeom) -> np.ndarray:
    """Section 2.3: Omega (3x3) mapping user-frame Bloch vectors to the frame of the rotated,
    corrected lattice of ``geom`` (from pcx_geometry with the same ``avec``)."""
    lib = L.load()
    out = L.c_double9()
    L.check(lib.pcx_omega(_avec9(avec), ctypes.byref(geom), out))
    return np.array(list(out)).reshape(3, 3)


def geom_dict(g: L.PcxGeom) -> dict:
    return {"n": tuple(g.n), "m": tuple(g.m), "rho": tuple(g.rho), "shift": tuple(g.shift),
            "delta": tuple(g.delta), "avec_rot": np.array(list(g.avec_rot)).reshape(3, 3),
            "cos_angles": tuple(g.cos_angles)}


def _torch():
    import torch
    return torch


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _kappa3(kappa) -> L.c_double3:
    k = [float(x) for x in kappa]
    if len(k) != 3:
        raise ValueError("kappa must have 3 entries")
    return L.c_double3(*k)


@dataclass
class SolveStats:
    iterations: int
    iterations_fp32: int
    matvecs: int
    matvecs_fp32: int
    seconds: float
    seconds_matvec: float
    residual: np.ndarray
    converged: int
    precond_applies: int = 0
    precond_applies_fp32: int = 0
    restarts: int = 0
    floor_mask: int = 0           # bit j: band j accepted at the absolute residual floor (next to Gamma)
    orth_fallbacks: int = 0       # phases that fell back to orthonormalising W on the host


class Plan:
    """pcx_plan: one lattice/grid on the current HIP device and torch stream."""

    def __init__(self, geom: L.PcxGeom, max_vectors: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("pcx needs a HIP device (torch.cuda.is_available() is False)")
        self._lib = L.load()
        self.geom = geom
        self.n = int(geom.n[0]) * int(geom.n[1]) * int(geom.n[2])
        ptr = ctypes.c_void_p()
        L.check(self._lib.pcx_plan_create(ctypes.byref(geom), int(max_vectors), _stream_handle(), ctypes.byref(ptr)))
        self._ptr = ptr
        self.max_vectors = max_vectors or L.PCX_MAX_BLOCK

    def close(self):
        if getattr(self, "_ptr", None) and self._ptr.value:
            self._lib.pcx_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- permittivity
    def pcx_plan_set_eps(self, eps, layout: int = L.PCX_EPS_YEE3):
        e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1))
        want = 3 * self.n if layout == L.PCX_EPS_YEE3 else self.n
        if e.size != want:
            raise ValueError(f"eps has {e.size} values, expected {want}")
        L.check(self._lib.pcx_plan_set_eps(self._ptr, e.ctypes.data_as(ctypes.c_void_p), int(layout)))

    def pcx_plan_set_variant(self, variant: int):
        """PCX_VARIANT_AUTO (fixed-size kernels where available), _GENERIC, _THREE_PLANE, _TWO_PLANE or
        _REGISTER."""
        L.check(self._lib.pcx_plan_set_variant(self._ptr, int(variant)))

    # -- operators
    def _check_block(self, t, per_vec: int, precision: int, name: str) -> int:
        torch = _torch()
        dt = torch.complex128 if precision in (L.PCX_FP64, L.PCX_FP64_OP32) else torch.complex64
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be a device tensor")
        if t.dtype != dt:
            raise ValueError(f"{name} must be {dt}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() % per_vec or t.numel() == 0:
            raise ValueError(f"{name} must hold whole vectors of {per_vec} entries")
        return t.numel() // per_vec

    def _apply(self, fn, kappa, precision, x, out, nin, nout):
        nv = self._check_block(x, nin, precision, "input")
        nv2 = self._check_block(out, nout, precision, "output")
        if nv != nv2:
            raise ValueError("input and output hold different numbers of vectors")
        L.check(fn(self._ptr, _kappa3(kappa), int(precision), ctypes.c_void_p(x.data_ptr()),
                   ctypes.c_void_p(out.data_ptr()), nv))
        return out

    def pcx_apply_Ar(self, kappa, y, z, precision=None):
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_apply_Ar, kappa, precision, y, z, 2 * self.n, 2 * self.n)

    def pcx_apply_curl(self, kappa, u, v, adjoint: bool = False, precision=None):
        """v = C u (or C^* u): the discrete curl on 3n-vectors (e-layout)."""
        precision = self._prec_of(u) if precision is None else precision
        nv = self._check_block(u, 3 * self.n, precision, "u")
        if self._check_block(v, 3 * self.n, precision, "v") != nv:
            raise ValueError("u and v hold different numbers of vectors")
        L.check(self._lib.pcx_apply_curl(self._ptr, _kappa3(kappa), int(precision), ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(v.data_ptr()), nv, int(bool(adjoint))))
        return v

    def pcx_hfield(self, kappa, y, h, precision=None):
        """h = P_r y = C Q_r Sigma_r^{-1} y: the magnetic field of an NFSEP vector (2n -> 3n)."""
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_hfield, kappa, precision, y, h, 2 * self.n, 3 * self.n)

    def pcx_apply_hfield_operator(self, kappa, h, z, precision=None):
        """z = C B^{-1} C^* h (3n -> 3n)."""
        precision = self._prec_of(h) if precision is None else precision
        return self._apply(self._lib.pcx_apply_hfield_operator, kappa, precision, h, z, 3 * self.n, 3 * self.n)

    def pcx_apply_Ar_noalloc(self, kappa, y, z, precision=None):
        """z = A_r y with every temporary in the library's static device scratch (no allocation);
        at most PCX_NOALLOC_SCRATCH_BYTES of codes and workspace per call."""
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_apply_Ar_noalloc, kappa, precision, y, z, 2 * self.n, 2 * self.n)

    def pcx_apply_precond(self, kappa, y, z, precision=None):
        """z = D Sigma_r Q_r^* B Q_r Sigma_r D y, D = Lambda_q^{-1}: the approximate-inverse
        preconditioner of the solver (z may be y).  precision PCX_FP64_OP32: complex128 y and z,
        the operator between the FP64 scalings in FP32 (the FP64 solver phase's form)."""
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_apply_precond, kappa, precision, y, z, 2 * self.n, 2 * self.n)

    def pcx_apply_Ar_multi(self, kappas, y, z, precision=None):
        """z = A_r(kappa_k) y for every wave vector in one launch per kernel; y, z hold
        len(kappas) equal groups of vectors, ordered [k][v]."""
        precision = self._prec_of(y) if precision is None else precision
        ks = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64).reshape(-1, 3))
        nv = self._check_block(y, 2 * self.n, precision, "y")
        if self._check_block(z, 2 * self.n, precision, "z") != nv or nv % len(ks):
            raise ValueError("y and z must hold the same whole number of vectors per wave vector")
        L.check(self._lib.pcx_apply_Ar_multi(self._ptr, len(ks), ks.ctypes.data_as(ctypes.c_void_p), int(precision),
                                             ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                             nv // len(ks)))
        return z

    def pcx_plan_autotune(self, kappa, precision=L.PCX_FP32, nvec: int = 8):
        """Times the kernel variants on this plan and keeps the fastest; returns (choice, ms):
        choice 0 = the plan's automatic choice, -1 / -2 / -3 = three-plane / two-plane fixed-size /
        register-resident kernels, else the generic plane work-group size."""
        ch = ctypes.c_int()
        ms = ctypes.c_double()
        L.check(self._lib.pcx_plan_autotune(self._ptr, _kappa3(kappa), int(precision), int(nvec), ctypes.byref(ch),
                                            ctypes.byref(ms)))
        return ch.value, ms.value

    def pcx_apply_QS(self, kappa, y, u, precision=None):
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_apply_QS, kappa, precision, y, u, 2 * self.n, 3 * self.n)

    def pcx_apply_QS_adjoint(self, kappa, u, z, precision=None):
        precision = self._prec_of(u) if precision is None else precision
        return self._apply(self._lib.pcx_apply_QS_adjoint, kappa, precision, u, z, 3 * self.n, 2 * self.n)

    def pcx_eigvec(self, kappa, y, x, precision=None):
        precision = self._prec_of(y) if precision is None else precision
        return self._apply(self._lib.pcx_eigvec, kappa, precision, y, x, 2 * self.n, 3 * self.n)

    def pcx_time_Ar_kernels(self, kappa, y, z, reps: int = 10):
        """Mean milliseconds per launch of the three A_r kernels (HIP events on the plan's stream)."""
        precision = self._prec_of(y)
        nv = self._check_block(y, 2 * self.n, precision, "y")
        self._check_block(z, 2 * self.n, precision, "z")
        ms = L.c_double3()
        L.check(self._lib.pcx_time_Ar_kernels(self._ptr, _kappa3(kappa), int(precision), ctypes.c_void_p(y.data_ptr()),
                                              ctypes.c_void_p(z.data_ptr()), nv, int(reps), ms))
        return list(ms)

    @staticmethod
    def _prec_of(t):
        torch = _torch()
        return L.PCX_FP64 if t.dtype == torch.complex128 else L.PCX_FP32

    # -- eigensolver
    def pcx_solve(self, kappa, nev: int, *, mode=L.PCX_MODE_FP64, block=0, max_iter=400, tol=1e-9,
                  tol_fp32=1e-3, seed=12345, precondition=True, verbose=False, want_y=True, want_x=False,
                  raise_on_noconv=True, y0=None, orthonormalize_w=False):
        """Returns (lambda[nev] numpy, y (nev, 2n) complex128 or None, x (nev, 3n) complex128 or None, stats).
        y0: optional warm start, a contiguous complex128 device tensor of whole 2n-vectors.
        orthonormalize_w: orthonormalise the new directions against X on the host in every
        iteration (two host synchronisations per iteration instead of one)."""
        torch = _torch()
        opts = L.PcxOpts()
        self._lib.pcx_opts_default(ctypes.byref(opts))
        opts.mode, opts.block, opts.max_iter = int(mode), int(block), int(max_iter)
        opts.tol, opts.tol_fp32, opts.seed = float(tol), float(tol_fp32), int(seed)
        opts.precondition, opts.verbose = _precond(precondition), int(bool(verbose))
        opts.orthonormalize_w = int(bool(orthonormalize_w))
        if y0 is not None:
            opts.y0 = ctypes.c_void_p(y0.data_ptr())
            opts.n_y0 = self._check_block(y0, 2 * self.n, L.PCX_FP64, "y0")
        lam = np.zeros(nev, dtype=np.float64)
        dev = torch.device("cuda", torch.cuda.current_device())
        y = torch.empty((nev, 2 * self.n), dtype=torch.complex128, device=dev) if (want_y or want_x) else None
        x = torch.empty((nev, 3 * self.n), dtype=torch.complex128, device=dev) if want_x else None
        st = L.PcxStats()
        code = self._lib.pcx_solve(self._ptr, _kappa3(kappa), int(nev), ctypes.byref(opts),
                                   lam.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(y.data_ptr()) if y is not None else None,
                                   ctypes.c_void_p(x.data_ptr()) if x is not None else None, ctypes.byref(st))
        stats = SolveStats(st.iterations, st.iterations_fp32, st.matvecs, st.matvecs_fp32, st.seconds,
                           st.seconds_matvec, np.array(list(st.residual))[:nev], st.converged, st.precond_applies,
                           st.precond_applies_fp32, st.restarts, st.floor_mask, st.orth_fallbacks)
        if code != L.PCX_OK and (raise_on_noconv or code != L.PCX_E_NOCONV):
            L.check(code)
        return lam, (y if want_y else None), x, stats

    def pcx_solve_lanczos(self, kappa, nev: int, *, tol_outer=1e-12, tol_inner=1e-13, max_steps=200, max_cg=2000,
                          seed=4242, raise_on_noconv=True):
        """The paper's driver: inverse Lanczos with CG inner solves (FP64).  Returns (lambda[nev]
        numpy ascending, stats dict)."""
        opts = L.PcxLanczosOpts()
        self._lib.pcx_lanczos_opts_default(ctypes.byref(opts))
        opts.tol_outer, opts.tol_inner = float(tol_outer), float(tol_inner)
        opts.max_steps, opts.max_cg, opts.seed = int(max_steps), int(max_cg), int(seed)
        lam = np.zeros(nev, dtype=np.float64)
        st = L.PcxLanczosStats()
        code = self._lib.pcx_solve_lanczos(self._ptr, _kappa3(kappa), int(nev), ctypes.byref(opts),
                                           lam.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st))
        stats = {"steps": st.steps, "cg_iterations": st.cg_iterations, "matvecs": st.matvecs,
                 "seconds": st.seconds, "residual": np.array(list(st.residual))[:nev], "converged": st.converged}
        if code != L.PCX_OK and (raise_on_noconv or code != L.PCX_E_NOCONV):
            L.check(code)
        return lam, stats

    def _opts(self, mode, block, max_iter, tol, tol_fp32, seed, precondition, verbose):
        opts = L.PcxOpts()
        self._lib.pcx_opts_default(ctypes.byref(opts))
        opts.mode, opts.block, opts.max_iter = int(mode), int(block), int(max_iter)
        opts.tol, opts.tol_fp32, opts.seed = float(tol), float(tol_fp32), int(seed)
        opts.precondition, opts.verbose = _precond(precondition), int(bool(verbose))
        return opts

    # -- the Rayleigh-Ritz products (Section 5.2), for tests and tools
    @staticmethod
    def _cols(t, name):
        torch = _torch()
        if t.device.type != "cuda" or t.dim() != 2 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous 2-D device tensor (columns x length)")
        if t.dtype not in (torch.complex128, torch.complex64):
            raise ValueError(f"{name} must be complex128 or complex64")
        return L.PCX_FP64 if t.dtype == torch.complex128 else L.PCX_FP32

    def pcx_block_gram(self, a, b=None, herm: bool = True):
        """G = A^H B (numpy complex128, ka x kb) for column blocks a (ka, len) and b (kb, len); herm:
        B = [A | b] (or A when b is None) with Hermitian halves, formed on their upper triangles."""
        prec = self._cols(a, "a")
        ka, n = a.shape
        if b is not None:
            if self._cols(b, "b") != prec or b.shape[1] != n:
                raise ValueError("a and b need the same precision and length")
        elif not herm:
            raise ValueError("the general product needs b")
        kb = (ka if b is None else 2 * ka) if herm else b.shape[0]
        if herm and b is not None and b.shape[0] != ka:
            raise ValueError("herm: b must have as many columns as a")
        g = np.zeros((ka, kb), dtype=np.complex128)
        L.check(self._lib.pcx_block_gram(self._ptr, prec, ctypes.c_void_p(a.data_ptr()), ka,
                                         ctypes.c_void_p(b.data_ptr()) if b is not None else None, kb, n, int(herm),
                                         g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def pcx_block_combine(self, s, c, y):
        """y = s c: s (ks, len) and y (m, len) device column blocks, c a (ks, m) complex128 array."""
        prec = self._cols(s, "s")
        if self._cols(y, "y") != prec or y.shape[1] != s.shape[1]:
            raise ValueError("s and y need the same precision and length")
        cc = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
        if cc.shape != (s.shape[0], y.shape[0]):
            raise ValueError("c must be ks x m")
        L.check(self._lib.pcx_block_combine(self._ptr, prec, ctypes.c_void_p(s.data_ptr()), s.shape[0],
                                            cc.ctypes.data_as(ctypes.c_void_p), y.shape[0],
                                            ctypes.c_void_p(y.data_ptr()), s.shape[1]))
        return y

    def pcx_grad_eps(self, x, weight, layout: int = L.PCX_EPS_YEE3):
        """-sum_t weight[t] |x_t|^2 per Yee point (or per voxel): d(sum_t w_t lambda_t)/d eps."""
        torch = _torch()
        nv = self._check_block(x, 3 * self.n, L.PCX_FP64, "x")
        w = np.ascontiguousarray(np.asarray(weight, dtype=np.float64).reshape(-1))
        if w.size != nv:
            raise ValueError("one weight per eigenvector is needed")
        out = torch.empty(3 * self.n if layout == L.PCX_EPS_YEE3 else self.n, dtype=torch.float64, device=x.device)
        L.check(self._lib.pcx_grad_eps(self._ptr, nv, ctypes.c_void_p(x.data_ptr()), w.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.c_void_p(out.data_ptr()), int(layout)))
        return out


def _precond(v) -> int:
    """True / False (the default PCX_PRECOND_INVERSE / PCX_PRECOND_NONE) or a PCX_PRECOND_* code."""
    if isinstance(v, bool):
        return L.PCX_PRECOND_INVERSE if v else L.PCX_PRECOND_NONE
    v = int(v)
    if v not in (L.PCX_PRECOND_NONE, L.PCX_PRECOND_DIAG, L.PCX_PRECOND_INVERSE):
        raise ValueError(f"unknown preconditioner {v}")
    return v


def pcx_solve_batch(problems, nev: int, *, mode=L.PCX_MODE_FP32_REFINE, block=0, max_iter=400, tol=1e-9,
                    tol_fp32=1e-3, seed=12345, precondition=True, nworkers=0, want_y=False,
                    raise_on_noconv=True):
    """Solves independent problems concurrently.  problems: list of (plan, [kappa, ...]).
    Returns (lambda (total, nev) numpy, list of y tensors (None where not requested) or None, list of
    SolveStats), problems in plan-major order.  want_y: False, True, or the problem indices."""
    torch = _torch()
    plans = [p for p, _ in problems]
    nk = np.array([len(ks) for _, ks in problems], dtype=np.int32)
    ks = np.ascontiguousarray(np.concatenate([np.asarray(k, dtype=np.float64).reshape(-1, 3)
                                              for _, k in problems]).reshape(-1))
    total = int(nk.sum())
    lib = plans[0]._lib
    opts = plans[0]._opts(mode, block, max_iter, tol, tol_fp32, seed, precondition, False)
    ptrs = (ctypes.c_void_p * len(plans))(*[p._ptr.value for p in plans])
    lam = np.zeros((total, nev), dtype=np.float64)
    st = (L.PcxStats * total)()
    ys, yp = None, None
    if want_y:
        # want_y: True for every problem, or an iterable of the problem indices to return y for
        keep = set(range(total)) if want_y is True else set(int(q) for q in want_y)
        dev = torch.device("cuda", torch.cuda.current_device())
        ys = []
        for p, kl in problems:
            for _ in range(len(kl)):
                q = len(ys)
                ys.append(torch.empty((nev, 2 * p.n), dtype=torch.complex128, device=dev) if q in keep else None)
        yp = (ctypes.c_void_p * total)(*[t.data_ptr() if t is not None else None for t in ys])
    torch.cuda.synchronize()
    code = lib.pcx_solve_batch(ptrs, len(plans), nk.ctypes.data_as(ctypes.c_void_p),
                               ks.ctypes.data_as(ctypes.c_void_p), int(nev), ctypes.byref(opts), int(nworkers),
                               lam.ctypes.data_as(ctypes.c_void_p), yp, st)
    stats = [SolveStats(s.iterations, s.iterations_fp32, s.matvecs, s.matvecs_fp32, s.seconds, s.seconds_matvec,
                        np.array(list(s.residual))[:nev], s.converged, s.precond_applies,
                        s.precond_applies_fp32, s.restarts, s.floor_mask, s.orth_fallbacks) for s in st]
    if code != L.PCX_OK and (raise_on_noconv or code != L.PCX_E_NOCONV):
        L.check(code)
    return lam, ys, stats
