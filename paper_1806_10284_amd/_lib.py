"""ctypes declarations of the C ABI in include/pcx.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcx.so")

PCX_OK, PCX_E_ARG, PCX_E_SIZE, PCX_E_LATTICE, PCX_E_NOCONV, PCX_E_OOM, PCX_E_DEVICE = 0, -1, -2, -3, -4, -5, -6
PCX_FP64, PCX_FP32 = 0, 1
PCX_FP64_OP32 = 2          # pcx_apply_precond only: complex128 buffers, operator in FP32
PCX_EPS_YEE3, PCX_EPS_VOXEL = 0, 1
PCX_MODE_FP64, PCX_MODE_FP32_REFINE, PCX_MODE_FP32 = 0, 1, 2
PCX_PRECOND_NONE, PCX_PRECOND_DIAG, PCX_PRECOND_INVERSE = 0, 1, 2
PCX_VARIANT_AUTO, PCX_VARIANT_GENERIC, PCX_VARIANT_THREE_PLANE, PCX_VARIANT_TWO_PLANE, PCX_VARIANT_REGISTER = 0, 1, 2, 3, 4
PCX_MAX_N = 256
PCX_MAX_BLOCK = 64

c_int3 = ctypes.c_int * 3
c_double3 = ctypes.c_double * 3
c_double9 = ctypes.c_double * 9


class PcxGeom(ctypes.Structure):
    _fields_ = [
        ("n", c_int3), ("m", c_int3), ("rho", c_int3), ("shift", c_int3),
        ("delta", c_double3), ("avec_rot", c_double9), ("cos_angles", c_double3),
    ]


class PcxOpts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int), ("block", ctypes.c_int), ("max_iter", ctypes.c_int),
        ("tol", ctypes.c_double), ("tol_fp32", ctypes.c_double),
        ("seed", ctypes.c_ulonglong), ("precondition", ctypes.c_int), ("verbose", ctypes.c_int),
        ("y0", ctypes.c_void_p), ("n_y0", ctypes.c_int), ("orthonormalize_w", ctypes.c_int),
    ]


class PcxStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int), ("iterations_fp32", ctypes.c_int),
        ("matvecs", ctypes.c_longlong), ("matvecs_fp32", ctypes.c_longlong),
        ("seconds", ctypes.c_double), ("seconds_matvec", ctypes.c_double),
        ("residual", ctypes.c_double * PCX_MAX_BLOCK), ("converged", ctypes.c_int),
        ("precond_applies", ctypes.c_longlong), ("precond_applies_fp32", ctypes.c_longlong),
        ("restarts", ctypes.c_int), ("floor_mask", ctypes.c_ulonglong), ("orth_fallbacks", ctypes.c_int),
    ]


class PcxLanczosOpts(ctypes.Structure):
    _fields_ = [
        ("tol_outer", ctypes.c_double), ("tol_inner", ctypes.c_double), ("max_steps", ctypes.c_int),
        ("max_cg", ctypes.c_int), ("seed", ctypes.c_ulonglong),
    ]


class PcxLanczosStats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int), ("cg_iterations", ctypes.c_longlong), ("matvecs", ctypes.c_longlong),
        ("seconds", ctypes.c_double), ("residual", ctypes.c_double * PCX_MAX_BLOCK), ("converged", ctypes.c_int),
    ]


class PcxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcx error {code}: {msg}")
        self.code = code


# (name, restype, argtypes)
_SIGS = [
    ("pcx_geometry", ctypes.c_int, [c_double9, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(PcxGeom)]),
    ("pcx_kappa_from_bloch", ctypes.c_int, [c_double9, c_double3, c_double3]),
    ("pcx_plan_create", ctypes.c_int, [ctypes.POINTER(PcxGeom), ctypes.c_int, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    ("pcx_plan_destroy", None, [ctypes.c_void_p]),
    ("pcx_plan_set_eps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    ("pcx_plan_set_variant", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("pcx_apply_Ar", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int]),
    ("pcx_lanczos_opts_default", None, [ctypes.POINTER(PcxLanczosOpts)]),
    ("pcx_solve_lanczos", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.POINTER(PcxLanczosOpts),
                                          ctypes.c_void_p, ctypes.POINTER(PcxLanczosStats)]),
    ("pcx_apply_precond", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int]),
    ("pcx_apply_curl", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int]),
    ("pcx_hfield", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int]),
    ("pcx_apply_hfield_operator", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_int]),
    ("pcx_omega", ctypes.c_int, [c_double9, ctypes.POINTER(PcxGeom), c_double9]),
    ("pcx_apply_Ar_noalloc", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int]),
    ("pcx_apply_Ar_multi", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]),
    ("pcx_solve_batch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    ("pcx_plan_autotune", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    ("pcx_apply_QS", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int]),
    ("pcx_apply_QS_adjoint", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int]),
    ("pcx_eigvec", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int]),
    ("pcx_block_gram", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_long, ctypes.c_int, ctypes.c_void_p]),
    ("pcx_block_combine", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_long]),
    ("pcx_opts_default", None, [ctypes.POINTER(PcxOpts)]),
    ("pcx_solve", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.POINTER(PcxOpts),
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(PcxStats)]),
    ("pcx_grad_eps", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int]),
    ("pcx_time_Ar_kernels", ctypes.c_int, [ctypes.c_void_p, c_double3, ctypes.c_int, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int, ctypes.c_int, c_double3]),
    ("pcx_last_error", ctypes.c_char_p, []),
]

EXPORTED = [s[0] for s in _SIGS]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpcx.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1806_10284_amd.build`")
    try:
        # torch first: its HIP runtime is then the one the library binds to, so device memory and
        # streams from torch are valid in the library's calls
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != PCX_OK:
        msg = load().pcx_last_error()
        raise PcxError(code, msg.decode() if msg else "")
    return code
