"""pcx: MI355X-native nullspace-free Maxwell eigensolver (Huang et al., arXiv:1806.10284).

The computation lives in libpcx.so (HIP kernels for gfx950 behind the C ABI of
include/pcx.h); ``api`` is a thin ctypes binding that passes torch device pointers
and the current stream.  Build with ``python -m paper_1806_10284_amd.build``.
"""
from ._lib import (PCX_EPS_VOXEL, PCX_EPS_YEE3, PCX_FP32, PCX_FP64, PCX_FP64_OP32, PCX_MODE_FP32, PCX_MODE_FP32_REFINE,
                   PCX_MODE_FP64, PCX_PRECOND_DIAG, PCX_PRECOND_INVERSE, PCX_PRECOND_NONE, PcxError)
from .api import Plan, geom_dict, pcx_geometry, pcx_kappa_from_bloch, pcx_omega, pcx_solve_batch

__all__ = [
    "Plan", "pcx_geometry", "pcx_kappa_from_bloch", "pcx_omega", "pcx_solve_batch", "geom_dict", "PcxError",
    "PCX_FP32", "PCX_FP64", "PCX_FP64_OP32", "PCX_EPS_YEE3", "PCX_EPS_VOXEL",
    "PCX_MODE_FP64", "PCX_MODE_FP32_REFINE", "PCX_MODE_FP32",
    "PCX_PRECOND_NONE", "PCX_PRECOND_DIAG", "PCX_PRECOND_INVERSE",
]
