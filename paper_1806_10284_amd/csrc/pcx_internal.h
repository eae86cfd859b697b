// Internal declarations shared by the HIP kernels and the host-side plan/solver.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcx.h"

namespace pcx {

// Kernel timing for the measurement hook: while a host thread has `start`/`stop` set, the A_r
// kernels it launches record them at their own start and end on the device (hipExtLaunchKernel),
// so the interval is the kernel's execution alone, as a profiler reports it.  Null: plain launch.
struct LaunchTimer {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchTimer g_launch_timer;
#define PCX_LAUNCH(kernel, grid, block, shmem, stream, ...)                                                  \
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, g_launch_timer.start, g_launch_timer.stop, 0, \
                          __VA_ARGS__)

constexpr int kMaxPasses = 8;
constexpr double kMixTau = 1e-3;   // switch to the fallback range basis below Lambda_p^2 / Lambda_q

// Mixed-radix Stockham factorisation of one axis (radices 8, 4, 2, 3, 5).
struct FftPlan {
    int n;
    int npass;
    int rad[kMaxPasses];
};

// Everything a matvec kernel needs about the grid and the Bloch phases.
struct Grid {
    int n1, n2, n3;
    int s1, s2, s3;          // signed shifts of the lattice rows in grid units
    double kap[3];           // kappa_l = k . a_l
    double dlt[3];           // mesh sizes
    FftPlan fx, fy, fz;
    const unsigned char* codes;  // mixing basis per mode (launch_modecode), n bytes
    // per precision [0] FP32, [1] FP64:
    int generic[2];          // 1: runtime-sized kernels only; 0: fixed-size kernels where they exist
    int plane_nt[2];         // generic plane kernels' work-group size: 0 automatic, 256 / 512 / 1024
    int fixed_kind[2];       // fixed-size plane kernels: 0 automatic (register kernels where they
                             // apply, else three-plane or two-plane), 3 three-plane only, 2 two-plane
                             // only, 4 register kernels where they apply
    int split[2];            // 1: plane too large for LDS, two passes through a second 3n-per-vector
                             //    workspace that follows the first one
    // several wave vectors in one launch: vectors are ordered [k][v] with nvk vectors per wave
    // vector; kaps (device, 3 per k) and codes (n bytes per k) then replace kap and codes
    int nvk;
    const double* kaps;
    // W of every mode for this kappa ([0] FP32, [1] FP64; layout [2l + c][i][j][k], c the column
    // of the 3 x 2 matrix, zero on the masked mode), or null: the fixed-size plane kernels then
    // form W per mode and vector.  Only the FP32 table is built, and only the adjoint plane
    // kernels read it: measured at 64^3, 32 vectors, it takes the FP32 adjoint from 153 to 134 us
    // (plane i runs on XCD i mod 8, so each XCD's eighth of the table stays in its L2 across the
    // vectors), leaves the forward kernels unchanged and slows the FP64 adjoint (96 B per mode)
    const void* wtab[2];
};

template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R x, y;
};

// device-side tables owned by a plan: twiddle LUTs exp(+2 pi i m / N) for the three axes,
// in both precisions, the half-turn table exp(i pi k / n3) in FP64, and the (n2 n3)-th roots
// of unity exp(-2 pi i m / (n2 n3)) in both precisions.
struct DeviceTables {
    cx<double>* tw64[3];
    cx<float>* tw32[3];
    cx<double>* halfz;
    cx<double>* rot64;
    cx<float>* rot32;
};

// ---- launchers (pcx_fft.hip) ----
// z = A_r y for nvec vectors; t is a 3n-per-vector workspace.
template <typename R>
hipError_t launch_apply_Ar(const Grid& g, const DeviceTables& tb, const R* inv_eps_n, const cx<R>* y,
                           cx<R>* z, cx<R>* t, int nvec, hipStream_t st);
// the three launches of launch_apply_Ar, `reps` times, with HIP events around each launch on `st`;
// ms[0..2] = mean milliseconds of the plane-forward, x-line and plane-adjoint kernels
template <typename R>
hipError_t time_apply_Ar(const Grid& g, const DeviceTables& tb, const R* inv_eps_n, const cx<R>* y, cx<R>* z,
                         cx<R>* t, int nvec, int reps, hipStream_t st, double ms[3]);
// u = (I3 (x) T)(W y) (scale_eps == nullptr) or x = B^{-1}(I3 (x) T)(W y) (scale_eps = 1/eps)
template <typename R>
hipError_t launch_QS(const Grid& g, const DeviceTables& tb, const R* inv_eps, const cx<R>* y, cx<R>* u,
                     cx<R>* t, int nvec, hipStream_t st);
// z = W^H (I3 (x) T*) u
template <typename R>
hipError_t launch_QS_adjoint(const Grid& g, const DeviceTables& tb, const cx<R>* u, cx<R>* z, cx<R>* t,
                             int nvec, hipStream_t st);
// mixing-basis code per mode for the grid's kappa (n bytes): decided once in FP64
hipError_t launch_modecode(const Grid& g, unsigned char* out, hipStream_t st);
// 1/Lambda_q per mode (0 at the masked mode), FP64, n values
hipError_t launch_precond_diag(const Grid& g, const DeviceTables& tb, double* out, hipStream_t st);
// set per-kernel LDS limits once per process
hipError_t configure_kernels();
// planes too large for LDS at this precision take the two-pass plane path; its LDS need
bool split_plane_needed(int n2, int n3, int fp64);
size_t split_kernel_lds(int n2, int n3, int fp64);

// ---- fixed-size kernels (pcx_fixed.hip) ----
// Each launcher sets *done when it has a kernel for the grid (and launched it), else leaves the
// work to the generic kernels.
template <typename R>
hipError_t launch_fixed_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<R>* y, cx<R>* t, int nvec,
                                  hipStream_t st, bool* done);
template <typename R>
hipError_t launch_fixed_plane_adj(const Grid& g, const DeviceTables& tb, const cx<R>* t, cx<R>* z, int nvec,
                                  hipStream_t st, bool* done);
template <typename R>
hipError_t launch_fixed_xline(const Grid& g, const DeviceTables& tb, const R* scale, cx<R>* t, int nvec,
                              hipStream_t st, bool* done);
// kind: 0 any, 3 the three-plane kernels, 2 the two-plane kernels
bool fixed_plane_available(int n2, int n3, int fp64, int kind = 0);
// W of every mode (the Grid's wtab layout) for a grid with fixed-size plane kernels
template <typename R>
hipError_t launch_wtable(const Grid& g, const DeviceTables& tb, cx<R>* out, hipStream_t st, bool* done);
bool fixed_xline_available(int n1, long np, int fp64);
// register-resident plane kernels (pcx_wave.hip): FP32 64 x 64 planes, n1 % 8 == 0, one wave vector,
// the FP32 W table present
bool wave_plane_available(const Grid& g, int fp64);
hipError_t launch_wave_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<float>* y, cx<float>* t, int nvec,
                                 hipStream_t st);
hipError_t launch_wave_plane_adj(const Grid& g, const DeviceTables& tb, const cx<float>* t, cx<float>* z, int nvec,
                                 hipStream_t st);
// the same kernels with FP64 input (forward) and FP64 output scaled per mode (adjoint, scale: n values)
hipError_t launch_wave_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<double>* y, cx<float>* t, int nvec,
                                 hipStream_t st);
hipError_t launch_wave_plane_adj(const Grid& g, const DeviceTables& tb, const cx<float>* t, cx<double>* z,
                                 const double* scale, int nvec, hipStream_t st);
// z = diag(scale) A_r(eps) y with FP64 y and z and the FP32 register kernels in between (the FP64
// solver's preconditioner); hipErrorNotSupported where the register kernels do not apply
hipError_t launch_precond_mixed(const Grid& g, const DeviceTables& tb, const float* epsn32, const cx<double>* y,
                                cx<double>* z, cx<float>* t, const double* scale, int nvec, hipStream_t st);
hipError_t configure_fixed_kernels();

// ---- block operations (pcx_block.hip) ----
// A set of vectors of length N given as up to kMaxSeg runs of contiguous columns (column stride N).
constexpr int kMaxSeg = 8;
struct ColSet {
    void* ptr[kMaxSeg];
    int ncols[kMaxSeg];
    __host__ __device__ int total() const {
        int t = 0;
        for (int s = 0; s < kMaxSeg; ++s) t += ncols[s];
        return t;
    }
};
inline ColSet colset(void* p0, int c0, void* p1 = nullptr, int c1 = 0, void* p2 = nullptr, int c2 = 0) {
    ColSet s;
    for (int q = 0; q < kMaxSeg; ++q) {
        s.ptr[q] = nullptr;
        s.ncols[q] = 0;
    }
    s.ptr[0] = p0; s.ncols[0] = c0;
    s.ptr[1] = p1; s.ncols[1] = c1;
    s.ptr[2] = p2; s.ncols[2] = c2;
    return s;
}
// [A | B]: the runs of A followed by the runs of B (at most kMaxSeg non-empty runs in total)
inline ColSet concat(const ColSet& A, const ColSet& B) {
    ColSet s = colset(nullptr, 0);
    int q = 0;
    for (const ColSet* x : {&A, &B})
        for (int r = 0; r < kMaxSeg; ++r)
            if (x->ncols[r] > 0 && q < kMaxSeg) {
                s.ptr[q] = x->ptr[r];
                s.ncols[q] = x->ncols[r];
                ++q;
            }
    return s;
}

// out (ka x kb, row-major) = A^H B with FP64 accumulation; part: workspace of (nchunk + 32) * ka * kb
// complex.  herm: B = [A] or [A | A'] (kb = ka or 2 ka) with every ka x ka half Hermitian; only the
// entries whose register blocks lie on or above the block diagonal of each half are written, the
// rest must be mirrored by the caller (mirror_upper does it on the host).
template <typename R>
hipError_t launch_gram(const ColSet& A, const ColSet& B, long N, cx<double>* part, int nchunk, cx<double>* out,
                       hipStream_t st, bool herm = false);
// Y[:, m] = sum_k S[:, k] C[k, m]  (C: ks x m row-major FP64 complex, device).  Y must not
// overlap S.
template <typename R>
hipError_t launch_combine(const ColSet& S, const cx<double>* C, const ColSet& Y, long N, hipStream_t st);
// R_j = AX_j - theta_j X_j ; W_j = prec .* R_j (prec: n doubles, applied to both y-blocks; nullptr = identity);
// out[j] = ||R_j||^2 (FP64).  theta: HOST array of X.total() <= PCX_MAX_BLOCK shifts, passed to the kernel
// by value (no copy to the device).
struct Shifts {
    double v[PCX_MAX_BLOCK];
};
template <typename R>
hipError_t launch_residual(const ColSet& X, const ColSet& AX, const double* theta, const double* prec, long n,
                           const ColSet& W, double* part, int nchunk, double* out, hipStream_t st);
// precision conversion of a contiguous complex array
hipError_t launch_convert(const cx<float>* in, cx<double>* out, long count, hipStream_t st);
hipError_t launch_convert(const cx<double>* in, cx<float>* out, long count, hipStream_t st);
// zero the masked mode: y *= (prec != 0) on both y-blocks of nvec vectors
template <typename R>
hipError_t launch_mask(cx<R>* y, const double* prec, long n, int nvec, hipStream_t st);
// out = prec * in per mode on both y-blocks of nvec vectors (out may equal in)
template <typename R>
hipError_t launch_scale_modes(const cx<R>* in, cx<R>* out, const double* prec, long n, int nvec, hipStream_t st);
// the same from FP32 into FP64
hipError_t launch_scale_modes(const cx<float>* in, cx<double>* out, const double* prec, long n, int nvec,
                              hipStream_t st);
// y = a x + b y over count complex FP64 entries
hipError_t launch_axpby(const cx<double>* x, cx<double>* y, cx<double> a, cx<double> b, long count, hipStream_t st);
// *out = a^H b over count complex FP64 entries; part: device, at least 1024 entries of scratch
hipError_t launch_dot(const cx<double>* a, const cx<double>* b, long count, cx<double>* part, cx<double>* out,
                      hipStream_t st);
// out = sqrt(in), count doubles
hipError_t launch_sqrt(const double* in, double* out, long count, hipStream_t st);
// grad[p] = -sum_t w_t |x_t(p)|^2 ; voxel: summed over the 3 components.  w: device, nvec doubles.
hipError_t launch_grad(const cx<double>* x, const double* w, int nvec, long n, double* grad, int voxel,
                       hipStream_t st);

// the discrete curl C of Section 3 (adjoint: C^*) on nvec 3n-vectors in the e-layout (real-space
// stencils with the quasi-periodic wraps); in and out must not overlap
template <typename R>
hipError_t launch_curl(const Grid& g, const cx<R>* in, cx<R>* out, int nvec, bool adjoint, hipStream_t st);
// x[v][q] *= s[q] for q < n3 (a 3n-long real scaling such as 1/eps)
template <typename R>
hipError_t launch_scale3(const R* s, cx<R>* x, long n3, int nvec, hipStream_t st);

// seeded complex normal deviates times `scale` (counter-based: element e of stream `seed`)
template <typename R>
hipError_t launch_random(cx<R>* y, long count, unsigned long long seed, double scale, hipStream_t st);
// y[idx[c]] = 1 for c < count (count <= PCX_MAX_BLOCK); the indices travel as a kernel argument
struct UnitList {
    long long idx[PCX_MAX_BLOCK];
    int count;
};
template <typename R>
hipError_t launch_set_units(cx<R>* y, const UnitList& u, hipStream_t st);
hipError_t configure_block_kernels();

// sizes used by the plan to reserve LDS and workspaces
size_t plane_kernel_lds(int n2, int n3, int fp64);
size_t xline_kernel_lds(int n1, int fp64);
int xline_kernel_tile(int n1);

}  // namespace pcx
