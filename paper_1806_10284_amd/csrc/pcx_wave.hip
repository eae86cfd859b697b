// Register-resident plane kernels for 64 x 64 planes in FP32 (the FCC / BCC 64^3 workloads).
//
// The same A_r factors as the other plane kernels (W of Section 5.1, the y and z passes of
// Algorithm 5.2 with their twiddles, and the reverse order with conjugate twiddles for
// Algorithm 5.1), arranged for the wavefront instead of for the work-group:
//
//   * a length-64 line is held by 8 lanes with 8 values each (lane q: elements q + 8m), so both
//     radix-8 passes of a 64-point transform run on registers; between them the 8 lanes of the
//     line exchange their pass-1 outputs through LDS rows owned by the wavefront (no work-group
//     barrier: a wavefront's LDS instructions execute in order);
//   * the work-group (8 wavefronts, 64 lines) holds one 64 x 64 plane of ONE field component in
//     LDS at a time, for the single row <-> column exchange between the z and y transforms; the
//     three components go through it in turn with two barriers each;
//   * W is formed per mode from FP64 per-plane tables (the same formula and tables as the
//     LDS-staged kernels), so the only global reads of a block are its own input: the forward
//     kernel reads y once and mixes all three components at the start, keeping them in
//     registers; the adjoint reads each component's input one component ahead of its use, keeps
//     the three transformed components (the first in LDS, 32 KB, so that the mixing does not spill
//     registers) and mixes them at the end.
//
// LDS layout (pslot below): rows of kLD = 72 complex (64 used), row a shifted by 2 ((a mod 8) / 2)
// slots.  Every row write and every column read of a quarter wavefront then falls in 16 distinct
// 8-byte slot classes (slot mod 16), each lane's eight addresses are one base plus immediate
// offsets, and wavefront w's rows 8w .. 8w + 7 (576 slots) double as its exchange region (xslot).
#include "pcx_plane_tables.h"

namespace pcx {

namespace {

constexpr int kN = 64;
constexpr int kNP = kN * kN;
constexpr int kNT = 512;
constexpr int kLD = 72;
constexpr int kXSlots = 8 * kLD;

DEV int pslot(int a, int b) { return a * kLD + b + (((a & 7) >> 1) << 1); }

// a wavefront's exchange region: line gl, lane index a, value b (writing lanes: a = lane, b = value;
// reading lanes: b = lane, a = value), each pattern conflict-free within a quarter wavefront
DEV int xslot(int gl, int a, int b) { return 72 * gl + 9 * a + b; }

DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of a block: the plane, the per-plane twiddles (FP32) and the FP64 tables of W
struct WaveLds {
    cx<float> pl[kN * kLD];
    cx<float> twz[kN], twy[kN], twb[kN], twc[kN];
    cx<double> halfz[kN], rowz[kN], lamy[kN], d10[kN];
    double a01[kN], p10[kN];
};

// the table layout p3_setup / p3_w expect, pointing into WaveLds
struct LdsView {
    cx<float>* twz; cx<float>* twy; cx<float>* twb; cx<float>* twc;
    cx<double>* halfz; cx<double>* rowz; cx<double>* lamy; cx<double>* d10;
    double* a01; double* p10;
    DEV explicit LdsView(WaveLds& s)
        : twz(s.twz), twy(s.twy), twb(s.twb), twc(s.twc), halfz(s.halfz), rowz(s.rowz), lamy(s.lamy), d10(s.d10),
          a01(s.a01), p10(s.p10) {}
};

// One length-64 transform with sign S of the line held by the 8 lanes (gl, 0..7): on entry lane q
// holds element q + 8m in v[m]; on return it holds output q + 8c in v[c].  tw64[m] = exp(2 pi i m / 64).
template <int S>
DEV void line64(cx<float> v[8], const cx<float>* tw64, cx<float>* __restrict__ xb, int gl, int q) {
    Bfly<float, 8>::run(v, S);
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        const cx<float> w = tw64[(q * c) & (kN - 1)];
        v[c] = S > 0 ? cmul(v[c], w) : cmulc(v[c], w);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) xb[xslot(gl, q, c)] = v[c];
    wave_sync();
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = xb[xslot(gl, a, q)];
    wave_sync();
    Bfly<float, 8>::run(v, S);
}

// exp(2 pi i c phi3(i, j)) = twc[c] exp(-2 pi i (c j s3 mod 4096) / 4096)
DEV cx<float> ztw(const cx<float>* twc, const cx<float>* __restrict__ rot, int c, int j, int s3m) {
    return cmul(twc[c], rot[(c * j * s3m) & (kNP - 1)]);
}

DEV KSel grid_k(const Grid& g) {
    KSel ks;
    ks.kap[0] = g.kap[0];
    ks.kap[1] = g.kap[1];
    ks.kap[2] = g.kap[2];
    ks.codes = g.codes;
    return ks;
}

}  // namespace

// y: [v][2][n1][64][64] -> t: [v][3][n1][c][b]; grid (n1, nvec).  TI: the input's precision (FP64
// input is rounded to FP32 as it is read: the FP64 solver's preconditioner)
template <typename TI>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(4)))
k_w64_fwd(Grid g, DeviceTables tb, const cx<TI>* __restrict__ y, cx<float>* __restrict__ t) {
    __shared__ WaveLds S;
    const LdsView L(S);
    const int i = blockIdx.x, v = blockIdx.y;
    const int tid = threadIdx.x, w = tid >> 6, gl = (tid >> 3) & 7, q = tid & 7;
    const long n = (long)g.n1 * kNP;
    // this lane's modes in the z phase: row j, k = q + 8m
    const int j = 8 * w + gl;
    const long mb = (long)i * kNP + j * kN + q;
    const cx<TI>* y1 = y + (long)v * 2 * n + mb;
    const unsigned char* codes = g.codes + mb;
    cx<float> a[8], b[8];
    int code[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const cx<TI> ya = y1[8 * m], yb = y1[n + 8 * m];
        a[m] = mk<float>((float)ya.x, (float)ya.y);
        b[m] = mk<float>((float)yb.x, (float)yb.y);
        code[m] = codes[8 * m];
    }
    const cx<double> L0 = p3_setup<float, kN, kN, kNT>(g, grid_k(g), tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    int s3m = g.s3 % kNP;
    if (s3m < 0) s3m += kNP;
    __syncthreads();
    // u_l = W_l1 y1 + W_l2 y2 for the three components
    cx<float> u[3][8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        if (code[m] == kMasked) {
            u[0][m] = u[1][m] = u[2][m] = mk<float>(0.0f, 0.0f);
        } else {
            cx<float> W[3][2];
            p3_w<float, kN, kN>(L, L0, j, q + 8 * m, code[m], idz, W);
#pragma unroll
            for (int l = 0; l < 3; ++l) u[l][m] = cmul(W[l][0], a[m]) + cmul(W[l][1], b[m]);
        }
    }
    cx<float> zt[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) zt[c] = ztw(S.twc, tb.rot32, q + 8 * c, j, s3m);   // column q + 8c of row j
    cx<float>* xb = S.pl + w * kXSlots;
    const int col = 8 * w + gl;                            // this lane's column in the y phase
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        line64<+1>(u[l], S.twz, xb, gl, q);
#pragma unroll
        for (int c = 0; c < 8; ++c) S.pl[pslot(j, q + 8 * c)] = cmul(u[l][c], zt[c]);
        __syncthreads();
        cx<float> x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = S.pl[pslot(q + 8 * m, col)];
        __syncthreads();
        line64<+1>(x, S.twy, xb, gl, q);
        cx<float>* out = t + ((long)v * 3 + l) * n + (long)i * kNP + col * kN + q;
#pragma unroll
        for (int c = 0; c < 8; ++c) out[8 * c] = cmul(x[c], S.twb[q + 8 * c]);
    }
}

// t: [v][3][n1][c][b] -> z: [v][2][n1][64][64]; grid (n1, nvec).  TO: the output's precision; scale
// (n values or null): a per-mode factor applied in FP64 on the way out (the FP64 solver's
// preconditioner writes D z in FP64)
template <typename TO>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(4)))
k_w64_adj(Grid g, DeviceTables tb, const cx<float>* __restrict__ t, cx<TO>* __restrict__ z,
          const double* __restrict__ scale) {
    __shared__ WaveLds S;
    const LdsView L(S);
    const int i = blockIdx.x, v = blockIdx.y;
    const int tid = threadIdx.x, w = tid >> 6, gl = (tid >> 3) & 7, q = tid & 7;
    const long n = (long)g.n1 * kNP;
    const int col = 8 * w + gl;                            // column of the y phase
    const int j = 8 * w + gl;                              // row of the z phase
    const long mb = (long)i * kNP + j * kN + q;            // modes (j, q + 8c) of the z phase
    const cx<float>* src = t + (long)v * 3 * n + (long)i * kNP + col * kN + q;
    cx<float> tin[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) tin[m] = src[8 * m];
    const cx<double> L0 = p3_setup<float, kN, kN, kNT>(g, grid_k(g), tb, i, L);
    int s3m = g.s3 % kNP;
    if (s3m < 0) s3m += kNP;
    __syncthreads();
    cx<float> zt[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) zt[c] = ztw(S.twc, tb.rot32, col, q + 8 * c, s3m);   // row q + 8c of column col
    cx<float>* xb = S.pl + w * kXSlots;
    // the z-phase outputs of the three components; component 0 waits in LDS for the final mixing
    // (32 KB), which otherwise runs out of registers beside the FP64 formation of W
    cx<float> sl[3][8];
    __shared__ cx<float> park[8][kNT];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        cx<float> x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = cmulc(tin[m], S.twb[q + 8 * m]);
        if (l < 2) {      // the next component's input, in flight during this component
#pragma unroll
            for (int m = 0; m < 8; ++m) tin[m] = src[(long)(l + 1) * n + 8 * m];
        }
        line64<-1>(x, S.twy, xb, gl, q);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 8; ++c) S.pl[pslot(q + 8 * c, col)] = cmulc(x[c], zt[c]);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) sl[l][m] = S.pl[pslot(j, q + 8 * m)];
        line64<-1>(sl[l], S.twz, xb, gl, q);
        if (l == 0) {
#pragma unroll
            for (int c = 0; c < 8; ++c) park[c][tid] = sl[0][c];
        }
    }
    // z = W^H s per mode
    const unsigned char* codes = g.codes + mb;
    const double idz = 1.0 / g.dlt[2];
    cx<TO>* zb = z + (long)v * 2 * n + mb;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int code = codes[8 * c];
        cx<float> a1 = mk<float>(0.0f, 0.0f), a2 = a1;
        if (code != kMasked) {
            cx<float> W[3][2];
            p3_w<float, kN, kN>(L, L0, j, q + 8 * c, code, idz, W);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const cx<float> sv = l == 0 ? park[c][tid] : sl[l][c];
                a1 = a1 + cmulc(sv, W[l][0]);
                a2 = a2 + cmulc(sv, W[l][1]);
            }
        }
        const double d = scale ? scale[mb + 8 * c] : 1.0;
        zb[8 * c] = mk<TO>((TO)(d * (double)a1.x), (TO)(d * (double)a1.y));
        zb[n + 8 * c] = mk<TO>((TO)(d * (double)a2.x), (TO)(d * (double)a2.y));
    }
}

bool wave_plane_available(const Grid& g, int fp64) {
    return !fp64 && g.n2 == kN && g.n3 == kN && g.nvk == 0;
}

hipError_t launch_wave_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<float>* y, cx<float>* t, int nvec,
                                 hipStream_t st) {
    PCX_LAUNCH(k_w64_fwd<float>, dim3(g.n1, nvec), dim3(kNT), 0, st, g, tb, y, t);
    return hipGetLastError();
}

hipError_t launch_wave_plane_adj(const Grid& g, const DeviceTables& tb, const cx<float>* t, cx<float>* z, int nvec,
                                 hipStream_t st) {
    PCX_LAUNCH(k_w64_adj<float>, dim3(g.n1, nvec), dim3(kNT), 0, st, g, tb, t, z, (const double*)nullptr);
    return hipGetLastError();
}

hipError_t launch_wave_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<double>* y, cx<float>* t, int nvec,
                                 hipStream_t st) {
    PCX_LAUNCH(k_w64_fwd<double>, dim3(g.n1, nvec), dim3(kNT), 0, st, g, tb, y, t);
    return hipGetLastError();
}

hipError_t launch_wave_plane_adj(const Grid& g, const DeviceTables& tb, const cx<float>* t, cx<double>* z,
                                 const double* scale, int nvec, hipStream_t st) {
    PCX_LAUNCH(k_w64_adj<double>, dim3(g.n1, nvec), dim3(kNT), 0, st, g, tb, t, z, scale);
    return hipGetLastError();
}

}  // namespace pcx
