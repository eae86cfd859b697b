// Fixed-size variants of the A_r kernels for the grid sizes of the standard workloads.
//
// Same mathematics as the generic kernels (Algorithms 5.1 and 5.2 around W of Section 5.1), with
// two changes that matter on gfx950, where the generic kernels are limited by VALU issue rather
// than by HBM:
//   * every transform length, line count and stride is a compile-time constant, so all index
//     arithmetic of the Stockham passes folds into shifts, masks and multiply-high;
//   * the plane kernels stage the three field components of one plane together (three planes in
//     LDS), so W of a mode is formed once per vector instead of once per component, and the three
//     transforms of a pass share their barriers.
// The x-line kernel keeps one component in LDS at a time (no W there) with a fixed line length.
#include "pcx_dev.h"
#include "pcx_plane_tables.h"

namespace pcx {

// ------------------------------------------------------------------ compile-time radix plan
struct RadPlan {
    int np;
    int r[kMaxPasses];
};

constexpr RadPlan rad_plan(int n) {
    RadPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    int m = n;
    while (m % 8 == 0) { p.r[p.np++] = 8; m /= 8; }
    while (m % 4 == 0) { p.r[p.np++] = 4; m /= 4; }
    while (m % 2 == 0) { p.r[p.np++] = 2; m /= 2; }
    while (m % 3 == 0) { p.r[p.np++] = 3; m /= 3; }
    while (m % 5 == 0) { p.r[p.np++] = 5; m /= 5; }
    return p;
}

// One Stockham pass over NL lines of length N in LDS, in place.  Line L lies at
// (L / LG) * GS + (L % LG) * LS and its element m at m * ES from there.  Butterfly
// b = tid + t NT -> (line b % NL, j = b / NL): neighbouring lanes work on neighbouring lines.
// Inputs j + r N/RAD, twiddle exp(sign 2 pi i r (j mod NS) / (NS RAD)), outputs
// (j / NS) NS RAD + (j mod NS) + r NS.  tw[m] = exp(+2 pi i m / N).
template <typename R, int N, int RAD, int NS, int NL, int LG, int GS, int LS, int ES, int NT, int SIGN>
DEV void fpass(cx<R>* __restrict__ buf, const cx<R>* __restrict__ tw) {
    constexpr int NR = N / RAD;
    constexpr int B = NL * NR;
    constexpr int PER = (B + NT - 1) / NT;
    constexpr int TWS = N / (NS * RAD);
    cx<R> v[PER][RAD];
    int base[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int b = threadIdx.x + t * NT;
        if (B % NT == 0 || b < B) {
            const int L = b % NL, j = b / NL;
            const int k = j % NS;
            base[t] = (L / LG) * GS + (L % LG) * LS + ((j / NS) * NS * RAD + k) * ES;
            const cx<R>* src = buf + (L / LG) * GS + (L % LG) * LS + j * ES;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[t][r] = src[r * NR * ES];
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    cx<R> w = tw[r * k * TWS];
                    if (SIGN < 0) w.y = -w.y;
                    v[t][r] = cmul(v[t][r], w);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int b = threadIdx.x + t * NT;
        if (B % NT == 0 || b < B) {
            Bfly<R, RAD>::run(v[t], SIGN);
            cx<R>* dst = buf + base[t];
#pragma unroll
            for (int r = 0; r < RAD; ++r) dst[r * NS * ES] = v[t][r];
        }
    }
    __syncthreads();
}

template <typename R, int N, int NL, int LG, int GS, int LS, int ES, int NT, int SIGN, int P = 0, int NS = 1>
DEV void ffft(cx<R>* buf, const cx<R>* tw) {
    constexpr RadPlan rp = rad_plan(N);
    if constexpr (P < rp.np) {
        constexpr int RAD = rp.r[P];
        fpass<R, N, RAD, NS, NL, LG, GS, LS, ES, NT, SIGN>(buf, tw);
        ffft<R, N, NL, LG, GS, LS, ES, NT, SIGN, P + 1, NS * RAD>(buf, tw);
    }
}

// ------------------------------------------------------------------ three-plane LDS layout
// planes  cx<R>[3][N2][N3 + 1]
// twz     cx<R>[N3]  exp(+2 pi i m / N3)       twy  cx<R>[N2]  exp(+2 pi i m / N2)
// twb     cx<R>[N2]  exp(2 pi i b phi2(i))     twc  cx<R>[N3]  exp(2 pi i c A(i))
// FP64 (16-byte aligned):
// halfz   [N3]  exp(i pi k / N3)               rowz [N2]  exp(i pi phi3(i, j))
// lamy    [N2]  Lambda_2(i, j)                 d10  [N2]  Lambda_2 - Lambda_1
// a01     [N2]  |Lambda_1|^2 + |Lambda_2|^2    p10  [N2]  |Lambda_2 - Lambda_1|^2
template <typename R, int N2, int N3>
struct P3 {
    static constexpr int LD = N3 + 1;
    static constexpr int PS = N2 * LD;
    static constexpr int NP = N2 * N3;
    static constexpr size_t kRbytes = sizeof(cx<R>) * (3 * (size_t)PS + 2 * N3 + 2 * N2);
    static constexpr size_t kRpad = (kRbytes + 15) & ~(size_t)15;
    static constexpr size_t bytes = kRpad + sizeof(cx<double>) * (N3 + 3 * N2) + sizeof(double) * 2 * N2;

    cx<R>* pl;
    cx<R>* twz;
    cx<R>* twy;
    cx<R>* twb;
    cx<R>* twc;
    cx<double>* halfz;
    cx<double>* rowz;
    cx<double>* lamy;
    cx<double>* d10;
    double* a01;
    double* p10;

    DEV P3(char* base) {
        pl = (cx<R>*)base;
        twz = pl + 3 * PS;
        twy = twz + N3;
        twb = twy + N2;
        twc = twb + N2;
        halfz = (cx<double>*)(base + kRpad);
        rowz = halfz + N3;
        lamy = rowz + N2;
        d10 = lamy + N2;
        a01 = (double*)(d10 + N2);
        p10 = a01 + N2;
    }
};

// ------------------------------------------------------------------ plane kernels
// y: [v][2][n1][N2][N3]  ->  t: [v][3][n1][N3][N2];   grid (n1, nvec)
template <typename R, int N2, int N3, int NT, bool WT>
__global__ void __launch_bounds__(NT) k_p3_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ y,
                                                cx<R>* __restrict__ t) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    using LT = P3<R, N2, N3>;
    constexpr int LD = LT::LD, PS = LT::PS, NP = LT::NP;
    constexpr int EPT = (NP + NT - 1) / NT;
    extern __shared__ __align__(16) char lds[];
    const LT L(lds);
    const int i = blockIdx.x, v = blockIdx.y;
    const long n = (long)g.n1 * NP;
    const cx<R>* yb = y + (long)v * 2 * n + (long)i * NP;
    const unsigned char* codes = ks.codes + (long)i * NP;
    const cx<R>* wt = WT ? (const cx<R>*)g.wtab[sizeof(R) == 8] : nullptr;
    cx<R> y1[EPT], y2[EPT];
    int code[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            y1[s] = yb[e];
            y2[s] = yb[n + e];
            code[s] = WT ? 0 : codes[e];
        }
    }
    const cx<double> L0 = p3_setup<R, N2, N3, NT>(g, ks, tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    int s3m = g.s3 % NP;
    if (s3m < 0) s3m += NP;
    __syncthreads();
    // u_l = W_l1 y1 + W_l2 y2 into plane l at [j][k]
    cx<R> tw[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, k = e % N3;
            tw[s] = p3_ztw<R, N2, N3>(L, rot, k, j, s3m);
            cx<R> u[3];
            if constexpr (WT) {
                cx<R> w[3][2];
                mode_w<R, N2, N3, true>(wt, n, (long)i * NP + e, L, L0, j, k, 0, idz, w);
#pragma unroll
                for (int l = 0; l < 3; ++l) u[l] = cmul(w[l][0], y1[s]) + cmul(w[l][1], y2[s]);
            } else if (code[s] == kMasked) {
                u[0] = u[1] = u[2] = mk<R>((R)0, (R)0);
            } else {
                cx<R> w[3][2];
                p3_w<R, N2, N3>(L, L0, j, k, code[s], idz, w);
#pragma unroll
                for (int l = 0; l < 3; ++l) u[l] = cmul(w[l][0], y1[s]) + cmul(w[l][1], y2[s]);
            }
#pragma unroll
            for (int l = 0; l < 3; ++l) L.pl[l * PS + j * LD + k] = u[l];
        }
    }
    __syncthreads();
    // z inverse DFT along the 3 N2 rows (uniform line stride LD across the three planes)
    ffft<R, N3, 3 * N2, 3 * N2, 0, LD, 1, NT, +1>(L.pl, L.twz);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, c = e % N3;
#pragma unroll
            for (int l = 0; l < 3; ++l) L.pl[l * PS + j * LD + c] = cmul(L.pl[l * PS + j * LD + c], tw[s]);
        }
    }
    __syncthreads();
    // y inverse DFT along the columns c of each plane
    ffft<R, N2, 3 * N3, N3, PS, 1, LD, NT, +1>(L.pl, L.twy);
    // t[v][l][i][c][b] = plane_l[b][c] exp(2 pi i b phi2)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        cx<R>* out = t + ((long)v * 3 + l) * n + (long)i * NP;
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (NP % NT == 0 || e < NP) {
                const int c = e / N2, b = e % N2;
                out[e] = cmul(L.pl[l * PS + b * LD + c], L.twb[b]);
            }
        }
    }
}

// t: [v][3][n1][N3][N2]  ->  z: [v][2][n1][N2][N3]
template <typename R, int N2, int N3, int NT, bool WT>
__global__ void __launch_bounds__(NT) k_p3_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ t,
                                                cx<R>* __restrict__ z) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    using LT = P3<R, N2, N3>;
    constexpr int LD = LT::LD, PS = LT::PS, NP = LT::NP;
    constexpr int EPT = (NP + NT - 1) / NT;
    extern __shared__ __align__(16) char lds[];
    const LT L(lds);
    const int i = blockIdx.x, v = blockIdx.y;
    const long n = (long)g.n1 * NP;
    cx<R> in[3][EPT];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const cx<R>* src = t + ((long)v * 3 + l) * n + (long)i * NP;
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (NP % NT == 0 || e < NP) in[l][s] = src[e];
        }
    }
    const cx<double> L0 = p3_setup<R, N2, N3, NT>(g, ks, tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    int s3m = g.s3 % NP;
    if (s3m < 0) s3m += NP;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int c = e / N2, b = e % N2;
            const cx<R> wb = L.twb[b];
#pragma unroll
            for (int l = 0; l < 3; ++l) L.pl[l * PS + b * LD + c] = cmulc(in[l][s], wb);
        }
    }
    __syncthreads();
    ffft<R, N2, 3 * N3, N3, PS, 1, LD, NT, -1>(L.pl, L.twy);      // b -> j along columns c
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, c = e % N3;
            const cx<R> tw = p3_ztw<R, N2, N3>(L, rot, c, j, s3m);
#pragma unroll
            for (int l = 0; l < 3; ++l) L.pl[l * PS + j * LD + c] = cmulc(L.pl[l * PS + j * LD + c], tw);
        }
    }
    __syncthreads();
    ffft<R, N3, 3 * N2, 3 * N2, 0, LD, 1, NT, -1>(L.pl, L.twz);   // c -> k along rows j
    const unsigned char* codes = ks.codes + (long)i * NP;
    const cx<R>* wt = WT ? (const cx<R>*)g.wtab[sizeof(R) == 8] : nullptr;
    cx<R>* zb = z + (long)v * 2 * n + (long)i * NP;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, k = e % N3;
            const int code = WT ? 0 : (int)codes[e];
            cx<R> a1 = mk<R>((R)0, (R)0), a2 = a1;
            if (WT || code != kMasked) {
                cx<R> w[3][2];
                if constexpr (WT) mode_w<R, N2, N3, true>(wt, n, (long)i * NP + e, L, L0, j, k, 0, idz, w);
                else p3_w<R, N2, N3>(L, L0, j, k, code, idz, w);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const cx<R> u = L.pl[l * PS + j * LD + k];
                    a1 = a1 + cmulc(u, w[l][0]);
                    a2 = a2 + cmulc(u, w[l][1]);
                }
            }
            zb[e] = a1;
            zb[n + e] = a2;
        }
    }
}

// ------------------------------------------------------------------ two-plane variant
// Two plane buffers instead of three: components 0 and 1 go through the LDS transforms together
// while component 2's mixed values wait in registers (forward), or its W^H row waits in registers
// (adjoint).  W is still formed once per mode and vector.  Half a 64 x 64 FP32 group's LDS (two
// groups per CU), and the only layout in which FP64 64 x 64 planes fit.
template <typename R, int N2, int N3>
struct P2 {
    static constexpr int LD = N3 + 1;
    static constexpr int PS = N2 * LD;
    static constexpr int NP = N2 * N3;
    static constexpr size_t kRbytes = sizeof(cx<R>) * (2 * (size_t)PS + 2 * N3 + 2 * N2);
    static constexpr size_t kRpad = (kRbytes + 15) & ~(size_t)15;
    static constexpr size_t bytes = kRpad + sizeof(cx<double>) * (N3 + 3 * N2) + sizeof(double) * 2 * N2;

    cx<R>* pl;
    cx<R>* twz;
    cx<R>* twy;
    cx<R>* twb;
    cx<R>* twc;
    cx<double>* halfz;
    cx<double>* rowz;
    cx<double>* lamy;
    cx<double>* d10;
    double* a01;
    double* p10;

    DEV P2(char* base) {
        pl = (cx<R>*)base;
        twz = pl + 2 * PS;
        twy = twz + N3;
        twb = twy + N2;
        twc = twb + N2;
        halfz = (cx<double>*)(base + kRpad);
        rowz = halfz + N3;
        lamy = rowz + N2;
        d10 = lamy + N2;
        a01 = (double*)(d10 + N2);
        p10 = a01 + N2;
    }
};

// the table itself: one work-group per plane i, W of its N2 N3 modes in precision R
template <typename R, int N2, int N3, int NT>
__global__ void __launch_bounds__(NT) k_wtable(Grid g, DeviceTables tb, cx<R>* __restrict__ out) {
    using LT = P2<R, N2, N3>;
    constexpr int NP = LT::NP;
    extern __shared__ __align__(16) char lds[];
    const LT L(lds);
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    const int i = blockIdx.x;
    const long n = (long)g.n1 * NP;
    const cx<double> L0 = p3_setup<R, N2, N3, NT>(g, ks, tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    __syncthreads();
    const unsigned char* codes = ks.codes + (long)i * NP;
    for (int e = threadIdx.x; e < NP; e += NT) {
        cx<R> w[3][2];
        mode_w<R, N2, N3, false>((const cx<R>*)nullptr, n, 0, L, L0, e / N3, e % N3, codes[e], idz, w);
#pragma unroll
        for (int q = 0; q < 6; ++q) out[(long)q * n + (long)i * NP + e] = w[q >> 1][q & 1];
    }
}

// z then y inverse transforms of NPL planes starting at plane 0, z-twiddles from registers
template <typename R, int N2, int N3, int NT, int NPL, int EPT>
DEV void p2_forward_planes(const P2<R, N2, N3>& L, const cx<R> tw[EPT]) {
    constexpr int LD = N3 + 1, PS = N2 * LD, NP = N2 * N3;
    ffft<R, N3, NPL * N2, NPL * N2, 0, LD, 1, NT, +1>(L.pl, L.twz);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, c = e % N3;
#pragma unroll
            for (int l = 0; l < NPL; ++l) L.pl[l * PS + j * LD + c] = cmul(L.pl[l * PS + j * LD + c], tw[s]);
        }
    }
    __syncthreads();
    ffft<R, N2, NPL * N3, N3, PS, 1, LD, NT, +1>(L.pl, L.twy);
}

template <typename R, int N2, int N3, int NT, bool WT>
__global__ void __launch_bounds__(NT) k_p2_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ y,
                                                cx<R>* __restrict__ t) {
    using LT = P2<R, N2, N3>;
    constexpr int LD = LT::LD, PS = LT::PS, NP = LT::NP;
    constexpr int EPT = (NP + NT - 1) / NT;
    extern __shared__ __align__(16) char lds[];
    const LT L(lds);
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    const int i = blockIdx.x, v = blockIdx.y;
    const long n = (long)g.n1 * NP;
    const cx<R>* yb = y + (long)v * 2 * n + (long)i * NP;
    const unsigned char* codes = ks.codes + (long)i * NP;
    const cx<R>* wt = WT ? (const cx<R>*)g.wtab[sizeof(R) == 8] : nullptr;
    cx<R> y1[EPT], y2[EPT];
    int code[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            y1[s] = yb[e];
            y2[s] = yb[n + e];
            code[s] = WT ? 0 : codes[e];
        }
    }
    const cx<double> L0 = p3_setup<R, N2, N3, NT>(g, ks, tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    int s3m = g.s3 % NP;
    if (s3m < 0) s3m += NP;
    __syncthreads();
    cx<R> tw[EPT], u2[EPT];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, k = e % N3;
            tw[s] = p3_ztw<R, N2, N3>(L, rot, k, j, s3m);
            cx<R> u[3];
            if constexpr (WT) {
                cx<R> w[3][2];
                mode_w<R, N2, N3, true>(wt, n, (long)i * NP + e, L, L0, j, k, 0, idz, w);
#pragma unroll
                for (int l = 0; l < 3; ++l) u[l] = cmul(w[l][0], y1[s]) + cmul(w[l][1], y2[s]);
            } else if (code[s] == kMasked) {
                u[0] = u[1] = u[2] = mk<R>((R)0, (R)0);
            } else {
                cx<R> w[3][2];
                p3_w<R, N2, N3>(L, L0, j, k, code[s], idz, w);
#pragma unroll
                for (int l = 0; l < 3; ++l) u[l] = cmul(w[l][0], y1[s]) + cmul(w[l][1], y2[s]);
            }
            L.pl[j * LD + k] = u[0];
            L.pl[PS + j * LD + k] = u[1];
            u2[s] = u[2];
        }
    }
    __syncthreads();
    p2_forward_planes<R, N2, N3, NT, 2, EPT>(L, tw);
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        cx<R>* out = t + ((long)v * 3 + l) * n + (long)i * NP;
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (NP % NT == 0 || e < NP) {
                const int c = e / N2, b = e % N2;
                out[e] = cmul(L.pl[l * PS + b * LD + c], L.twb[b]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) L.pl[(e / N3) * LD + e % N3] = u2[s];
    }
    __syncthreads();
    p2_forward_planes<R, N2, N3, NT, 1, EPT>(L, tw);
    cx<R>* out = t + ((long)v * 3 + 2) * n + (long)i * NP;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int c = e / N2, b = e % N2;
            out[e] = cmul(L.pl[b * LD + c], L.twb[b]);
        }
    }
}

// load components [l0, l0 + NPL) of t into the planes (conjugate y-twiddle), y then z forward
// transforms with the conjugate z-twiddle in between
template <typename R, int N2, int N3, int NT, int NPL>
DEV void p2_adjoint_planes(const P2<R, N2, N3>& L, const cx<R>* __restrict__ t, long n, int v, int i, int l0,
                           const cx<R>* __restrict__ rot, int s3m) {
    constexpr int LD = N3 + 1, PS = N2 * LD, NP = N2 * N3;
    constexpr int EPT = (NP + NT - 1) / NT;
#pragma unroll
    for (int l = 0; l < NPL; ++l) {
        const cx<R>* src = t + ((long)v * 3 + l0 + l) * n + (long)i * NP;
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (NP % NT == 0 || e < NP) {
                const int c = e / N2, b = e % N2;
                L.pl[l * PS + b * LD + c] = cmulc(src[e], L.twb[b]);
            }
        }
    }
    __syncthreads();
    ffft<R, N2, NPL * N3, N3, PS, 1, LD, NT, -1>(L.pl, L.twy);
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, c = e % N3;
            const cx<R> tw = p3_ztw<R, N2, N3>(L, rot, c, j, s3m);
#pragma unroll
            for (int l = 0; l < NPL; ++l) L.pl[l * PS + j * LD + c] = cmulc(L.pl[l * PS + j * LD + c], tw);
        }
    }
    __syncthreads();
    ffft<R, N3, NPL * N2, NPL * N2, 0, LD, 1, NT, -1>(L.pl, L.twz);
}

// FP32: at most 128 registers per lane (4 waves per SIMD), so two 512-thread groups share a CU
template <typename R, int N2, int N3, int NT, bool WT>
__global__ void __launch_bounds__(NT, sizeof(R) == 4 ? 4 : 1) k_p2_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ t,
                                                cx<R>* __restrict__ z) {
    using LT = P2<R, N2, N3>;
    constexpr int LD = LT::LD, PS = LT::PS, NP = LT::NP;
    constexpr int EPT = (NP + NT - 1) / NT;
    extern __shared__ __align__(16) char lds[];
    const LT L(lds);
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    const int i = blockIdx.x, v = blockIdx.y;
    const long n = (long)g.n1 * NP;
    const cx<double> L0 = p3_setup<R, N2, N3, NT>(g, ks, tb, i, L);
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    int s3m = g.s3 % NP;
    if (s3m < 0) s3m += NP;
    __syncthreads();
    p2_adjoint_planes<R, N2, N3, NT, 2>(L, t, n, v, i, 0, rot, s3m);
    const unsigned char* codes = ks.codes + (long)i * NP;
    const cx<R>* wt = WT ? (const cx<R>*)g.wtab[sizeof(R) == 8] : nullptr;
    // FP32: W's third row is formed (or read) again at the end rather than held, so that the
    // group fits in 128 registers per lane (two groups per CU); FP64 groups are one per CU by
    // LDS anyway
    constexpr bool kHoldW2 = sizeof(R) == 8;
    constexpr int NW = kHoldW2 ? EPT : 1;
    cx<R> a1[EPT], a2[EPT], w2a[NW], w2b[NW];
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        a1[s] = a2[s] = mk<R>((R)0, (R)0);
        if (kHoldW2) w2a[s % NW] = w2b[s % NW] = mk<R>((R)0, (R)0);
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, k = e % N3;
            const int code = WT ? 0 : (int)codes[e];
            if (WT || code != kMasked) {
                cx<R> w[3][2];
                if constexpr (WT) mode_w<R, N2, N3, true>(wt, n, (long)i * NP + e, L, L0, j, k, 0, idz, w);
                else p3_w<R, N2, N3>(L, L0, j, k, code, idz, w);
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    const cx<R> u = L.pl[l * PS + j * LD + k];
                    a1[s] = a1[s] + cmulc(u, w[l][0]);
                    a2[s] = a2[s] + cmulc(u, w[l][1]);
                }
                if (kHoldW2) {
                    w2a[s % NW] = w[2][0];
                    w2b[s % NW] = w[2][1];
                }
            }
        }
    }
    __syncthreads();
    p2_adjoint_planes<R, N2, N3, NT, 1>(L, t, n, v, i, 2, rot, s3m);
    cx<R>* zb = z + (long)v * 2 * n + (long)i * NP;
#pragma unroll
    for (int s = 0; s < EPT; ++s) {
        const int e = threadIdx.x + s * NT;
        if (NP % NT == 0 || e < NP) {
            const int j = e / N3, k = e % N3;
            const cx<R> u = L.pl[j * LD + k];
            cx<R> wa = mk<R>((R)0, (R)0), wb = wa;
            if (kHoldW2) {
                wa = w2a[s % NW];
                wb = w2b[s % NW];
            } else if (WT) {
                wa = wt[4 * n + (long)i * NP + e];
                wb = wt[5 * n + (long)i * NP + e];
            } else {
                const int code = codes[e];
                if (code != kMasked) {
                    cx<R> w[3][2];
                    p3_w<R, N2, N3>(L, L0, j, k, code, idz, w);
                    wa = w[2][0];
                    wb = w[2][1];
                }
            }
            zb[e] = a1[s] + cmulc(u, wa);
            zb[n + e] = a2[s] + cmulc(u, wb);
        }
    }
}

// ------------------------------------------------------------------ x-line kernel
// Tile = TB consecutive (c, b) positions q, all N1 values of i, one component at a time:
// t -> x-IDFT -> * inv_eps / n -> x-DFT -> t (in place).  scale is in the [l][q][a] layout.
template <typename R, int N1, int TB, int NT>
__global__ void __launch_bounds__(NT) k_xl_fixed(Grid g, DeviceTables tb, const R* __restrict__ scale,
                                                  cx<R>* __restrict__ t) {
    constexpr int LDX = N1 + 1;
    constexpr int TOT = N1 * TB;
    constexpr int EPT = (TOT + NT - 1) / NT;
    extern __shared__ __align__(16) char lds[];
    cx<R>* buf = (cx<R>*)lds;
    cx<R>* twx = buf + TB * LDX;
    const long np = (long)g.n2 * g.n3;
    const long n = (long)N1 * np;
    const int v = blockIdx.y;
    const long q0 = (long)blockIdx.x * TB;
    const cx<R>* twx_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[0] : (const cx<R>*)tb.tw32[0];
    for (int a = threadIdx.x; a < N1; a += NT) twx[a] = twx_g[a];
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        cx<R>* tl = t + ((long)v * 3 + l) * n;
        const R* sl = scale + (long)l * n + q0 * N1;
        cx<R> val[EPT];
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (TOT % NT == 0 || e < TOT) val[s] = tl[(long)(e / TB) * np + q0 + e % TB];
        }
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (TOT % NT == 0 || e < TOT) buf[(e % TB) * LDX + e / TB] = val[s];
        }
        __syncthreads();
        ffft<R, N1, TB, TB, 0, LDX, 1, NT, +1>(buf, twx);     // i -> a
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (TOT % NT == 0 || e < TOT) {
                const int ql = e / N1, a = e % N1;
                buf[ql * LDX + a] = cscale(buf[ql * LDX + a], sl[e]);
            }
        }
        __syncthreads();
        ffft<R, N1, TB, TB, 0, LDX, 1, NT, -1>(buf, twx);     // a -> i
#pragma unroll
        for (int s = 0; s < EPT; ++s) {
            const int e = threadIdx.x + s * NT;
            if (TOT % NT == 0 || e < TOT) tl[(long)(e / TB) * np + q0 + e % TB] = buf[(e % TB) * LDX + e / TB];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ instantiation table
// Plane kernels: (N2, N3, threads).  Work-groups of up to 1024 threads, about 4 modes per thread.
#ifndef PCX_P3_NT64
#define PCX_P3_NT64 1024
#endif
#define PCX_P3_SIZES(X) \
    X(16, 16, 256)      \
    X(32, 32, 256)      \
    X(32, 40, 320)      \
    X(48, 40, 512)      \
    X(48, 48, 576)      \
    X(40, 40, 448)      \
    X(64, 64, PCX_P3_NT64)

// Two-plane kernels: (N2, N3, threads)
#define PCX_P2_SIZES(X) \
    X(64, 64, 512)

#ifndef PCX_XL_NT64
#define PCX_XL_NT64 512
#endif
// x-line kernels: (N1, tile, threads)
#define PCX_XL_SIZES(X) \
    X(16, 128, 256)     \
    X(32, 64, 256)      \
    X(40, 64, 256)      \
    X(48, 64, 256)      \
    X(60, 64, 256)      \
    X(64, 64, PCX_XL_NT64)  \
    X(128, 32, 256)

template <typename F>
static hipError_t lds_limit(F f) {
    return hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

constexpr size_t kLdsMax = 160 * 1024;

template <typename R>
static hipError_t p3_fwd(const Grid& g, const DeviceTables& tb, const cx<R>* y, cx<R>* t, int nvec,
                         hipStream_t st, bool* done) {
    *done = false;
    // automatic choice: the register kernels where they apply, else the two-plane kernel where
    // compiled (measured faster for the forward pass at 64 x 64), else the three-plane one
    const int kind0 = g.fixed_kind[sizeof(R) == 8];
    if constexpr (sizeof(R) == 4) {
        if ((kind0 == 0 || kind0 == 4) && wave_plane_available(g, 0)) {
            *done = true;
            return launch_wave_plane_fwd(g, tb, y, t, nvec, st);
        }
    }
    const int kind = kind0 == 4 ? 0 : kind0;     // register kernels not applicable: automatic choice
    if (kind == 2 || (kind == 0 && fixed_plane_available(g.n2, g.n3, sizeof(R) == 8, 2))) goto two;
#define X(A, B, T)                                                                                           \
    if (g.n2 == A && g.n3 == B && P3<R, A, B>::bytes <= kLdsMax) {                                          \
        PCX_LAUNCH((k_p3_fwd<R, A, B, T, false>), dim3(g.n1, nvec), dim3(T), (P3<R, A, B>::bytes), st, g, tb, y, t); \
        *done = true;                                                                                        \
        return hipGetLastError();                                                                            \
    }
    PCX_P3_SIZES(X)
#undef X
    if (kind == 3) return hipSuccess;
two:
#define X(A, B, T)                                                                                           \
    if (g.n2 == A && g.n3 == B && P2<R, A, B>::bytes <= kLdsMax) {                                          \
        PCX_LAUNCH((k_p2_fwd<R, A, B, T, false>), dim3(g.n1, nvec), dim3(T), (P2<R, A, B>::bytes), st, g, tb, y, t); \
        *done = true;                                                                                        \
        return hipGetLastError();                                                                            \
    }
    PCX_P2_SIZES(X)
#undef X
    return hipSuccess;
}

template <typename R>
static hipError_t p3_adj(const Grid& g, const DeviceTables& tb, const cx<R>* t, cx<R>* z, int nvec,
                         hipStream_t st, bool* done) {
    *done = false;
    const int kind0 = g.fixed_kind[sizeof(R) == 8];
    if constexpr (sizeof(R) == 4) {
        if ((kind0 == 0 || kind0 == 4) && wave_plane_available(g, 0)) {
            *done = true;
            return launch_wave_plane_adj(g, tb, t, z, nvec, st);
        }
    }
    const int kind = kind0 == 4 ? 0 : kind0;
    if (kind == 2) goto two;
#define X(A, B, T)                                                                                           \
    if (g.n2 == A && g.n3 == B && P3<R, A, B>::bytes <= kLdsMax) {                                          \
        if (g.wtab[sizeof(R) == 8])                                                                          \
            PCX_LAUNCH((k_p3_adj<R, A, B, T, true>), dim3(g.n1, nvec), dim3(T), (P3<R, A, B>::bytes), st, g, tb, t, z); \
        else                                                                                                 \
            PCX_LAUNCH((k_p3_adj<R, A, B, T, false>), dim3(g.n1, nvec), dim3(T), (P3<R, A, B>::bytes), st, g, tb, t, z); \
        *done = true;                                                                                        \
        return hipGetLastError();                                                                            \
    }
    PCX_P3_SIZES(X)
#undef X
    if (kind == 3) return hipSuccess;
two:
#define X(A, B, T)                                                                                           \
    if (g.n2 == A && g.n3 == B && P2<R, A, B>::bytes <= kLdsMax) {                                          \
        if (g.wtab[sizeof(R) == 8])                                                                          \
            PCX_LAUNCH((k_p2_adj<R, A, B, T, true>), dim3(g.n1, nvec), dim3(T), (P2<R, A, B>::bytes), st, g, tb, t, z); \
        else                                                                                                 \
            PCX_LAUNCH((k_p2_adj<R, A, B, T, false>), dim3(g.n1, nvec), dim3(T), (P2<R, A, B>::bytes), st, g, tb, t, z); \
        *done = true;                                                                                        \
        return hipGetLastError();                                                                            \
    }
    PCX_P2_SIZES(X)
#undef X
    return hipSuccess;
}

template <typename R>
static hipError_t xl_fixed(const Grid& g, const DeviceTables& tb, const R* scale, cx<R>* t, int nvec,
                           hipStream_t st, bool* done) {
    *done = false;
    const long np = (long)g.n2 * g.n3;
#define X(A, TBV, T)                                                                                         \
    if (g.n1 == A && np % TBV == 0) {                                                                        \
        const size_t lds = sizeof(cx<R>) * ((size_t)TBV * (A + 1) + A);                                      \
        if (lds <= kLdsMax) {                                                                                \
            PCX_LAUNCH((k_xl_fixed<R, A, TBV, T>), dim3((unsigned)(np / TBV), nvec), dim3(T), lds, st, g, \
                               tb, scale, t);                                                                \
            *done = true;                                                                                    \
            return hipGetLastError();                                                                        \
        }                                                                                                    \
    }
    PCX_XL_SIZES(X)
#undef X
    return hipSuccess;
}

template <typename R>
hipError_t launch_wtable(const Grid& g, const DeviceTables& tb, cx<R>* out, hipStream_t st, bool* done) {
    *done = false;
#define X(A, B, T)                                                                                           \
    if (g.n2 == A && g.n3 == B && P2<R, A, B>::bytes <= kLdsMax) {                                          \
        hipLaunchKernelGGL((k_wtable<R, A, B, T>), dim3(g.n1), dim3(T), (P2<R, A, B>::bytes), st, g, tb, out); \
        *done = true;                                                                                        \
        return hipGetLastError();                                                                            \
    }
    PCX_P3_SIZES(X)
#undef X
    return hipSuccess;
}

bool fixed_plane_available(int n2, int n3, int fp64, int kind) {
    if (kind != 2) {
#define X(A, B, T) \
    if (n2 == A && n3 == B && (fp64 ? P3<double, A, B>::bytes : P3<float, A, B>::bytes) <= kLdsMax) return true;
        PCX_P3_SIZES(X)
#undef X
    }
    if (kind != 3) {
#define X(A, B, T) \
    if (n2 == A && n3 == B && (fp64 ? P2<double, A, B>::bytes : P2<float, A, B>::bytes) <= kLdsMax) return true;
        PCX_P2_SIZES(X)
#undef X
    }
    return false;
}

bool fixed_xline_available(int n1, long np, int fp64) {
#define X(A, TBV, T)                                                                                         \
    if (n1 == A && np % TBV == 0)                                                                            \
        return (fp64 ? sizeof(cx<double>) : sizeof(cx<float>)) * ((size_t)TBV * (A + 1) + A) <= kLdsMax;
    PCX_XL_SIZES(X)
#undef X
    return false;
}

template <typename R>
hipError_t launch_fixed_plane_fwd(const Grid& g, const DeviceTables& tb, const cx<R>* y, cx<R>* t, int nvec,
                                  hipStream_t st, bool* done) {
    return p3_fwd<R>(g, tb, y, t, nvec, st, done);
}
template <typename R>
hipError_t launch_fixed_plane_adj(const Grid& g, const DeviceTables& tb, const cx<R>* t, cx<R>* z, int nvec,
                                  hipStream_t st, bool* done) {
    return p3_adj<R>(g, tb, t, z, nvec, st, done);
}
template <typename R>
hipError_t launch_fixed_xline(const Grid& g, const DeviceTables& tb, const R* scale, cx<R>* t, int nvec,
                              hipStream_t st, bool* done) {
    return xl_fixed<R>(g, tb, scale, t, nvec, st, done);
}

template <typename R>
static hipError_t fixed_limits() {
    hipError_t e = hipSuccess;
#define X(A, B, T)                                                                 \
    if (e == hipSuccess && P3<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p3_fwd<R, A, B, T, false>); \
    if (e == hipSuccess && P3<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p3_adj<R, A, B, T, false>); \
    if (e == hipSuccess && P3<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p3_adj<R, A, B, T, true>); \
    if (e == hipSuccess && P2<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_wtable<R, A, B, T>);
    PCX_P3_SIZES(X)
#undef X
#define X(A, B, T)                                                                 \
    if (e == hipSuccess && P2<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p2_fwd<R, A, B, T, false>); \
    if (e == hipSuccess && P2<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p2_adj<R, A, B, T, false>); \
    if (e == hipSuccess && P2<R, A, B>::bytes <= kLdsMax) e = lds_limit(k_p2_adj<R, A, B, T, true>);
    PCX_P2_SIZES(X)
#undef X
#define X(A, TBV, T) \
    if (e == hipSuccess) e = lds_limit(k_xl_fixed<R, A, TBV, T>);
    PCX_XL_SIZES(X)
#undef X
    return e;
}

hipError_t configure_fixed_kernels() {
    hipError_t e = fixed_limits<float>();
    if (e != hipSuccess) return e;
    return fixed_limits<double>();
}

template hipError_t launch_fixed_plane_fwd<float>(const Grid&, const DeviceTables&, const cx<float>*, cx<float>*,
                                                  int, hipStream_t, bool*);
template hipError_t launch_fixed_plane_fwd<double>(const Grid&, const DeviceTables&, const cx<double>*, cx<double>*,
                                                   int, hipStream_t, bool*);
template hipError_t launch_fixed_plane_adj<float>(const Grid&, const DeviceTables&, const cx<float>*, cx<float>*,
                                                  int, hipStream_t, bool*);
template hipError_t launch_fixed_plane_adj<double>(const Grid&, const DeviceTables&, const cx<double>*, cx<double>*,
                                                   int, hipStream_t, bool*);
template hipError_t launch_wtable<float>(const Grid&, const DeviceTables&, cx<float>*, hipStream_t, bool*);
template hipError_t launch_wtable<double>(const Grid&, const DeviceTables&, cx<double>*, hipStream_t, bool*);
template hipError_t launch_fixed_xline<float>(const Grid&, const DeviceTables&, const float*, cx<float>*, int,
                                              hipStream_t, bool*);
template hipError_t launch_fixed_xline<double>(const Grid&, const DeviceTables&, const double*, cx<double>*, int,
                                               hipStream_t, bool*);

}  // namespace pcx
