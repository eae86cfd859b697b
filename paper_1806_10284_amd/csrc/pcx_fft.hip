// Nullspace-free matvec A_r y = W^H (I3 (x) T*) B^{-1} (I3 (x) T) W y on gfx950.
//
// T is the Fourier basis of Section 4.2 (eq. T): mode nu = (i,j,k) is the plane wave
// exp(i g.p), g = 2 pi t with turns
//     t_x = (kappa1 + i)/n1,  t_y = (kappa2 + j - s1 t_x)/n2,  t_z = (kappa3 + k - s2 t_x - s3 t_y)/n3,
// and T q is evaluated as in Algorithm 5.2: an inverse DFT along z, the twiddle
// exp(2 pi i c phi3(i,j)), an inverse DFT along y, the twiddle exp(2 pi i b phi2(i)), an
// inverse DFT along x and the twiddle exp(2 pi i a phi1), with
//     phi1 = kappa1/n1, phi2(i) = (kappa2 - s1 t_x)/n2, phi3(i,j) = (kappa3 - s2 t_x - s3 t_y)/n3.
// T* reverses the order with conjugate twiddles (Algorithm 5.1).  W (3 x 2 per mode) is the
// SVD factor Q_r Sigma_r of Section 5.1 (eqs. range_basis1/2).
//
// One matvec is three kernels over HBM-resident data:
//   k_plane_fwd  (plane i):   y -> W y -> z-IDFT -> twiddle -> y-IDFT -> twiddle  -> t[l][i][c][b]
//   k_xline      (x lines):   t -> x-IDFT -> (1/(n eps)) -> x-DFT                 -> t (in place)
//   k_plane_adj  (plane i):   t -> twiddle* -> y-DFT -> twiddle* -> z-DFT -> W^H   -> z
// The x twiddles exp(+-2 pi i a phi1) cancel around the diagonal 1/eps and are not applied.
// Every 1-D transform is a mixed-radix (8,4,2,3,5) Stockham FFT done in LDS by the whole
// work-group; every global read and write is coalesced along the unit-stride index.
#include "pcx_dev.h"

#include <vector>

namespace pcx {

thread_local LaunchTimer g_launch_timer;

// ------------------------------------------------------------------ Stockham pass in LDS
// nlines transforms of length N, element stride es and line stride ls (in elements), in place,
// by a work-group of NT threads.  Butterfly b -> (line = b % nlines, j = b / nlines) so
// neighbouring lanes touch neighbouring lines (unit stride for the strided axis).  Pass with
// radix RAD after the radices whose product is Ns (Stockham autosort): inputs j + r N/RAD,
// twiddle w^{r (j mod Ns)}, w = exp(sign 2 pi i / (Ns RAD)); outputs (j / Ns) Ns RAD + j mod Ns + r Ns.
template <typename R, int RAD, int MAXB, int NT>
DEV void stockham_pass(cx<R>* buf, int N, int Ns, int nlines, int es, int ls, const cx<R>* tw, int sign) {
    const int NR = N / RAD;
    const int total = NR * nlines;
    const int twstep = N / (Ns * RAD);
    // butterfly b = tid + t NT -> (line, j) = (b % nlines, b / nlines), advanced incrementally
    const int dj = NT / nlines, dl = NT % nlines;
    const int line0 = threadIdx.x % nlines, j0 = threadIdx.x / nlines;
    cx<R> v[MAXB][RAD];
    {
        int line = line0, j = j0;
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            if (threadIdx.x + t * NT < total) {
                const cx<R>* src = buf + line * ls + j * es;
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[t][r] = src[r * NR * es];
                const int k = j % Ns;
                if (k) {
#pragma unroll
                    for (int r = 1; r < RAD; ++r) {
                        cx<R> w = tw[r * k * twstep];
                        if (sign < 0) w.y = -w.y;
                        v[t][r] = cmul(v[t][r], w);
                    }
                }
            }
            line += dl;
            j += dj;
            if (line >= nlines) {
                line -= nlines;
                ++j;
            }
        }
    }
    __syncthreads();
    {
        int line = line0, j = j0;
#pragma unroll
        for (int t = 0; t < MAXB; ++t) {
            if (threadIdx.x + t * NT < total) {
                const int k = j % Ns;
                Bfly<R, RAD>::run(v[t], sign);
                cx<R>* dst = buf + line * ls + ((j / Ns) * Ns * RAD + k) * es;
#pragma unroll
                for (int r = 0; r < RAD; ++r) dst[r * Ns * es] = v[t][r];
            }
            line += dl;
            j += dj;
            if (line >= nlines) {
                line -= nlines;
                ++j;
            }
        }
    }
    __syncthreads();
}

// All nlines transforms, in chunks of lines so that each thread holds at most kEpc elements per
// pass (lines are independent, so a chunk runs all its passes before the next chunk starts).
constexpr int kEpc = 4;

template <typename R, int EPC, int NT>
DEV void fft_lines(cx<R>* buf, const FftPlan& fp, int nlines, int es, int ls, const cx<R>* tw, int sign) {
    const int lpc = (EPC * NT) / fp.n > 0 ? (EPC * NT) / fp.n : 1;
#pragma unroll 1
    for (int l0 = 0; l0 < nlines; l0 += lpc) {
        const int nl = nlines - l0 < lpc ? nlines - l0 : lpc;
        cx<R>* b0 = buf + l0 * ls;
        int Ns = 1;
#pragma unroll 1
        for (int p = 0; p < fp.npass; ++p) {
            const int rad = fp.rad[p];
            switch (rad) {
                case 8: stockham_pass<R, 8, (EPC + 7) / 8, NT>(b0, fp.n, Ns, nl, es, ls, tw, sign); break;
                case 4: stockham_pass<R, 4, (EPC + 3) / 4, NT>(b0, fp.n, Ns, nl, es, ls, tw, sign); break;
                case 2: stockham_pass<R, 2, (EPC + 1) / 2, NT>(b0, fp.n, Ns, nl, es, ls, tw, sign); break;
                case 3: stockham_pass<R, 3, (EPC + 2) / 3, NT>(b0, fp.n, Ns, nl, es, ls, tw, sign); break;
                default: stockham_pass<R, 5, (EPC + 4) / 5, NT>(b0, fp.n, Ns, nl, es, ls, tw, sign); break;
            }
            Ns *= rad;
        }
    }
}

// ------------------------------------------------------------------ plane set-up (shared by both plane kernels)
// LDS layout of a plane kernel (dynamic shared memory):
//   plane  cx<R>[n2 * (n3 + 1)]      row j (or b) has n3 (+1 pad) entries
//   twz    cx<R>[n3]  LUT exp(+2 pi i m / n3)
//   twy    cx<R>[n2]  LUT exp(+2 pi i m / n2)
//   twb    cx<R>[n2]  exp(2 pi i b phi2(i))
//   twc    cx<R>[n3]  exp(2 pi i c A(i)), the j-independent part of exp(2 pi i c phi3(i, j))
//   lamy   cx<double>[n2]  Lambda_2(i, j)
//   halfz  cx<double>[n3]  exp(i pi k / n3)
//   rowz   cx<double>[n2]  exp(i pi phi3(i, j))
// With t_y = (kappa2 + j - s1 t_x)/n2, phi3(i, j) = A(i) - s3 j / (n2 n3) where
// A(i) = (kappa3 - s2 t_x - s3 (kappa2 - s1 t_x) / n2) / n3, so
//   exp(2 pi i c phi3) = twc[c] * exp(-2 pi i ((c j s3) mod n2 n3) / (n2 n3))
// and the second factor is read from the plan's table of (n2 n3)-th roots of unity.
template <typename R>
struct PlaneLds {
    cx<R>* plane;
    cx<R>* twz;
    cx<R>* twy;
    cx<R>* twb;
    cx<R>* twc;
    cx<double>* lamy;
    cx<double>* halfz;
    cx<double>* rowz;
    double* phi3;
};

template <typename R>
__host__ DEV size_t plane_lds_bytes(int n2, int n3) {
    size_t b = sizeof(cx<R>) * ((size_t)n2 * (n3 + 1) + 2 * n3 + 2 * n2);
    b = (b + 15) & ~(size_t)15;
    b += sizeof(cx<double>) * (n3 + 2 * n2) + sizeof(double) * n2;
    return b;
}

template <typename R>
DEV PlaneLds<R> plane_lds(char* base, int n2, int n3) {
    PlaneLds<R> L;
    L.plane = (cx<R>*)base;
    L.twz = L.plane + (size_t)n2 * (n3 + 1);
    L.twy = L.twz + n3;
    L.twb = L.twy + n2;
    L.twc = L.twb + n2;
    size_t off = sizeof(cx<R>) * ((size_t)n2 * (n3 + 1) + 2 * n3 + 2 * n2);
    off = (off + 15) & ~(size_t)15;
    L.halfz = (cx<double>*)(base + off);
    L.rowz = L.halfz + n3;
    L.lamy = L.rowz + n2;
    L.phi3 = (double*)(L.lamy + n2);
    return L;
}

// Fills the tables for plane i; returns Lambda_1(i).
template <typename R, int NT>
DEV cx<double> plane_setup(const Grid& g, const KSel& ks, const DeviceTables& tb, int i, PlaneLds<R>& L) {
    const int n2 = g.n2, n3 = g.n3;
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const cx<R>* twz_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[2] : (const cx<R>*)tb.tw32[2];
    const cx<R>* twy_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[1] : (const cx<R>*)tb.tw32[1];
    const double phi2 = (ks.kap[1] - (double)g.s1 * tx) / (double)n2;
    const double Ai = ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ((ks.kap[1] - (double)g.s1 * tx) / (double)n2)) /
                      (double)n3;
    for (int q = threadIdx.x; q < n3; q += NT) {
        L.twz[q] = twz_g[q];
        L.halfz[q] = tb.halfz[q];
        L.twc[q] = cis_turns<R>((double)q * Ai);
    }
    for (int j = threadIdx.x; j < n2; j += NT) {
        L.twy[j] = twy_g[j];
        L.twb[j] = cis_turns<R>((double)j * phi2);
        const double ty = ((ks.kap[1] + (double)j) - (double)g.s1 * tx) / (double)n2;
        L.lamy[j] = lam_of_turn(ty, 1.0 / g.dlt[1]);
        const double p3 = ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ty) / (double)n3;
        L.phi3[j] = p3;
        double s, c;
        sincospi(p3, &s, &c);
        L.rowz[j] = mk<double>(c, s);
    }
    return lam_of_turn(tx, 1.0 / g.dlt[0]);
}

// Lambda_3 at mode (j, k) from exp(i pi t_z) = exp(i pi k / n3) exp(i pi phi3(i, j)) (FP64)
template <typename R>
DEV cx<double> lam_z(const PlaneLds<R>& L, int j, int k, double inv_dz) {
    const cx<double> h = cmul(L.halfz[k], L.rowz[j]);
    return lam_from_halfturn(h.y, h.x, inv_dz);
}

// exp(2 pi i c phi3(i, j)): FP64 as the product of the per-plane factor and a root of unity from
// the plan's table; FP32 by sincospif of the turn c phi3 reduced in FP64.
DEV cx<double> z_twiddle(const PlaneLds<double>& L, const cx<double>* __restrict__ rot, int c, int j, int s3, int M) {
    int m = (c * j * s3) % M;
    if (m < 0) m += M;
    return cmul(L.twc[c], rot[m]);
}
DEV cx<float> z_twiddle(const PlaneLds<float>& L, const cx<float>* __restrict__ rot, int c, int j, int s3, int M) {
    return cis_turns<float>((double)c * L.phi3[j]);
}

// ------------------------------------------------------------------ kernel 1: W y, then z and y inverse DFTs
// y: [v][2][n1][n2][n3]   ->   t: [v][3][n1][n3][n2];   grid (n1, nvec), NT threads.
// Each thread owns the modes e = tid + s NT (s < EPT): their y values and z-twiddles stay in
// registers for the three components.
template <typename R, int NT, int EPT>
__global__ void __launch_bounds__(NT) k_plane_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ y,
                                                   cx<R>* __restrict__ t) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    extern __shared__ __align__(16) char lds[];
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const int i = blockIdx.x;
    const int v = blockIdx.y;
    const long n = (long)n1 * n2 * n3;
    const int np = n2 * n3;
    const int ld = n3 + 1;
    PlaneLds<R> L = plane_lds<R>(lds, n2, n3);
    const cx<double> lamx = plane_setup<R, NT>(g, ks, tb, i, L);
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    const unsigned char* codes = ks.codes + (long)i * np;
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* yb = y + (long)v * 2 * n + (long)i * np;
    // modes per thread small enough: y and the z-twiddles of the owned modes stay in registers
    constexpr bool kRegY = sizeof(R) == 4 ? EPT <= 4 : EPT <= 8;
    constexpr int NY = kRegY ? EPT : 1;
    cx<R> y1[NY], y2[NY], tw[NY];
    if (kRegY) {
#pragma unroll
        for (int s = 0; s < NY; ++s) {
            const int e = threadIdx.x + s * NT;
            if (e < np) {
                y1[s] = yb[e];
                y2[s] = yb[n + e];
            }
        }
    }
    __syncthreads();
    if (kRegY) {
#pragma unroll
        for (int s = 0; s < NY; ++s) {
            const int e = threadIdx.x + s * NT;
            if (e < np) tw[s] = z_twiddle(L, rot, e % n3, e / n3, g.s3, np);
        }
    }
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        // u_l = W_l1 y1 + W_l2 y2 into the plane [j][k]
        if (kRegY) {
#pragma unroll
            for (int s = 0; s < NY; ++s) {
                const int e = threadIdx.x + s * NT;
                if (e < np) {
                    const int j = e / n3, k = e % n3;
                    const int code = codes[e];
                    cx<R> u = mk<R>((R)0, (R)0);
                    if (code != kMasked) {
                        cx<R> w1, w2;
                        w_row_code<R>(lamx, L.lamy[j], lam_z(L, j, k, idz), code, l, &w1, &w2);
                        u = cmul(w1, y1[s]) + cmul(w2, y2[s]);
                    }
                    L.plane[j * ld + k] = u;
                }
            }
        } else {
#pragma unroll 1
            for (int e = threadIdx.x; e < np; e += NT) {
                const int j = e / n3, k = e % n3;
                const int code = codes[e];
                cx<R> u = mk<R>((R)0, (R)0);
                if (code != kMasked) {
                    cx<R> w1, w2;
                    w_row_code<R>(lamx, L.lamy[j], lam_z(L, j, k, idz), code, l, &w1, &w2);
                    u = cmul(w1, yb[e]) + cmul(w2, yb[n + e]);
                }
                L.plane[j * ld + k] = u;
            }
        }
        __syncthreads();
        fft_lines<R, kEpc, NT>(L.plane, g.fz, n2, 1, ld, L.twz, +1);    // k -> c along rows j
        if (kRegY) {
#pragma unroll
            for (int s = 0; s < NY; ++s) {
                const int e = threadIdx.x + s * NT;
                if (e < np) {
                    const int j = e / n3, c = e % n3;
                    L.plane[j * ld + c] = cmul(L.plane[j * ld + c], tw[s]);
                }
            }
        } else {
#pragma unroll 1
            for (int e = threadIdx.x; e < np; e += NT) {
                const int j = e / n3, c = e % n3;
                L.plane[j * ld + c] = cmul(L.plane[j * ld + c], z_twiddle(L, rot, c, j, g.s3, np));
            }
        }
        __syncthreads();
        fft_lines<R, kEpc, NT>(L.plane, g.fy, n3, ld, 1, L.twy, +1);    // j -> b along columns c
        // write t[v][l][i][c][b] = plane[b][c] * exp(2 pi i b phi2)
        cx<R>* tb_out = t + ((long)v * 3 + l) * n + (long)i * np;
#pragma unroll 1
        for (int e = threadIdx.x; e < np; e += NT) {
            const int c = e / n2, b = e % n2;
            tb_out[e] = cmul(L.plane[b * ld + c], L.twb[b]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ kernel 3: y and z forward DFTs, then W^H
// t: [v][3][n1][n3][n2]  ->  z: [v][2][n1][n2][n3]
template <typename R, int NT, int EPT>
__global__ void __launch_bounds__(NT) k_plane_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ t,
                                                   cx<R>* __restrict__ z) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    extern __shared__ __align__(16) char lds[];
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const int i = blockIdx.x;
    const int v = blockIdx.y;
    const long n = (long)n1 * n2 * n3;
    const int np = n2 * n3;
    const int ld = n3 + 1;
    PlaneLds<R> L = plane_lds<R>(lds, n2, n3);
    const cx<double> lamx = plane_setup<R, NT>(g, ks, tb, i, L);
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    const unsigned char* codes = ks.codes + (long)i * np;
    __syncthreads();
    const double idz = 1.0 / g.dlt[2];
    constexpr bool kRegAcc = sizeof(R) == 4 ? EPT <= 4 : EPT <= 8;   // accumulators in registers
    constexpr int NA = kRegAcc ? EPT : 1;
    cx<R> acc1[NA], acc2[NA], tw[NA];
#pragma unroll
    for (int s = 0; s < NA; ++s) acc1[s] = acc2[s] = mk<R>((R)0, (R)0);
    if (kRegAcc) {
#pragma unroll
        for (int s = 0; s < NA; ++s) {
            const int e = threadIdx.x + s * NT;
            if (e < np) tw[s] = z_twiddle(L, rot, e % n3, e / n3, g.s3, np);
        }
    }
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const cx<R>* tin = t + ((long)v * 3 + l) * n + (long)i * np;
#pragma unroll 1
        for (int e = threadIdx.x; e < np; e += NT) {
            const int c = e / n2, b = e % n2;
            L.plane[b * ld + c] = cmulc(tin[e], L.twb[b]);
        }
        __syncthreads();
        fft_lines<R, kEpc, NT>(L.plane, g.fy, n3, ld, 1, L.twy, -1);    // b -> j along columns c
        if (kRegAcc) {
#pragma unroll
            for (int s = 0; s < NA; ++s) {
                const int e = threadIdx.x + s * NT;
                if (e < np) {
                    const int j = e / n3, c = e % n3;
                    L.plane[j * ld + c] = cmulc(L.plane[j * ld + c], tw[s]);
                }
            }
        } else {
#pragma unroll 1
            for (int e = threadIdx.x; e < np; e += NT) {
                const int j = e / n3, c = e % n3;
                L.plane[j * ld + c] = cmulc(L.plane[j * ld + c], z_twiddle(L, rot, c, j, g.s3, np));
            }
        }
        __syncthreads();
        fft_lines<R, kEpc, NT>(L.plane, g.fz, n2, 1, ld, L.twz, -1);    // c -> k along rows j
        if (kRegAcc) {
            // accumulate W^H v in registers
#pragma unroll
            for (int s = 0; s < NA; ++s) {
                const int e = threadIdx.x + s * NT;
                if (e < np) {
                    const int j = e / n3, k = e % n3;
                    const int code = codes[e];
                    if (code != kMasked) {
                        cx<R> w1, w2;
                        w_row_code<R>(lamx, L.lamy[j], lam_z(L, j, k, idz), code, l, &w1, &w2);
                        const cx<R> val = L.plane[j * ld + k];
                        acc1[s] = acc1[s] + cmulc(val, w1);
                        acc2[s] = acc2[s] + cmulc(val, w2);
                    }
                }
            }
        } else {
            // many modes per thread: accumulate in the (thread-private) output entries
            cx<R>* zb = z + (long)v * 2 * n + (long)i * np;
#pragma unroll 1
            for (int e = threadIdx.x; e < np; e += NT) {
                const int j = e / n3, k = e % n3;
                const int code = codes[e];
                cx<R> a1 = mk<R>((R)0, (R)0), a2 = a1;
                if (l > 0) {
                    a1 = zb[e];
                    a2 = zb[n + e];
                }
                if (code != kMasked) {
                    cx<R> w1, w2;
                    w_row_code<R>(lamx, L.lamy[j], lam_z(L, j, k, idz), code, l, &w1, &w2);
                    const cx<R> val = L.plane[j * ld + k];
                    a1 = a1 + cmulc(val, w1);
                    a2 = a2 + cmulc(val, w2);
                }
                zb[e] = a1;
                zb[n + e] = a2;
            }
        }
        __syncthreads();
    }
    if (kRegAcc) {
        cx<R>* zb = z + (long)v * 2 * n + (long)i * np;
#pragma unroll
        for (int s = 0; s < NA; ++s) {
            const int e = threadIdx.x + s * NT;
            if (e < np) {
                zb[e] = acc1[s];
                zb[n + e] = acc2[s];
            }
        }
    }
}

// ------------------------------------------------------------------ planes too large for LDS
// When one n2 x n3 plane does not fit in LDS (FP64 at 128 x 128), or would leave room for only one
// work-group per CU (FP32 planes above 80 KB), the plane kernels are split in two passes through an
// intermediate u[v][l][i][j][c] in HBM:
//   k_zpass_fwd (rows j0..j0+RB of plane i): W y -> z-IDFT -> z-twiddle -> u
//   k_ypass_fwd (columns c0..c0+CB):          u -> y-IDFT -> y-twiddle -> t[l][i][c][b]
//   k_ypass_adj / k_zpass_adj: the reverse, with W^H summed over l.
// The row passes hold the three components of their rows in LDS together, so W of a mode is
// formed once for all three, and each thread keeps one column c: the twiddle index c j s3 mod
// n2 n3 advances by a fixed step from row to row instead of taking a modulo per element.
constexpr int kSplitModes = 1024;   // modes per row block and component (FP32; half in FP64): about
                                    // 30 KB of LDS, five work-groups per CU

static int split_rows(int n2, int n3, bool fp64) {
    int rb = (kSplitModes / (fp64 ? 2 : 1)) / n3;
    if (rb > n2) rb = n2;
    return rb < 1 ? 1 : rb;
}
static int split_cols(int n3) { return n3 < 16 ? n3 : 16; }

template <typename R>
__host__ DEV size_t zpass_lds_bytes(int rb, int n3) {
    size_t b = sizeof(cx<R>) * ((size_t)3 * rb * (n3 + 1) + 2 * n3);
    b = (b + 15) & ~(size_t)15;
    return b + sizeof(cx<double>) * (n3 + 2 * rb);
}
template <typename R>
__host__ DEV size_t ypass_lds_bytes(int cb, int n2) {
    return sizeof(cx<R>) * ((size_t)cb * (n2 + 1) + 2 * n2);
}

// per-row tables of rows j0.. of plane i; returns Lambda_1(i)
template <typename R>
DEV cx<double> zpass_setup(const Grid& g, const KSel& ks, const DeviceTables& tb, int i, int j0, int rows,
                           cx<R>* twz, cx<R>* twc, cx<double>* halfz, cx<double>* rowz, cx<double>* lamy) {
    const int n2 = g.n2, n3 = g.n3;
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const double Ai = ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ((ks.kap[1] - (double)g.s1 * tx) / (double)n2)) /
                      (double)n3;
    const cx<R>* twz_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[2] : (const cx<R>*)tb.tw32[2];
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
        twz[q] = twz_g[q];
        halfz[q] = tb.halfz[q];
        twc[q] = cis_turns<R>((double)q * Ai);
    }
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const int j = j0 + r;
        const double ty = ((ks.kap[1] + (double)j) - (double)g.s1 * tx) / (double)n2;
        lamy[r] = lam_of_turn(ty, 1.0 / g.dlt[1]);
        const double p3 = ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ty) / (double)n3;
        double sn, cs;
        sincospi(p3, &sn, &cs);
        rowz[r] = mk<double>(cs, sn);
    }
    return lam_of_turn(tx, 1.0 / g.dlt[0]);
}

// the thread's column and first row of a row pass (n3 <= 256 = blockDim.x), and the z-twiddle
// index (c j s3 mod M) of that first row with its step from row to row (all below 2^24: c, j < 256,
// M <= 65536)
struct RowWalk {
    int c, r0, rstep;
    bool active;
    unsigned idx, step;
};
DEV RowWalk row_walk(int n3, int j0, int s3m, int M) {
    RowWalk w;
    w.rstep = (int)blockDim.x / n3 > 0 ? (int)blockDim.x / n3 : 1;
    w.c = (int)threadIdx.x % n3;
    w.r0 = (int)threadIdx.x / n3;
    w.active = (int)threadIdx.x < w.rstep * n3;
    const unsigned uc = (unsigned)w.c, um = (unsigned)M;
    w.idx = (uc * (((unsigned)(j0 + w.r0) * (unsigned)s3m) % um)) % um;
    w.step = (uc * (((unsigned)w.rstep * (unsigned)s3m) % um)) % um;
    return w;
}

template <typename R>
__global__ void __launch_bounds__(256) k_zpass_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ y,
                                                    cx<R>* __restrict__ u, int RB) {
    extern __shared__ __align__(16) char lds[];
    const int n2 = g.n2, n3 = g.n3, ld = n3 + 1;
    const long n = (long)g.n1 * n2 * n3, np = (long)n2 * n3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, j0 = blockIdx.z * RB;
    const int rows = min(RB, n2 - j0);
    cx<R>* buf = (cx<R>*)lds;                       // component l, row r at (l RB + r) ld
    cx<R>* twz = buf + (size_t)3 * RB * ld;
    cx<R>* twc = twz + n3;
    size_t off = (sizeof(cx<R>) * ((size_t)3 * RB * ld + 2 * n3) + 15) & ~(size_t)15;
    cx<double>* halfz = (cx<double>*)(lds + off);
    cx<double>* rowz = halfz + n3;
    cx<double>* lamy = rowz + RB;
    const cx<double> L0 = zpass_setup<R>(g, ks, tb, i, j0, rows, twz, twc, halfz, rowz, lamy);
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    const int M = n2 * n3;
    int s3m = g.s3 % M;
    if (s3m < 0) s3m += M;
    const double idz = 1.0 / g.dlt[2];
    const long base = (long)i * np + (long)j0 * n3;
    const cx<R>* y1 = y + (long)v * 2 * n + base;
    const cx<R>* y2 = y1 + n;
    const unsigned char* codes = ks.codes + base;
    RowWalk wk = row_walk(n3, j0, s3m, M);
    const int c = wk.c;
    __syncthreads();
    // u_l = W_l1 y1 + W_l2 y2 for the three components, W formed once per mode
    if (wk.active) {
        for (int r = wk.r0; r < rows; r += wk.rstep) {
            const int e = r * n3 + c;
            const int code = codes[e];
            cx<R> u3[3] = {mk<R>((R)0, (R)0), mk<R>((R)0, (R)0), mk<R>((R)0, (R)0)};
            if (code != kMasked) {
                const cx<double> h = cmul(halfz[c], rowz[r]);
                const cx<double> L2 = lam_from_halfturn(h.y, h.x, idz);
                const cx<R> a = y1[e], b = y2[e];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    cx<R> w1, w2;
                    w_row_code<R>(L0, lamy[r], L2, code, l, &w1, &w2);
                    u3[l] = cmul(w1, a) + cmul(w2, b);
                }
            }
#pragma unroll
            for (int l = 0; l < 3; ++l) buf[(l * RB + r) * ld + c] = u3[l];
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < 3; ++l) fft_lines<R, kEpc, 256>(buf + (size_t)l * RB * ld, g.fz, rows, 1, ld, twz, +1);
    cx<R>* ub = u + (long)v * 3 * n + base;
    if (wk.active) {
        unsigned idx = wk.idx;
        for (int r = wk.r0; r < rows; r += wk.rstep) {
            const cx<R> tw = cmul(twc[c], rot[idx]);
#pragma unroll
            for (int l = 0; l < 3; ++l) ub[(long)l * n + r * n3 + c] = cmul(buf[(l * RB + r) * ld + c], tw);
            idx += wk.step;
            if (idx >= (unsigned)M) idx -= (unsigned)M;
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ypass_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ u,
                                                    cx<R>* __restrict__ t, int CB) {
    extern __shared__ __align__(16) char lds[];
    const int n2 = g.n2, n3 = g.n3, ld = n2 + 1;
    const long n = (long)g.n1 * n2 * n3, np = (long)n2 * n3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, c0 = blockIdx.z * CB;
    const int cols = min(CB, n3 - c0);
    cx<R>* buf = (cx<R>*)lds;
    cx<R>* twy = buf + (size_t)CB * ld;
    cx<R>* twb = twy + n2;
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const double phi2 = (ks.kap[1] - (double)g.s1 * tx) / (double)n2;
    const cx<R>* twy_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[1] : (const cx<R>*)tb.tw32[1];
    for (int b = threadIdx.x; b < n2; b += blockDim.x) {
        twy[b] = twy_g[b];
        twb[b] = cis_turns<R>((double)b * phi2);
    }
    const int tot = n2 * cols;
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const cx<R>* ul = u + ((long)v * 3 + l) * n + (long)i * np;
        __syncthreads();
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int j = e / cols, q = e % cols;
            buf[q * ld + j] = ul[(long)j * n3 + c0 + q];
        }
        __syncthreads();
        fft_lines<R, kEpc, 256>(buf, g.fy, cols, 1, ld, twy, +1);
        cx<R>* tl = t + ((long)v * 3 + l) * n + (long)i * np + (long)c0 * n2;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int q = e / n2, b = e % n2;
            tl[e] = cmul(buf[q * ld + b], twb[b]);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ypass_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ t,
                                                    cx<R>* __restrict__ u, int CB) {
    extern __shared__ __align__(16) char lds[];
    const int n2 = g.n2, n3 = g.n3, ld = n2 + 1;
    const long n = (long)g.n1 * n2 * n3, np = (long)n2 * n3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, c0 = blockIdx.z * CB;
    const int cols = min(CB, n3 - c0);
    cx<R>* buf = (cx<R>*)lds;
    cx<R>* twy = buf + (size_t)CB * ld;
    cx<R>* twb = twy + n2;
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const double phi2 = (ks.kap[1] - (double)g.s1 * tx) / (double)n2;
    const cx<R>* twy_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[1] : (const cx<R>*)tb.tw32[1];
    for (int b = threadIdx.x; b < n2; b += blockDim.x) {
        twy[b] = twy_g[b];
        twb[b] = cis_turns<R>((double)b * phi2);
    }
    const int tot = n2 * cols;
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const cx<R>* tl = t + ((long)v * 3 + l) * n + (long)i * np + (long)c0 * n2;
        __syncthreads();
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int q = e / n2, b = e % n2;
            buf[q * ld + b] = cmulc(tl[e], twb[b]);
        }
        __syncthreads();
        fft_lines<R, kEpc, 256>(buf, g.fy, cols, 1, ld, twy, -1);
        cx<R>* ul = u + ((long)v * 3 + l) * n + (long)i * np;
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int j = e / cols, q = e % cols;
            ul[(long)j * n3 + c0 + q] = buf[q * ld + j];
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_zpass_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ u,
                                                    cx<R>* __restrict__ z, int RB) {
    extern __shared__ __align__(16) char lds[];
    const int n2 = g.n2, n3 = g.n3, ld = n3 + 1;
    const long n = (long)g.n1 * n2 * n3, np = (long)n2 * n3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, j0 = blockIdx.z * RB;
    const int rows = min(RB, n2 - j0);
    cx<R>* buf = (cx<R>*)lds;
    cx<R>* twz = buf + (size_t)3 * RB * ld;
    cx<R>* twc = twz + n3;
    size_t off = (sizeof(cx<R>) * ((size_t)3 * RB * ld + 2 * n3) + 15) & ~(size_t)15;
    cx<double>* halfz = (cx<double>*)(lds + off);
    cx<double>* rowz = halfz + n3;
    cx<double>* lamy = rowz + RB;
    const cx<double> L0 = zpass_setup<R>(g, ks, tb, i, j0, rows, twz, twc, halfz, rowz, lamy);
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    const int M = n2 * n3;
    int s3m = g.s3 % M;
    if (s3m < 0) s3m += M;
    const double idz = 1.0 / g.dlt[2];
    const long base = (long)i * np + (long)j0 * n3;
    const unsigned char* codes = ks.codes + base;
    const cx<R>* ub = u + (long)v * 3 * n + base;
    RowWalk wk = row_walk(n3, j0, s3m, M);
    const int c = wk.c;
    __syncthreads();
    if (wk.active) {
        unsigned idx = wk.idx;
        for (int r = wk.r0; r < rows; r += wk.rstep) {
            const cx<R> tw = cmul(twc[c], rot[idx]);
#pragma unroll
            for (int l = 0; l < 3; ++l) buf[(l * RB + r) * ld + c] = cmulc(ub[(long)l * n + r * n3 + c], tw);
            idx += wk.step;
            if (idx >= (unsigned)M) idx -= (unsigned)M;
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < 3; ++l) fft_lines<R, kEpc, 256>(buf + (size_t)l * RB * ld, g.fz, rows, 1, ld, twz, -1);
    // z = W^H s per mode, W formed once for the three components
    cx<R>* zb = z + (long)v * 2 * n + base;
    if (wk.active) {
        for (int r = wk.r0; r < rows; r += wk.rstep) {
            const int e = r * n3 + c;
            const int code = codes[e];
            cx<R> a1 = mk<R>((R)0, (R)0), a2 = a1;
            if (code != kMasked) {
                const cx<double> h = cmul(halfz[c], rowz[r]);
                const cx<double> L2 = lam_from_halfturn(h.y, h.x, idz);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    cx<R> w1, w2;
                    w_row_code<R>(L0, lamy[r], L2, code, l, &w1, &w2);
                    const cx<R> val = buf[(l * RB + r) * ld + c];
                    a1 = a1 + cmulc(val, w1);
                    a2 = a2 + cmulc(val, w2);
                }
            }
            zb[e] = a1;
            zb[n + e] = a2;
        }
    }
}

// Row passes for n3 = 128 on registers: a 128-point row is held by 16 lanes with 8 values each
// (lane q: elements q + 16 m).  With k = k1 + 8 k2 and x = q + 16 m, the transform is an 8-point
// DFT over m in each lane, the twiddle w128^(q k1), and a 16-point DFT over q; that one is split
// again as q = q1 + 2 q2: after one exchange of the 8 x 16 intermediate through LDS rows owned by
// the wavefront (no work-group barrier), lane p = 2 k1 + q1 takes an 8-point DFT over q2, the
// twiddle w16^(q1 r) and a 2-point DFT with its neighbour lane p ^ 1 (a DPP lane move).  On
// return lane p holds output k1 + 8 r + 64 q1 in v[r].  Four rows per wavefront, 16 rows per
// work-group; the work-group shares only its tables.
constexpr int kRow128Slots = 4 * 16 * 9;      // exchange slots of a wavefront: 4 rows x 16 lanes x (8 + 1)

DEV float lane_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
DEV double lane_xor1(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)u, (int)(unsigned)u, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(u >> 32), (int)(unsigned)(u >> 32), 0xB1, 0xF, 0xF,
                                               false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

DEV void row_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sign S transform of the row held by the 16 lanes (q = lane mod 16) of one row group; tw[m] =
// exp(2 pi i m / 128); xb: the row's 144 exchange slots
template <typename R, int S>
DEV void line128(cx<R> v[8], const cx<R>* tw, cx<R>* __restrict__ xb, int q) {
    Bfly<R, 8>::run(v, S);
#pragma unroll
    for (int k1 = 1; k1 < 8; ++k1) {
        const cx<R> w = tw[(q * k1) & 127];
        v[k1] = S > 0 ? cmul(v[k1], w) : cmulc(v[k1], w);
    }
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) xb[q * 9 + k1] = v[k1];
    row_wave_sync();
    const int k1 = q >> 1, q1 = q & 1;
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) v[q2] = xb[(q1 + 2 * q2) * 9 + k1];
    row_wave_sync();
    Bfly<R, 8>::run(v, S);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        cx<R> z = v[r];
        if (q1 && r) {
            const cx<R> w = tw[8 * r];
            z = S > 0 ? cmul(z, w) : cmulc(z, w);
        }
        cx<R> pz;
        pz.x = lane_xor1(z.x);
        pz.y = lane_xor1(z.y);
        v[r] = q1 ? pz - z : z + pz;
    }
}

// the row pass's tables (zpass_setup) and exchange slots
template <typename R>
struct Row128Lds {
    cx<R> xch[4 * kRow128Slots];
    cx<R> twz[128], twc[128];
    cx<double> halfz[128], rowz[16], lamy[16];
};

template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_zrow128_fwd(Grid g, DeviceTables tb, const cx<R>* __restrict__ y,
                                                      cx<R>* __restrict__ u) {
    __shared__ Row128Lds<R> S;
    constexpr int N3 = 128;
    const int n2 = g.n2;
    const long n = (long)g.n1 * n2 * N3, np = (long)n2 * N3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, j0 = blockIdx.z * 16;
    const int rows = min(16, n2 - j0);
    const cx<double> L0 = zpass_setup<R>(g, ks, tb, i, j0, rows, S.twz, S.twc, S.halfz, S.rowz, S.lamy);
    const int tid = threadIdx.x, w = tid >> 6, gl = (tid >> 4) & 3, q = tid & 15;
    const int r = 4 * w + gl;
    const bool valid = r < rows;
    const int rr = valid ? r : 0;                  // rows past the grid compute on row 0 and store nothing
    const long base = (long)i * np + (long)(j0 + rr) * N3;
    const cx<R>* y1 = y + (long)v * 2 * n + base;
    const unsigned char* codes = ks.codes + base;
    cx<R> a[8], b[8];
    int code[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        a[m] = y1[q + 16 * m];
        b[m] = y1[n + q + 16 * m];
        code[m] = codes[q + 16 * m];
    }
    const int M = n2 * N3;
    int s3m = g.s3 % M;
    if (s3m < 0) s3m += M;
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    __syncthreads();
    // u_l = W_l1 y1 + W_l2 y2, W formed once per mode
    cx<R> uu[3][8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int k = q + 16 * m;
        uu[0][m] = uu[1][m] = uu[2][m] = mk<R>((R)0, (R)0);
        if (code[m] != kMasked) {
            const cx<double> h = cmul(S.halfz[k], S.rowz[rr]);
            const cx<double> L2 = lam_from_halfturn(h.y, h.x, idz);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                cx<R> w1, w2;
                w_row_code<R>(L0, S.lamy[rr], L2, code[m], l, &w1, &w2);
                uu[l][m] = cmul(w1, a[m]) + cmul(w2, b[m]);
            }
        }
    }
    // z twiddles of this lane's outputs c = (q >> 1) + 8 s + 64 (q & 1)
    const unsigned jm = ((unsigned)(j0 + rr) * (unsigned)s3m) % (unsigned)M;
    cx<R> zt[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int c = (q >> 1) + 8 * s + 64 * (q & 1);
        zt[s] = cmul(S.twc[c], rot[((unsigned)c * jm) % (unsigned)M]);
    }
    cx<R>* xb = S.xch + w * kRow128Slots + gl * 144;
    cx<R>* ub = u + (long)v * 3 * n + base;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        line128<R, +1>(uu[l], S.twz, xb, q);
        if (valid) {
#pragma unroll
            for (int s = 0; s < 8; ++s) ub[(long)l * n + (q >> 1) + 8 * s + 64 * (q & 1)] = cmul(uu[l][s], zt[s]);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_zrow128_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ u,
                                                      cx<R>* __restrict__ z) {
    __shared__ Row128Lds<R> S;
    constexpr int N3 = 128;
    const int n2 = g.n2;
    const long n = (long)g.n1 * n2 * N3, np = (long)n2 * N3;
    const KSel ks = select_k(g, n);
    const int i = blockIdx.x, v = blockIdx.y, j0 = blockIdx.z * 16;
    const int rows = min(16, n2 - j0);
    const cx<double> L0 = zpass_setup<R>(g, ks, tb, i, j0, rows, S.twz, S.twc, S.halfz, S.rowz, S.lamy);
    const int tid = threadIdx.x, w = tid >> 6, gl = (tid >> 4) & 3, q = tid & 15;
    const int r = 4 * w + gl;
    const bool valid = r < rows;
    const int rr = valid ? r : 0;
    const long base = (long)i * np + (long)(j0 + rr) * N3;
    const cx<R>* ub = u + (long)v * 3 * n + base;
    cx<R> tin[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) tin[m] = ub[q + 16 * m];
    const int M = n2 * N3;
    int s3m = g.s3 % M;
    if (s3m < 0) s3m += M;
    const double idz = 1.0 / g.dlt[2];
    const cx<R>* rot = sizeof(R) == 8 ? (const cx<R>*)tb.rot64 : (const cx<R>*)tb.rot32;
    __syncthreads();
    // z twiddles of this lane's inputs c = q + 16 m (conjugated below)
    const unsigned jm = ((unsigned)(j0 + rr) * (unsigned)s3m) % (unsigned)M;
    cx<R> zt[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int c = q + 16 * m;
        zt[m] = cmul(S.twc[c], rot[((unsigned)c * jm) % (unsigned)M]);
    }
    cx<R>* xb = S.xch + w * kRow128Slots + gl * 144;
    cx<R> s3[3][8];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int m = 0; m < 8; ++m) s3[l][m] = cmulc(tin[m], zt[m]);
        if (l < 2) {      // the next component's input, in flight during this component's transform
#pragma unroll
            for (int m = 0; m < 8; ++m) tin[m] = ub[(long)(l + 1) * n + q + 16 * m];
        }
        line128<R, -1>(s3[l], S.twz, xb, q);
    }
    // z = W^H s for this lane's modes k = (q >> 1) + 8 s + 64 (q & 1)
    const unsigned char* codes = ks.codes + base;
    cx<R>* zb = z + (long)v * 2 * n + base;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int k = (q >> 1) + 8 * s + 64 * (q & 1);
        const int code = codes[k];
        cx<R> a1 = mk<R>((R)0, (R)0), a2 = a1;
        if (code != kMasked) {
            const cx<double> h = cmul(S.halfz[k], S.rowz[rr]);
            const cx<double> L2 = lam_from_halfturn(h.y, h.x, idz);
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                cx<R> w1, w2;
                w_row_code<R>(L0, S.lamy[rr], L2, code, l, &w1, &w2);
                a1 = a1 + cmulc(s3[l][s], w1);
                a2 = a2 + cmulc(s3[l][s], w2);
            }
        }
        if (valid) {
            zb[k] = a1;
            zb[n + k] = a2;
        }
    }
}

// Adjoint column pass for n2 = 128 on registers: 16 columns per work-group, each held by 16 lanes
// with 8 values (line128), loaded straight from t[c][b] and stored as rows u[j][c0 .. c0 + 15]
// through an LDS tile (128-byte row segments).  (A forward counterpart, staging its input rows
// through the tile, ran no faster than the LDS-staged column pass in FP32 and 6 % slower in FP64.)
template <typename R>
struct Col128Lds {
    cx<R> tile[16 * 129];                       // column q, row j at q * 129 + j
    cx<R> xch[4 * kRow128Slots];
    cx<R> twy[128], twb[128];
};

template <typename R>
DEV void col128_tables(const Grid& g, const DeviceTables& tb, int i, Col128Lds<R>& S) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const double phi2 = (ks.kap[1] - (double)g.s1 * tx) / 128.0;
    const cx<R>* twy_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[1] : (const cx<R>*)tb.tw32[1];
    for (int b = threadIdx.x; b < 128; b += blockDim.x) {
        S.twy[b] = twy_g[b];
        S.twb[b] = cis_turns<R>((double)b * phi2);
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ycol128_adj(Grid g, DeviceTables tb, const cx<R>* __restrict__ t,
                                                      cx<R>* __restrict__ u) {
    __shared__ Col128Lds<R> S;
    const int n3 = g.n3;
    const long n = (long)g.n1 * 128 * n3, np = 128L * n3;
    const int i = blockIdx.x, v = blockIdx.y, c0 = blockIdx.z * 16;
    const int cols = min(16, n3 - c0);
    col128_tables<R>(g, tb, i, S);
    const int tid = threadIdx.x, w = tid >> 6, gl = (tid >> 4) & 3, q = tid & 15;
    const int col = 4 * w + gl;
    const int cc = col < cols ? col : 0;          // columns past the grid transform column 0, store nothing
    cx<R>* xb = S.xch + w * kRow128Slots + gl * 144;
    __syncthreads();
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        const cx<R>* tl = t + ((long)v * 3 + l) * n + (long)i * np + (long)(c0 + cc) * 128;
        cx<R> x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = cmulc(tl[q + 16 * m], S.twb[q + 16 * m]);
        line128<R, -1>(x, S.twy, xb, q);
        __syncthreads();                           // the previous component's rows are stored
#pragma unroll
        for (int s = 0; s < 8; ++s) S.tile[col * 129 + (q >> 1) + 8 * s + 64 * (q & 1)] = x[s];
        __syncthreads();
        cx<R>* ul = u + ((long)v * 3 + l) * n + (long)i * np;
        for (int e = tid; e < 128 * 16; e += 256) {
            const int j = e >> 4, qq = e & 15;
            if (qq < cols) ul[(long)j * n3 + c0 + qq] = S.tile[qq * 129 + j];
        }
    }
}

template <typename R>
static hipError_t split_fwd(const Grid& g, const DeviceTables& tb, const cx<R>* y, cx<R>* t, cx<R>* u, int nvec,
                            hipStream_t st) {
    const int RB = split_rows(g.n2, g.n3, sizeof(R) == 8), CB = split_cols(g.n3);
    // a timed pair: the start event at the first kernel's start, the stop event at the second's end
    const LaunchTimer pair = g_launch_timer;
    g_launch_timer.stop = nullptr;
    if (g.n3 == 128)
        PCX_LAUNCH((k_zrow128_fwd<R>), dim3(g.n1, nvec, (g.n2 + 15) / 16), dim3(256), 0, st, g, tb, y, u);
    else
        PCX_LAUNCH((k_zpass_fwd<R>), dim3(g.n1, nvec, (g.n2 + RB - 1) / RB), dim3(256),
                           zpass_lds_bytes<R>(RB, g.n3), st, g, tb, y, u, RB);
    hipError_t e = hipGetLastError();
    g_launch_timer = {nullptr, pair.stop};
    if (e == hipSuccess) {
        PCX_LAUNCH((k_ypass_fwd<R>), dim3(g.n1, nvec, (g.n3 + CB - 1) / CB), dim3(256),
                           ypass_lds_bytes<R>(CB, g.n2), st, g, tb, u, t, CB);
        e = hipGetLastError();
    }
    g_launch_timer = pair;
    return e;
}

template <typename R>
static hipError_t split_adj(const Grid& g, const DeviceTables& tb, const cx<R>* t, cx<R>* z, cx<R>* u, int nvec,
                            hipStream_t st) {
    const int RB = split_rows(g.n2, g.n3, sizeof(R) == 8), CB = split_cols(g.n3);
    const LaunchTimer pair = g_launch_timer;
    g_launch_timer.stop = nullptr;
    if (g.n2 == 128)
        PCX_LAUNCH((k_ycol128_adj<R>), dim3(g.n1, nvec, (g.n3 + 15) / 16), dim3(256), 0, st, g, tb, t, u);
    else
        PCX_LAUNCH((k_ypass_adj<R>), dim3(g.n1, nvec, (g.n3 + CB - 1) / CB), dim3(256),
                           ypass_lds_bytes<R>(CB, g.n2), st, g, tb, t, u, CB);
    hipError_t e = hipGetLastError();
    g_launch_timer = {nullptr, pair.stop};
    if (e == hipSuccess) {
        // FP64 adjoint: the register version needs 256 VGPRs (one wavefront per SIMD) and gains nothing
        if (g.n3 == 128 && sizeof(R) == 4)
            PCX_LAUNCH((k_zrow128_adj<R>), dim3(g.n1, nvec, (g.n2 + 15) / 16), dim3(256), 0, st, g, tb, u, z);
        else
            PCX_LAUNCH((k_zpass_adj<R>), dim3(g.n1, nvec, (g.n2 + RB - 1) / RB), dim3(256),
                               zpass_lds_bytes<R>(RB, g.n3), st, g, tb, u, z, RB);
        e = hipGetLastError();
    }
    g_launch_timer = pair;
    return e;
}

// ------------------------------------------------------------------ kernel 2: x-line transforms
// Tile = TB consecutive (c, b) positions q = c * n2 + b, all i.
// MODE 0: t -> IDFT_x -> * inv_eps/n -> DFT_x -> t            (matvec, in place)
// MODE 1: t -> IDFT_x -> * exp(2 pi i a phi1) n^{-1/2} (* inv_eps if given) -> u (e-layout)
// MODE 2: u (e-layout) -> * exp(-2 pi i a phi1) n^{-1/2} -> DFT_x -> t
template <typename R, int EPT, int MODE>
__global__ void __launch_bounds__(256) k_xline(Grid g, DeviceTables tb, const R* __restrict__ scale,
                                                     cx<R>* __restrict__ t, cx<R>* __restrict__ u, int TB) {
    const KSel ks = select_k(g, (long)g.n1 * g.n2 * g.n3);
    extern __shared__ __align__(16) char lds[];
    const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
    const long n = (long)n1 * n2 * n3;
    const long np = (long)n2 * n3;
    const int v = blockIdx.y;
    const long q0 = (long)blockIdx.x * TB;
    const int qn = (int)((np - q0) < TB ? (np - q0) : TB);
    const int ld = n1 + 1;
    cx<R>* buf = (cx<R>*)lds;
    cx<R>* twx = buf + (size_t)TB * ld;
    cx<R>* twa = twx + n1;
    const cx<R>* twx_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[0] : (const cx<R>*)tb.tw32[0];
    const double phi1 = ks.kap[0] / (double)n1;
    for (int a = threadIdx.x; a < n1; a += 256) {
        twx[a] = twx_g[a];
        if (MODE != 0) twa[a] = cis_turns<R>((double)a * phi1);
    }
    const R rsq = (R)(1.0 / sqrt((double)n));
    const int tot = n1 * qn;
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
        cx<R>* tl = t + ((long)v * 3 + l) * n;
        cx<R>* ul = u + ((long)v * 3 + l) * n;
        __syncthreads();
        if (MODE != 2) {
            // load t[i][q0 + ql] -> buf[ql][i]
            for (int e = threadIdx.x; e < tot; e += 256) {
                const int ii = e / qn, ql = e % qn;
                buf[ql * ld + ii] = tl[(long)ii * np + q0 + ql];
            }
            __syncthreads();
            fft_lines<R, (EPT < 16 ? EPT : 16), 256>(buf, g.fx, qn, 1, ld, twx, +1);            // i -> a
        } else {
            // load u[(q0 + ql) * n1 + a] -> buf[ql][a] with the conjugate x twiddle
            for (int e = threadIdx.x; e < tot; e += 256) {
                const int ql = e / n1, a = e % n1;
                cx<R> val = ul[(q0 + ql) * n1 + a];
                buf[ql * ld + a] = cscale(cmulc(val, twa[a]), rsq);
            }
            __syncthreads();
        }
        if (MODE == 0) {
            const R* sl = scale + (long)l * n;
            for (int e = threadIdx.x; e < tot; e += 256) {
                const int ql = e / n1, a = e % n1;
                buf[ql * ld + a] = cscale(buf[ql * ld + a], sl[(q0 + ql) * n1 + a]);
            }
            __syncthreads();
        }
        if (MODE == 1) {
            const R* sl = scale ? scale + (long)l * n : nullptr;
            for (int e = threadIdx.x; e < tot; e += 256) {
                const int ql = e / n1, a = e % n1;
                R f = rsq;
                if (sl) f *= sl[(q0 + ql) * n1 + a];
                ul[(q0 + ql) * n1 + a] = cscale(cmul(buf[ql * ld + a], twa[a]), f);
            }
            continue;
        }
        fft_lines<R, (EPT < 16 ? EPT : 16), 256>(buf, g.fx, qn, 1, ld, twx, -1);                // a -> i
        for (int e = threadIdx.x; e < tot; e += 256) {
            const int ii = e / qn, ql = e % qn;
            tl[(long)ii * np + q0 + ql] = buf[ql * ld + ii];
        }
    }
}

// ------------------------------------------------------------------ mixing basis per mode
// FP64 decision, shared by the FP32 and FP64 kernels: kMasked where Lambda_q = 0 (t_x, t_y, t_z all
// whole), else mix_code of the FP64 symbols.
__global__ void k_modecode(Grid g, unsigned char* __restrict__ out) {
    const long n = (long)g.n1 * g.n2 * g.n3;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int k = (int)(e % g.n3);
        const int j = (int)((e / g.n3) % g.n2);
        const int i = (int)(e / ((long)g.n2 * g.n3));
        const double tx = (g.kap[0] + (double)i) / (double)g.n1;
        const double ty = ((g.kap[1] + (double)j) - (double)g.s1 * tx) / (double)g.n2;
        const double Rz = (g.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ty;
        const double tz = ((g.kap[2] + (double)k) - (double)g.s2 * tx - (double)g.s3 * ty) / (double)g.n3;
        bool masked = false;
        if (tx == rint(tx) && ty == rint(ty) && Rz == rint(Rz)) {
            long kk = (-(long)rint(Rz)) % g.n3;
            if (kk < 0) kk += g.n3;
            masked = (kk == k);
        }
        out[e] = masked ? kMasked
                        : mix_code(lam_of_turn(tx, 1.0 / g.dlt[0]), lam_of_turn(ty, 1.0 / g.dlt[1]),
                                   lam_of_turn(tz, 1.0 / g.dlt[2]));
    }
}

hipError_t launch_modecode(const Grid& g, unsigned char* out, hipStream_t st) {
    const long n = (long)g.n1 * g.n2 * g.n3;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_modecode, dim3(blocks), dim3(256), 0, st, g, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ preconditioner diagonal
__global__ void k_precond(Grid g, DeviceTables tb, double* __restrict__ out) {
    const long n = (long)g.n1 * g.n2 * g.n3;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const int k = (int)(e % g.n3);
        const int j = (int)((e / g.n3) % g.n2);
        const int i = (int)(e / ((long)g.n2 * g.n3));
        const double tx = (g.kap[0] + (double)i) / (double)g.n1;
        const double ty = ((g.kap[1] + (double)j) - (double)g.s1 * tx) / (double)g.n2;
        const double Rz = (g.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ty;
        const double tz = ((g.kap[2] + (double)k) - (double)g.s2 * tx - (double)g.s3 * ty) / (double)g.n3;
        bool masked = false;
        if (tx == rint(tx) && ty == rint(ty) && Rz == rint(Rz)) {
            long kk = (-(long)rint(Rz)) % g.n3;
            if (kk < 0) kk += g.n3;
            masked = (kk == k);
        }
        double Lq = abs2(lam_of_turn(tx, 1.0 / g.dlt[0])) + abs2(lam_of_turn(ty, 1.0 / g.dlt[1])) +
                    abs2(lam_of_turn(tz, 1.0 / g.dlt[2]));
        out[e] = masked ? 0.0 : 1.0 / Lq;
    }
}

// ------------------------------------------------------------------ launchers
constexpr int kXThreads = 256;     // x-line kernel work-group

static int pow2_at_least(long e) {
    int p = 1;
    while (p < e) p <<= 1;
    return p;
}

// plane kernels: enough threads that each owns at most 4 modes (up to 1024 threads; FP64 up to
// 512 so that the 128 registers a 1024-thread group allows per lane are not exceeded), unless the
// plan's tuned work-group size (256 / 512 / 1024, FP64 at most 512) says otherwise
static void plane_shape(long np, int fp64, int want, int* nt, int* ept) {
    int t = 256;
    const int tmax = fp64 ? 512 : 1024;
    while (t < tmax && (np + t - 1) / t > 4) t <<= 1;
    if (want == 256 || want == 512 || (want == 1024 && !fp64)) t = want;
    *nt = t;
    *ept = pow2_at_least((np + t - 1) / t);
}

static int xline_tile(int n1) {
    // enough lines per tile to give every thread a few elements, and whole 64-wide segments
    int tb = 64;
    if (n1 <= 16) tb = 128;
    return tb;
}

template <typename R>
static size_t xline_lds_bytes(int n1, int TB) {
    return sizeof(cx<R>) * ((size_t)TB * (n1 + 1) + 2 * n1);
}

#define PCX_PLANE_DISPATCH(NTV, EPTV, CALL)                     \
    if (NTV == 1024) {                                          \
        switch (EPTV) {                                         \
            case 1: CALL(1024, 1); break;                       \
            case 2: CALL(1024, 2); break;                       \
            case 4: CALL(1024, 4); break;                       \
            case 8: CALL(1024, 8); break;                       \
            case 16: CALL(1024, 16); break;                     \
            case 32: CALL(1024, 32); break;                     \
            case 64: CALL(1024, 64); break;                     \
            default: return hipErrorInvalidValue;               \
        }                                                       \
    } else if (NTV == 512) {                                    \
        switch (EPTV) {                                         \
            case 4: CALL(512, 4); break;                        \
            case 8: CALL(512, 8); break;                        \
            case 16: CALL(512, 16); break;                      \
            case 32: CALL(512, 32); break;                      \
            case 64: CALL(512, 64); break;                      \
            default: return hipErrorInvalidValue;               \
        }                                                       \
    } else {                                                    \
        switch (EPTV) {                                         \
            case 1: CALL(256, 1); break;                        \
            case 2: CALL(256, 2); break;                        \
            case 4: CALL(256, 4); break;                        \
            case 8: CALL(256, 8); break;                        \
            case 16: CALL(256, 16); break;                      \
            case 32: CALL(256, 32); break;                      \
            case 64: CALL(256, 64); break;                      \
            default: return hipErrorInvalidValue;               \
        }                                                       \
    }

#define PCX_EPT_DISPATCH(EPTV, CALL) \
    switch (EPTV) {                  \
        case 1: CALL(1); break;      \
        case 2: CALL(2); break;      \
        case 4: CALL(4); break;      \
        case 8: CALL(8); break;      \
        case 16: CALL(16); break;    \
        case 32: CALL(32); break;    \
        case 64: CALL(64); break;    \
        default: return hipErrorInvalidValue; \
    }

template <typename R>
static hipError_t plane_fwd(const Grid& g, const DeviceTables& tb, const cx<R>* y, cx<R>* t, int nvec,
                            hipStream_t st) {
    if (g.split[sizeof(R) == 8]) return split_fwd<R>(g, tb, y, t, t + (size_t)nvec * 3 * g.n1 * g.n2 * g.n3, nvec, st);
    if (!g.generic[sizeof(R) == 8]) {
        bool done = false;
        hipError_t e = launch_fixed_plane_fwd<R>(g, tb, y, t, nvec, st, &done);
        if (done || e != hipSuccess) return e;
    }
    dim3 grid(g.n1, nvec);
    const size_t lds = plane_lds_bytes<R>(g.n2, g.n3);
    int nt, ept;
    plane_shape((long)g.n2 * g.n3, sizeof(R) == 8, g.plane_nt[sizeof(R) == 8], &nt, &ept);
#define CALLF(NT, E) PCX_LAUNCH((k_plane_fwd<R, NT, E>), grid, dim3(NT), lds, st, g, tb, y, t)
    PCX_PLANE_DISPATCH(nt, ept, CALLF)
#undef CALLF
    return hipGetLastError();
}

template <typename R>
static hipError_t plane_adj(const Grid& g, const DeviceTables& tb, const cx<R>* t, cx<R>* z, int nvec,
                            hipStream_t st) {
    if (g.split[sizeof(R) == 8])
        return split_adj<R>(g, tb, t, z, const_cast<cx<R>*>(t) + (size_t)nvec * 3 * g.n1 * g.n2 * g.n3, nvec, st);
    if (!g.generic[sizeof(R) == 8]) {
        bool done = false;
        hipError_t e = launch_fixed_plane_adj<R>(g, tb, t, z, nvec, st, &done);
        if (done || e != hipSuccess) return e;
    }
    dim3 grid(g.n1, nvec);
    const size_t lds = plane_lds_bytes<R>(g.n2, g.n3);
    int nt, ept;
    plane_shape((long)g.n2 * g.n3, sizeof(R) == 8, g.plane_nt[sizeof(R) == 8], &nt, &ept);
#define CALLA(NT, E) PCX_LAUNCH((k_plane_adj<R, NT, E>), grid, dim3(NT), lds, st, g, tb, t, z)
    PCX_PLANE_DISPATCH(nt, ept, CALLA)
#undef CALLA
    return hipGetLastError();
}

template <typename R, int MODE>
static hipError_t xline(const Grid& g, const DeviceTables& tb, const R* scale, cx<R>* t, cx<R>* u, int nvec,
                        hipStream_t st) {
    if (MODE == 0 && !g.generic[sizeof(R) == 8]) {
        bool done = false;
        hipError_t e = launch_fixed_xline<R>(g, tb, scale, t, nvec, st, &done);
        if (done || e != hipSuccess) return e;
    }
    const int TB = xline_tile(g.n1);
    const long np = (long)g.n2 * g.n3;
    dim3 grid((unsigned)((np + TB - 1) / TB), nvec);
    const size_t lds = xline_lds_bytes<R>(g.n1, TB);
    const int ept = pow2_at_least(((long)g.n1 * TB + kXThreads - 1) / kXThreads);
#define CALLX(E) PCX_LAUNCH((k_xline<R, E, MODE>), grid, dim3(kXThreads), lds, st, g, tb, scale, t, u, TB)
    PCX_EPT_DISPATCH(ept, CALLX)
#undef CALLX
    return hipGetLastError();
}

hipError_t launch_precond_mixed(const Grid& g, const DeviceTables& tb, const float* epsn32, const cx<double>* y,
                                cx<double>* z, cx<float>* t, const double* scale, int nvec, hipStream_t st) {
    // exactly where the FP32 A_r takes the register kernels (plane_fwd / plane_adj)
    const int kind0 = g.fixed_kind[0];
    if (g.split[0] || g.generic[0] || !(kind0 == 0 || kind0 == 4) || !wave_plane_available(g, 0))
        return hipErrorNotSupported;
    hipError_t e = launch_wave_plane_fwd(g, tb, y, t, nvec, st);
    if (e == hipSuccess) e = xline<float, 0>(g, tb, epsn32, t, nullptr, nvec, st);
    if (e == hipSuccess) e = launch_wave_plane_adj(g, tb, t, z, scale, nvec, st);
    return e;
}

template <typename R>
hipError_t launch_apply_Ar(const Grid& g, const DeviceTables& tb, const R* inv_eps_n, const cx<R>* y, cx<R>* z,
                           cx<R>* t, int nvec, hipStream_t st) {
    hipError_t e = plane_fwd<R>(g, tb, y, t, nvec, st);
    if (e != hipSuccess) return e;
    e = xline<R, 0>(g, tb, inv_eps_n, t, nullptr, nvec, st);
    if (e != hipSuccess) return e;
    return plane_adj<R>(g, tb, t, z, nvec, st);
}

template <typename R>
hipError_t time_apply_Ar(const Grid& g, const DeviceTables& tb, const R* inv_eps_n, const cx<R>* y, cx<R>* z,
                         cx<R>* t, int nvec, int reps, hipStream_t st, double ms[3]) {
    // `reps` applications queued back to back, in the solver's order; each kernel records its own
    // start and end events at dispatch (g_launch_timer), so nothing is inserted between kernels
    std::vector<hipEvent_t> ev((size_t)6 * reps);
    size_t made = 0;
    hipError_t e = hipSuccess;
    for (; made < ev.size() && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) --made;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        hipEvent_t* q = &ev[(size_t)6 * r];
        g_launch_timer = {q[0], q[1]};
        e = plane_fwd<R>(g, tb, y, t, nvec, st);
        g_launch_timer = {q[2], q[3]};
        if (e == hipSuccess) e = xline<R, 0>(g, tb, inv_eps_n, t, nullptr, nvec, st);
        g_launch_timer = {q[4], q[5]};
        if (e == hipSuccess) e = plane_adj<R>(g, tb, t, z, nvec, st);
        g_launch_timer = {};
    }
    g_launch_timer = {};
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    double acc[3] = {0, 0, 0};
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            float f = 0.0f;
            e = hipEventElapsedTime(&f, ev[(size_t)6 * r + 2 * k], ev[(size_t)6 * r + 2 * k + 1]);
            acc[k] += f;
        }
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    for (int k = 0; k < 3; ++k) ms[k] = reps > 0 ? acc[k] / reps : 0.0;
    return e;
}

template <typename R>
hipError_t launch_QS(const Grid& g, const DeviceTables& tb, const R* inv_eps, const cx<R>* y, cx<R>* u, cx<R>* t,
                     int nvec, hipStream_t st) {
    hipError_t e = plane_fwd<R>(g, tb, y, t, nvec, st);
    if (e != hipSuccess) return e;
    return xline<R, 1>(g, tb, inv_eps, t, u, nvec, st);
}

template <typename R>
hipError_t launch_QS_adjoint(const Grid& g, const DeviceTables& tb, const cx<R>* u, cx<R>* z, cx<R>* t, int nvec,
                             hipStream_t st) {
    hipError_t e = xline<R, 2>(g, tb, nullptr, t, const_cast<cx<R>*>(u), nvec, st);
    if (e != hipSuccess) return e;
    return plane_adj<R>(g, tb, t, z, nvec, st);
}

hipError_t launch_precond_diag(const Grid& g, const DeviceTables& tb, double* out, hipStream_t st) {
    const long n = (long)g.n1 * g.n2 * g.n3;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_precond, dim3(blocks), dim3(256), 0, st, g, tb, out);
    return hipGetLastError();
}

template <typename F>
static hipError_t set_max_lds(F f) {
    return hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename R, int NT, int E>
static hipError_t set_plane() {
    hipError_t e = set_max_lds(k_plane_fwd<R, NT, E>);
    if (e == hipSuccess) e = set_max_lds(k_plane_adj<R, NT, E>);
    return e;
}

template <typename R, int E>
static hipError_t set_xline() {
    hipError_t e = set_max_lds(k_xline<R, E, 0>);
    if (e == hipSuccess) e = set_max_lds(k_xline<R, E, 1>);
    if (e == hipSuccess) e = set_max_lds(k_xline<R, E, 2>);
    return e;
}

template <typename R>
static hipError_t set_lds_limits() {
    hipError_t e = hipSuccess;
#define CHK(x) \
    if (e == hipSuccess) e = (x)
    CHK((set_plane<R, 1024, 1>()));
    CHK((set_plane<R, 1024, 2>()));
    CHK((set_plane<R, 1024, 4>()));
    CHK((set_plane<R, 1024, 8>()));
    CHK((set_plane<R, 1024, 16>()));
    CHK((set_plane<R, 1024, 32>()));
    CHK((set_plane<R, 1024, 64>()));
    CHK((set_plane<R, 512, 4>()));
    CHK((set_plane<R, 512, 8>()));
    CHK((set_plane<R, 512, 16>()));
    CHK((set_plane<R, 512, 32>()));
    CHK((set_plane<R, 512, 64>()));
    CHK((set_plane<R, 256, 1>()));
    CHK((set_plane<R, 256, 2>()));
    CHK((set_plane<R, 256, 4>()));
    CHK((set_plane<R, 256, 8>()));
    CHK((set_plane<R, 256, 16>()));
    CHK((set_plane<R, 256, 32>()));
    CHK((set_plane<R, 256, 64>()));
    CHK((set_xline<R, 1>()));
    CHK((set_xline<R, 2>()));
    CHK((set_xline<R, 4>()));
    CHK((set_xline<R, 8>()));
    CHK((set_xline<R, 16>()));
    CHK((set_xline<R, 32>()));
    CHK((set_xline<R, 64>()));
#undef CHK
    return e;
}

template <typename R>
static hipError_t split_limits() {
    hipError_t e = set_max_lds(k_zpass_fwd<R>);
    if (e == hipSuccess) e = set_max_lds(k_zpass_adj<R>);
    if (e == hipSuccess) e = set_max_lds(k_ypass_fwd<R>);
    if (e == hipSuccess) e = set_max_lds(k_ypass_adj<R>);
    return e;
}

bool split_plane_needed(int n2, int n3, int fp64) {
    // FP64: the plane does not fit in LDS; FP32: one plane would leave room for one work-group per
    // CU (at 128 x 128 the single-plane kernel moves 1 TB/s, the two passes about twice that)
    return (fp64 ? plane_lds_bytes<double>(n2, n3) : plane_lds_bytes<float>(n2, n3)) > (fp64 ? 160 : 80) * 1024;
}
size_t split_kernel_lds(int n2, int n3, int fp64) {
    const int RB = split_rows(n2, n3, fp64 != 0), CB = split_cols(n3);
    const size_t a = fp64 ? zpass_lds_bytes<double>(RB, n3) : zpass_lds_bytes<float>(RB, n3);
    const size_t b = fp64 ? ypass_lds_bytes<double>(CB, n2) : ypass_lds_bytes<float>(CB, n2);
    return a > b ? a : b;
}

hipError_t configure_kernels() {
    hipError_t e = set_lds_limits<float>();
    if (e != hipSuccess) return e;
    e = set_lds_limits<double>();
    if (e == hipSuccess) e = split_limits<float>();
    if (e == hipSuccess) e = split_limits<double>();
    if (e != hipSuccess) return e;
    return configure_fixed_kernels();
}

size_t plane_kernel_lds(int n2, int n3, int fp64) {
    return fp64 ? plane_lds_bytes<double>(n2, n3) : plane_lds_bytes<float>(n2, n3);
}
size_t xline_kernel_lds(int n1, int fp64) {
    const int TB = xline_tile(n1);
    return fp64 ? xline_lds_bytes<double>(n1, TB) : xline_lds_bytes<float>(n1, TB);
}
int xline_kernel_tile(int n1) { return xline_tile(n1); }

template hipError_t launch_apply_Ar<float>(const Grid&, const DeviceTables&, const float*, const cx<float>*,
                                           cx<float>*, cx<float>*, int, hipStream_t);
template hipError_t launch_apply_Ar<double>(const Grid&, const DeviceTables&, const double*, const cx<double>*,
                                            cx<double>*, cx<double>*, int, hipStream_t);
template hipError_t time_apply_Ar<float>(const Grid&, const DeviceTables&, const float*, const cx<float>*,
                                         cx<float>*, cx<float>*, int, int, hipStream_t, double*);
template hipError_t time_apply_Ar<double>(const Grid&, const DeviceTables&, const double*, const cx<double>*,
                                          cx<double>*, cx<double>*, int, int, hipStream_t, double*);
template hipError_t launch_QS<float>(const Grid&, const DeviceTables&, const float*, const cx<float>*, cx<float>*,
                                     cx<float>*, int, hipStream_t);
template hipError_t launch_QS<double>(const Grid&, const DeviceTables&, const double*, const cx<double>*,
                                      cx<double>*, cx<double>*, int, hipStream_t);
template hipError_t launch_QS_adjoint<float>(const Grid&, const DeviceTables&, const cx<float>*, cx<float>*,
                                             cx<float>*, int, hipStream_t);
template hipError_t launch_QS_adjoint<double>(const Grid&, const DeviceTables&, const cx<double>*, cx<double>*,
                                              cx<double>*, int, hipStream_t);

}  // namespace pcx
