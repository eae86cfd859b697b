// Block-vector kernels for the LOBPCG driver: Gram products A^H B (FP64 accumulation),
// small-matrix combinations S C, residual + Lambda_q^{-1} preconditioner, conversions.
// Vectors are columns of length N stored contiguously; a ColSet lists up to 4 runs of columns.
#include "pcx_internal.h"

namespace pcx {

#define DEV __device__ __forceinline__

constexpr int kMaxCols = 6 * PCX_MAX_BLOCK;
constexpr int kGramRows = 32;      // rows staged per sub-tile
constexpr int kBlk = 4;            // 4 x 4 register tile of Gram entries per thread

template <typename R>
DEV cx<double> to64(cx<R> a) {
    cx<double> z;
    z.x = (double)a.x;
    z.y = (double)a.y;
    return z;
}

// pointer to column c of the set
template <typename R>
DEV R* col_ptr(const ColSet& S, int c, long N) {
    int off = 0;
    for (int s = 0; s < kMaxSeg; ++s) {
        if (c < off + S.ncols[s]) return (R*)S.ptr[s] + (long)(c - off) * N;
        off += S.ncols[s];
    }
    return nullptr;
}

// ------------------------------------------------------------------ Gram: part[chunk] = A^H B over the chunk rows
template <typename R>
__global__ void __launch_bounds__(256) k_gram(ColSet A, ColSet B, long N, long rows_per_chunk,
                                               cx<double>* __restrict__ part, int round) {
    extern __shared__ __align__(16) char lds[];
    const int ka = A.total(), kb = B.total();
    const int ka4 = (ka + kBlk - 1) / kBlk * kBlk, kb4 = (kb + kBlk - 1) / kBlk * kBlk;
    cx<double>* As = (cx<double>*)lds;                  // [ka4][kGramRows]
    cx<double>* Bs = As + (size_t)ka4 * kGramRows;       // [kb4][kGramRows]
    const cx<R>** acol = (const cx<R>**)(Bs + (size_t)kb4 * kGramRows);
    const cx<R>** bcol = acol + kMaxCols;
    for (int c = threadIdx.x; c < ka; c += blockDim.x) acol[c] = col_ptr<const cx<R>>(A, c, N);
    for (int c = threadIdx.x; c < kb; c += blockDim.x) bcol[c] = col_ptr<const cx<R>>(B, c, N);

    const long r0 = (long)blockIdx.x * rows_per_chunk;
    const long r1 = min(N, r0 + rows_per_chunk);
    const int nbA = ka4 / kBlk, nbB = kb4 / kBlk;
    const int PB = nbA * nbB;
    constexpr int kMaxPB = 2;   // pair-blocks per thread and round
    const int pb0 = round * kMaxPB * 256;
    cx<double> acc[kMaxPB][kBlk][kBlk];
#pragma unroll
    for (int p = 0; p < kMaxPB; ++p)
#pragma unroll
        for (int u = 0; u < kBlk; ++u)
#pragma unroll
            for (int w = 0; w < kBlk; ++w) acc[p][u][w].x = acc[p][u][w].y = 0.0;
    __syncthreads();

    for (long rt = r0; rt < r1; rt += kGramRows) {
        const int rows = (int)min((long)kGramRows, r1 - rt);
        for (int e = threadIdx.x; e < ka4 * kGramRows; e += blockDim.x) {
            const int c = e / kGramRows, r = e % kGramRows;
            cx<double> val;
            val.x = val.y = 0.0;
            if (c < ka && r < rows) val = to64(acol[c][rt + r]);
            As[e] = val;
        }
        for (int e = threadIdx.x; e < kb4 * kGramRows; e += blockDim.x) {
            const int c = e / kGramRows, r = e % kGramRows;
            cx<double> val;
            val.x = val.y = 0.0;
            if (c < kb && r < rows) val = to64(bcol[c][rt + r]);
            Bs[e] = val;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kMaxPB; ++p) {
            const int pb = pb0 + threadIdx.x + p * blockDim.x;
            if (pb < PB) {
                const int ba = pb / nbB, bb = pb % nbB;
                const cx<double>* ap = As + (size_t)ba * kBlk * kGramRows;
                const cx<double>* bp = Bs + (size_t)bb * kBlk * kGramRows;
                for (int r = 0; r < kGramRows; ++r) {
                    cx<double> av[kBlk], bv[kBlk];
#pragma unroll
                    for (int u = 0; u < kBlk; ++u) av[u] = ap[u * kGramRows + r];
#pragma unroll
                    for (int w = 0; w < kBlk; ++w) bv[w] = bp[w * kGramRows + r];
#pragma unroll
                    for (int u = 0; u < kBlk; ++u)
#pragma unroll
                        for (int w = 0; w < kBlk; ++w) {
                            // conj(a) * b
                            acc[p][u][w].x += av[u].x * bv[w].x + av[u].y * bv[w].y;
                            acc[p][u][w].y += av[u].x * bv[w].y - av[u].y * bv[w].x;
                        }
                }
            }
        }
        __syncthreads();
    }
    cx<double>* out = part + (size_t)blockIdx.x * ka * kb;
#pragma unroll
    for (int p = 0; p < kMaxPB; ++p) {
        const int pb = pb0 + threadIdx.x + p * blockDim.x;
        if (pb < PB) {
            const int ba = pb / nbB, bb = pb % nbB;
#pragma unroll
            for (int u = 0; u < kBlk; ++u)
#pragma unroll
                for (int w = 0; w < kBlk; ++w) {
                    const int ia = ba * kBlk + u, ib = bb * kBlk + w;
                    if (ia < ka && ib < kb) out[(size_t)ia * kb + ib] = acc[p][u][w];
                }
        }
    }
}

__global__ void k_reduce_parts(const cx<double>* __restrict__ part, int nchunk, int count, cx<double>* __restrict__ out) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            cx<double> v = part[(size_t)c * count + e];
            sx += v.x;
            sy += v.y;
        }
        out[e].x = sx;
        out[e].y = sy;
    }
}

template <typename R>
hipError_t launch_gram(const ColSet& A, const ColSet& B, long N, cx<double>* part, int nchunk, cx<double>* out,
                       hipStream_t st) {
    const int ka = A.total(), kb = B.total();
    if (ka < 1 || kb < 1 || ka > kMaxCols || kb > kMaxCols) return hipErrorInvalidValue;
    const int ka4 = (ka + kBlk - 1) / kBlk * kBlk, kb4 = (kb + kBlk - 1) / kBlk * kBlk;
    long rpc = (N + nchunk - 1) / nchunk;
    rpc = (rpc + kGramRows - 1) / kGramRows * kGramRows;
    const int chunks = (int)((N + rpc - 1) / rpc);
    const size_t lds = sizeof(cx<double>) * (size_t)(ka4 + kb4) * kGramRows + 2 * sizeof(void*) * kMaxCols;
    const int PB = (ka4 / kBlk) * (kb4 / kBlk);
    const int rounds = (PB + 2 * 256 - 1) / (2 * 256);
    for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL((k_gram<R>), dim3(chunks), dim3(256), lds, st, A, B, N, rpc, part, r);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int count = ka * kb;
    hipLaunchKernelGGL(k_reduce_parts, dim3((count + 255) / 256), dim3(256), 0, st, part, chunks, count, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Y = S C
constexpr int kOutChunk = 8;

template <typename R>
__global__ void __launch_bounds__(256) k_combine(ColSet S, const cx<double>* __restrict__ C, ColSet Y, long N) {
    __shared__ const cx<R>* scol[kMaxCols];
    __shared__ cx<R>* ycol[kMaxCols];
    const int ks = S.total(), m = Y.total();
    for (int c = threadIdx.x; c < ks; c += blockDim.x) scol[c] = col_ptr<const cx<R>>(S, c, N);
    for (int c = threadIdx.x; c < m; c += blockDim.x) ycol[c] = col_ptr<cx<R>>(Y, c, N);
    __syncthreads();
    for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < N; r += (long)gridDim.x * blockDim.x) {
        for (int m0 = 0; m0 < m; m0 += kOutChunk) {
            cx<double> acc[kOutChunk];
#pragma unroll
            for (int u = 0; u < kOutChunk; ++u) acc[u].x = acc[u].y = 0.0;
            for (int k = 0; k < ks; ++k) {
                const cx<double> s = to64(scol[k][r]);
                const cx<double>* crow = C + (size_t)k * m + m0;
#pragma unroll
                for (int u = 0; u < kOutChunk; ++u) {
                    if (m0 + u < m) {
                        const cx<double> c = crow[u];
                        acc[u].x += s.x * c.x - s.y * c.y;
                        acc[u].y += s.x * c.y + s.y * c.x;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kOutChunk; ++u) {
                if (m0 + u < m) {
                    cx<R> o;
                    o.x = (R)acc[u].x;
                    o.y = (R)acc[u].y;
                    ycol[m0 + u][r] = o;
                }
            }
        }
    }
}

template <typename R>
hipError_t launch_combine(const ColSet& S, const cx<double>* C, const ColSet& Y, long N, hipStream_t st) {
    if (S.total() < 1 || Y.total() < 1 || S.total() > kMaxCols || Y.total() > kMaxCols) return hipErrorInvalidValue;
    long blocks = (N + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL((k_combine<R>), dim3((unsigned)blocks), dim3(256), 0, st, S, C, Y, N);
    return hipGetLastError();
}

// ------------------------------------------------------------------ residual + preconditioner
DEV double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

template <typename R>
__global__ void __launch_bounds__(256) k_residual(ColSet X, ColSet AX, const double* __restrict__ theta,
                                                   const double* __restrict__ prec, long n, ColSet W,
                                                   long rows_per_chunk, double* __restrict__ part) {
    __shared__ double red[4];
    const int ka = X.total();
    const long N = 2 * n;
    const long r0 = (long)blockIdx.x * rows_per_chunk;
    const long r1 = min(N, r0 + rows_per_chunk);
    for (int j = 0; j < ka; ++j) {
        const cx<R>* x = col_ptr<const cx<R>>(X, j, N);
        const cx<R>* ax = col_ptr<const cx<R>>(AX, j, N);
        cx<R>* w = col_ptr<cx<R>>(W, j, N);
        const double th = theta[j];
        double s = 0.0;
        for (long r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            const cx<double> xv = to64(x[r]), av = to64(ax[r]);
            const double rx = av.x - th * xv.x, ry = av.y - th * xv.y;
            s += rx * rx + ry * ry;
            const double p = prec ? prec[r < n ? r : r - n] : 1.0;
            cx<R> o;
            o.x = (R)(p * rx);
            o.y = (R)(p * ry);
            w[r] = o;
        }
        s = block_sum(s, red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * ka + j] = s;
    }
}

__global__ void k_reduce_real(const double* __restrict__ part, int nchunk, int count, double* __restrict__ out) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * count + e];
        out[e] = s;
    }
}

template <typename R>
hipError_t launch_residual(const ColSet& X, const ColSet& AX, const double* theta, const double* prec, long n,
                           const ColSet& W, double* part, int nchunk, double* out, hipStream_t st) {
    const long N = 2 * n;
    long rpc = (N + nchunk - 1) / nchunk;
    rpc = (rpc + 255) / 256 * 256;
    const int chunks = (int)((N + rpc - 1) / rpc);
    hipLaunchKernelGGL((k_residual<R>), dim3(chunks), dim3(256), 0, st, X, AX, theta, prec, n, W, rpc, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int count = X.total();
    hipLaunchKernelGGL(k_reduce_real, dim3((count + 255) / 256), dim3(256), 0, st, part, chunks, count, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ small element-wise kernels
template <typename A, typename B>
__global__ void k_convert(const cx<A>* __restrict__ in, cx<B>* __restrict__ out, long count) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        cx<B> o;
        o.x = (B)in[e].x;
        o.y = (B)in[e].y;
        out[e] = o;
    }
}

static unsigned grid_for(long count) {
    long b = (count + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_convert(const cx<float>* in, cx<double>* out, long count, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(count)), dim3(256), 0, st, in, out, count);
    return hipGetLastError();
}
hipError_t launch_convert(const cx<double>* in, cx<float>* out, long count, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(count)), dim3(256), 0, st, in, out, count);
    return hipGetLastError();
}

template <typename R>
__global__ void k_mask(cx<R>* __restrict__ y, const double* __restrict__ prec, long n, long count) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        if (prec[e % n] == 0.0) {
            y[e].x = (R)0;
            y[e].y = (R)0;
        }
    }
}

template <typename R>
hipError_t launch_mask(cx<R>* y, const double* prec, long n, int nvec, hipStream_t st) {
    const long count = 2 * n * (long)nvec;
    hipLaunchKernelGGL((k_mask<R>), dim3(grid_for(count)), dim3(256), 0, st, y, prec, n, count);
    return hipGetLastError();
}

__global__ void k_grad(const cx<double>* __restrict__ x, const double* __restrict__ w, int nvec, long n,
                       double* __restrict__ grad, int voxel) {
    const long cnt = voxel ? n : 3 * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < cnt; e += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int t = 0; t < nvec; ++t) {
            const cx<double>* xt = x + (long)t * 3 * n;
            if (voxel) {
                for (int l = 0; l < 3; ++l) {
                    const cx<double> v = xt[l * n + e];
                    s -= w[t] * (v.x * v.x + v.y * v.y);
                }
            } else {
                const cx<double> v = xt[e];
                s -= w[t] * (v.x * v.x + v.y * v.y);
            }
        }
        grad[e] = s;
    }
}

hipError_t launch_grad(const cx<double>* x, const double* w, int nvec, long n, double* grad, int voxel,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_grad, dim3(grid_for(voxel ? n : 3 * n)), dim3(256), 0, st, x, w, nvec, n, grad, voxel);
    return hipGetLastError();
}

// counter-based normal deviates: splitmix64 of (seed, index) -> two uniforms -> Box-Muller
DEV unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

template <typename R>
__global__ void k_random(cx<R>* __restrict__ y, long count, unsigned long long seed, double scale) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const unsigned long long h = splitmix64(seed ^ splitmix64((unsigned long long)e));
        const double u1 = ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = ((double)(splitmix64(h) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double rad = scale * sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        cx<R> o;
        o.x = (R)(rad * c);
        o.y = (R)(rad * s);
        y[e] = o;
    }
}

template <typename R>
hipError_t launch_random(cx<R>* y, long count, unsigned long long seed, double scale, hipStream_t st) {
    hipLaunchKernelGGL((k_random<R>), dim3(grid_for(count)), dim3(256), 0, st, y, count, seed, scale);
    return hipGetLastError();
}

hipError_t configure_block_kernels() {
    const int maxb = 160 * 1024;
    hipError_t e = hipFuncSetAttribute((const void*)k_gram<float>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_gram<double>, hipFuncAttributeMaxDynamicSharedMemorySize, maxb);
}

template hipError_t launch_random<float>(cx<float>*, long, unsigned long long, double, hipStream_t);
template hipError_t launch_random<double>(cx<double>*, long, unsigned long long, double, hipStream_t);
template hipError_t launch_gram<float>(const ColSet&, const ColSet&, long, cx<double>*, int, cx<double>*, hipStream_t);
template hipError_t launch_gram<double>(const ColSet&, const ColSet&, long, cx<double>*, int, cx<double>*, hipStream_t);
template hipError_t launch_combine<float>(const ColSet&, const cx<double>*, const ColSet&, long, hipStream_t);
template hipError_t launch_combine<double>(const ColSet&, const cx<double>*, const ColSet&, long, hipStream_t);
template hipError_t launch_residual<float>(const ColSet&, const ColSet&, const double*, const double*, long,
                                           const ColSet&, double*, int, double*, hipStream_t);
template hipError_t launch_residual<double>(const ColSet&, const ColSet&, const double*, const double*, long,
                                            const ColSet&, double*, int, double*, hipStream_t);
template hipError_t launch_mask<float>(cx<float>*, const double*, long, int, hipStream_t);
template hipError_t launch_mask<double>(cx<double>*, const double*, long, int, hipStream_t);

}  // namespace pcx
