// Block-vector kernels for the LOBPCG driver: Gram products A^H B (FP64 accumulation),
// small-matrix combinations S C, residual + Lambda_q^{-1} preconditioner, conversions.
// Vectors are columns of length N stored contiguously; a ColSet lists up to 4 runs of columns.
#include "pcx_internal.h"

namespace pcx {

#define DEV __device__ __forceinline__

constexpr int kMaxCols = 6 * PCX_MAX_BLOCK;

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
// Each work-group stages kGramRows rows of all A and B columns in LDS, and each thread accumulates
// a BLK x BLK tile of Gram entries (a pair of column blocks) in FP64.  Within a staged row the
// columns are interleaved by block: column u of block q sits at u * nblocks + q, so the lanes of a
// wave, which hold consecutive blocks, read consecutive 16-byte words (no bank conflicts).
// HERM: B = [A] or [A | A'] (kb = nh ka, nh = 1 or 2; the first ka columns of B are the columns of
// A) with every ka x ka half of A^H B Hermitian, so A is staged once, as B's first half, and only
// the block upper triangle of each half is computed (the caller mirrors the rest).
// The source column and the interleaved position of every tile column are worked out once per
// work-group (tables in LDS), so staging a row tile is a table read, a load and a store.
constexpr int kGramRows = 16;
constexpr int kTileCols = 2 * kMaxCols + 8;    // A and B columns with block padding
constexpr int kMaxPB = 2;      // pair-blocks per thread (MPB = 1 or 2 per instantiation)

template <int BLK, bool HERM>
DEV void pair_block(int pb, int nbA, int nbB, int* ba, int* bb) {
    if (!HERM) {
        *ba = pb / nbB;
        *bb = pb % nbB;
        return;
    }
    const int tri = nbA * (nbA + 1) / 2;
    const int h = pb / tri;
    int rem = pb - h * tri, row = 0;
    while (rem >= nbA - row) {
        rem -= nbA - row;
        ++row;
    }
    *ba = row;
    *bb = h * nbA + row + rem;          // block column within the (ka-aligned) B layout
}

template <typename R, int BLK, bool HERM, int MPB>
__global__ void __launch_bounds__(256) k_gram(ColSet A, ColSet B, long N, long rows_per_chunk,
                                               cx<double>* __restrict__ part) {
    extern __shared__ __align__(16) char lds[];
    const int ka = A.total(), kb = B.total();
    const int kaP = (ka + BLK - 1) / BLK * BLK;
    // B columns in LDS: plain, or (HERM) each half padded to kaP so blocks never straddle halves
    const int kbP = HERM ? (kb / ka) * kaP : (kb + BLK - 1) / BLK * BLK;
    const int bofs = HERM ? 0 : kaP;                    // first B column in the tile
    const int ncol = bofs + kbP;
    const int ldr = ncol + 1;                           // row stride (complex), padded
    cx<double>* T = (cx<double>*)lds;                   // [kGramRows][ldr]: A columns then B columns
    const cx<R>** tsrc = (const cx<R>**)(T + (size_t)kGramRows * ldr);   // [ncol] source column or null
    int* tpos = (int*)(tsrc + kTileCols);                                 // [ncol] interleaved position
    const long r0 = (long)blockIdx.x * rows_per_chunk;
    const long r1 = min(N, r0 + rows_per_chunk);
    const int nbA = kaP / BLK, nbB = kbP / BLK;
    const int PB = HERM ? (kb / ka) * nbA * (nbA + 1) / 2 : nbA * nbB;
    // padded column c of the tile: A columns [0, kaP) unless HERM, then B columns (HERM: half h at
    // h kaP), stored at its interleaved position
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
        const cx<R>* src = nullptr;
        int pos;
        if (c < bofs) {
            pos = (c % BLK) * nbA + c / BLK;
            if (c < ka) src = col_ptr<const cx<R>>(A, c, N);
        } else {
            int cb = c - bofs;
            pos = bofs + (cb % BLK) * nbB + cb / BLK;
            if (HERM) {
                const int h = cb / kaP, q = cb % kaP;
                cb = q < ka ? h * ka + q : -1;
            }
            if (cb >= 0 && cb < kb) src = col_ptr<const cx<R>>(B, cb, N);
        }
        tsrc[c] = src;
        tpos[c] = pos;
    }
    int pba[MPB], pbb[MPB];
#pragma unroll
    for (int p = 0; p < MPB; ++p) {
        // gridDim.y slices of MPB * 256 pair-blocks each
        const int pb = blockIdx.y * MPB * (int)blockDim.x + threadIdx.x + p * blockDim.x;
        pba[p] = pbb[p] = -1;
        if (pb < PB) pair_block<BLK, HERM>(pb, nbA, nbB, &pba[p], &pbb[p]);
    }
    cx<double> acc[MPB][BLK][BLK];
#pragma unroll
    for (int p = 0; p < MPB; ++p)
#pragma unroll
        for (int u = 0; u < BLK; ++u)
#pragma unroll
            for (int w = 0; w < BLK; ++w) acc[p][u][w].x = acc[p][u][w].y = 0.0;
    __syncthreads();

    for (long rt = r0; rt < r1; rt += kGramRows) {
        const int rows = (int)min((long)kGramRows, r1 - rt);
        for (int e = threadIdx.x; e < ncol * kGramRows; e += blockDim.x) {
            const int c = e / kGramRows, r = e % kGramRows;
            const cx<R>* src = tsrc[c];
            cx<double> val;
            val.x = val.y = 0.0;
            if (src && r < rows) val = to64(src[rt + r]);
            T[(size_t)r * ldr + tpos[c]] = val;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < MPB; ++p) {
            if (pba[p] >= 0) {
                // HERM: A is B's first half, interleaved with B's block count
                const int sa = HERM ? nbB : nbA;
                const cx<double>* ap = T + pba[p];
                const cx<double>* bp = T + bofs + pbb[p];
#pragma unroll 4
                for (int r = 0; r < kGramRows; ++r) {
                    cx<double> av[BLK], bv[BLK];
#pragma unroll
                    for (int u = 0; u < BLK; ++u) av[u] = ap[(size_t)r * ldr + u * sa];
#pragma unroll
                    for (int w = 0; w < BLK; ++w) bv[w] = bp[(size_t)r * ldr + w * nbB];
#pragma unroll
                    for (int u = 0; u < BLK; ++u)
#pragma unroll
                        for (int w = 0; w < BLK; ++w) {
                            // conj(a) * b, as a chain of FMAs into the accumulator
                            acc[p][u][w].x = fma(av[u].x, bv[w].x, acc[p][u][w].x);
                            acc[p][u][w].x = fma(av[u].y, bv[w].y, acc[p][u][w].x);
                            acc[p][u][w].y = fma(av[u].x, bv[w].y, acc[p][u][w].y);
                            acc[p][u][w].y = fma(-av[u].y, bv[w].x, acc[p][u][w].y);
                        }
                }
            }
        }
        __syncthreads();
    }
    cx<double>* out = part + (size_t)blockIdx.x * ka * kb;
#pragma unroll
    for (int p = 0; p < MPB; ++p) {
        if (pba[p] >= 0) {
#pragma unroll
            for (int u = 0; u < BLK; ++u)
#pragma unroll
                for (int w = 0; w < BLK; ++w) {
                    const int ia = pba[p] * BLK + u;
                    int ib = pbb[p] * BLK + w;
                    if (HERM) {
                        const int h = ib / kaP, q = ib % kaP;
                        ib = q < ka ? h * ka + q : kb;
                    }
                    if (ia < ka && ib < kb) out[(size_t)ia * kb + ib] = acc[p][u][w];
                }
        }
    }
}

// out[e] = sum over chunks of part[c][e]: stage 1 sums chunk groups in parallel, stage 2 the groups
constexpr int kRedGroups = 32;

__global__ void k_reduce_stage1(const cx<double>* __restrict__ part, int nchunk, int count,
                                cx<double>* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (e >= count) return;
    double sx = 0.0, sy = 0.0;
    for (int c = g; c < nchunk; c += kRedGroups) {
        const cx<double> v = part[(size_t)c * count + e];
        sx += v.x;
        sy += v.y;
    }
    out[(size_t)g * count + e].x = sx;
    out[(size_t)g * count + e].y = sy;
}

__global__ void k_reduce_stage2(const cx<double>* __restrict__ mid, int count, cx<double>* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double sx = 0.0, sy = 0.0;
    for (int g = 0; g < kRedGroups; ++g) {
        const cx<double> v = mid[(size_t)g * count + e];
        sx += v.x;
        sy += v.y;
    }
    out[e].x = sx;
    out[e].y = sy;
}

template <typename R, int BLK, bool HERM>
static hipError_t gram_impl(const ColSet& A, const ColSet& B, long N, cx<double>* part, int chunks, long rpc,
                            hipStream_t st) {
    const int ka = A.total(), kb = B.total();
    const int kaP = (ka + BLK - 1) / BLK * BLK;
    const int kbP = HERM ? (kb / ka) * kaP : (kb + BLK - 1) / BLK * BLK;
    const int nbA = kaP / BLK, nbB = kbP / BLK;
    const int PB = HERM ? (kb / ka) * nbA * (nbA + 1) / 2 : nbA * nbB;
    const size_t lds = sizeof(cx<double>) * (size_t)kGramRows * ((HERM ? 0 : kaP) + kbP + 1) +
                       (sizeof(void*) + sizeof(int)) * kTileCols;
    // more than kMaxPB * 256 pair-blocks: slices of them in separate work-groups (grid y)
    const int slices = (PB + kMaxPB * 256 - 1) / (kMaxPB * 256);
    if (PB <= 256)
        hipLaunchKernelGGL((k_gram<R, BLK, HERM, 1>), dim3(chunks), dim3(256), lds, st, A, B, N, rpc, part);
    else
        hipLaunchKernelGGL((k_gram<R, BLK, HERM, 2>), dim3(chunks, slices), dim3(256), lds, st, A, B, N, rpc,
                           part);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gram(const ColSet& A, const ColSet& B, long N, cx<double>* part, int nchunk, cx<double>* out,
                       hipStream_t st, bool herm) {
    const int ka = A.total(), kb = B.total();
    if (ka < 1 || kb < 1 || ka > kMaxCols || kb > kMaxCols) return hipErrorInvalidValue;
    if (herm && kb != ka && kb != 2 * ka) return hipErrorInvalidValue;
    long rpc = (N + nchunk - 1) / nchunk;
    rpc = (rpc + kGramRows - 1) / kGramRows * kGramRows;
    const int chunks = (int)((N + rpc - 1) / rpc);
    // register tile: every thread of the group waits for the busiest, so the cost of a tile size
    // is (rounds of 256 pair-blocks) x BLK^2; the cheapest, larger BLK on ties (fewer LDS reads per
    // product).  A second round (two pair-blocks per thread) counts 2.5: half the group idles
    // through it and the doubled registers lower the occupancy (measured: the 36-column Hermitian
    // Rayleigh-Ritz product takes 207 us with BLK 3 in one round, 248 us with BLK 2 in two); beyond
    // 2 rounds the pair-blocks go to several work-groups per row chunk, each of which stages the
    // rows again, so those rounds count double
    hipError_t e;
    auto pbs = [&](int blk) {
        const int a = (ka + blk - 1) / blk;
        return herm ? (kb / ka) * a * (a + 1) / 2 : a * ((kb + blk - 1) / blk);
    };
    int blk = 4;
    double best = -1;
    for (int t = 4; t >= 1; --t) {
        const int pb = pbs(t);
        const long rounds = (pb + 255) / 256;
        const double cost = (rounds == 1 ? 1.0 : rounds <= kMaxPB ? 2.5 : 2.0 * rounds) * t * t;
        if (best < 0 || cost < best) {
            best = cost;
            blk = t;
        }
    }
    switch (blk * 2 + (herm ? 1 : 0)) {
        case 2: e = gram_impl<R, 1, false>(A, B, N, part, chunks, rpc, st); break;
        case 3: e = gram_impl<R, 1, true>(A, B, N, part, chunks, rpc, st); break;
        case 4: e = gram_impl<R, 2, false>(A, B, N, part, chunks, rpc, st); break;
        case 5: e = gram_impl<R, 2, true>(A, B, N, part, chunks, rpc, st); break;
        case 6: e = gram_impl<R, 3, false>(A, B, N, part, chunks, rpc, st); break;
        case 7: e = gram_impl<R, 3, true>(A, B, N, part, chunks, rpc, st); break;
        case 8: e = gram_impl<R, 4, false>(A, B, N, part, chunks, rpc, st); break;
        default: e = gram_impl<R, 4, true>(A, B, N, part, chunks, rpc, st); break;
    }
    if (e != hipSuccess) return e;
    const int count = ka * kb;
    cx<double>* mid = part + (size_t)chunks * count;
    hipLaunchKernelGGL(k_reduce_stage1, dim3((count + 255) / 256, kRedGroups), dim3(256), 0, st, part, chunks, count,
                       mid);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_stage2, dim3((count + 255) / 256), dim3(256), 0, st, mid, count, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Y = S C
// Each thread takes kRowsPerThread rows (a work-group's rows are consecutive per pass, so every
// column access is coalesced), and the outputs in chunks of kOutChunk FP64 accumulators per row,
// S re-read per chunk (from L2 when the work-group's rows are still resident).  C (ks x m) is
// staged in LDS when it fits and read there by all lanes at once (a broadcast, reused for all the
// thread's rows), else taken through the scalar cache.
#ifndef PCX_COMBINE_CHUNK
#define PCX_COMBINE_CHUNK 12
#endif
#ifndef PCX_COMBINE_ROWS
#define PCX_COMBINE_ROWS 2
#endif
constexpr int kOutChunk = PCX_COMBINE_CHUNK;
constexpr int kRowsPerThread = PCX_COMBINE_ROWS;
constexpr int kCombineLds = 64 * 1024;     // C in LDS up to this size

template <typename R, bool CLDS>
__global__ void __launch_bounds__(256) k_combine(ColSet S, const cx<double>* __restrict__ C, ColSet Y, long N) {
    extern __shared__ __align__(16) char lds[];
    __shared__ const cx<R>* scol[kMaxCols];
    __shared__ cx<R>* ycol[kMaxCols];
    const int ks = S.total(), m = Y.total();
    for (int c = threadIdx.x; c < ks; c += blockDim.x) scol[c] = col_ptr<const cx<R>>(S, c, N);
    for (int c = threadIdx.x; c < m; c += blockDim.x) ycol[c] = col_ptr<cx<R>>(Y, c, N);
    const cx<double>* Cm = C;
    if (CLDS) {
        cx<double>* Cs = (cx<double>*)lds;
        for (int e = threadIdx.x; e < ks * m; e += blockDim.x) Cs[e] = C[e];
        Cm = Cs;
    }
    __syncthreads();
    const long span = (long)blockDim.x * kRowsPerThread;
    for (long base = blockIdx.x * span; base < N; base += (long)gridDim.x * span) {
        long row[kRowsPerThread];
#pragma unroll
        for (int j = 0; j < kRowsPerThread; ++j) row[j] = base + threadIdx.x + (long)j * blockDim.x;
        for (int m0 = 0; m0 < m; m0 += kOutChunk) {
            cx<double> acc[kRowsPerThread][kOutChunk];
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j)
#pragma unroll
                for (int u = 0; u < kOutChunk; ++u) acc[j][u].x = acc[j][u].y = 0.0;
            for (int k = 0; k < ks; ++k) {
                cx<double> s[kRowsPerThread];
#pragma unroll
                for (int j = 0; j < kRowsPerThread; ++j) {
                    s[j].x = s[j].y = 0.0;
                    if (row[j] < N) s[j] = to64(scol[k][row[j]]);
                }
                const cx<double>* crow = Cm + (size_t)k * m + m0;
#pragma unroll
                for (int u = 0; u < kOutChunk; ++u) {
                    if (m0 + u < m) {
                        const cx<double> c = crow[u];
#pragma unroll
                        for (int j = 0; j < kRowsPerThread; ++j) {
                            acc[j][u].x = fma(s[j].x, c.x, acc[j][u].x);
                            acc[j][u].x = fma(-s[j].y, c.y, acc[j][u].x);
                            acc[j][u].y = fma(s[j].x, c.y, acc[j][u].y);
                            acc[j][u].y = fma(s[j].y, c.x, acc[j][u].y);
                        }
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kRowsPerThread; ++j) {
                if (row[j] >= N) continue;
#pragma unroll
                for (int u = 0; u < kOutChunk; ++u) {
                    if (m0 + u < m) {
                        cx<R> o;
                        o.x = (R)acc[j][u].x;
                        o.y = (R)acc[j][u].y;
                        ycol[m0 + u][row[j]] = o;
                    }
                }
            }
        }
    }
}

template <typename R>
hipError_t launch_combine(const ColSet& S, const cx<double>* C, const ColSet& Y, long N, hipStream_t st) {
    if (S.total() < 1 || Y.total() < 1 || S.total() > kMaxCols || Y.total() > kMaxCols) return hipErrorInvalidValue;
    const long span = 256L * kRowsPerThread;
    long blocks = (N + span - 1) / span;
    if (blocks > 8192) blocks = 8192;
    const size_t cbytes = sizeof(cx<double>) * (size_t)S.total() * Y.total();
    if (cbytes <= (size_t)kCombineLds)
        hipLaunchKernelGGL((k_combine<R, true>), dim3((unsigned)blocks), dim3(256), cbytes, st, S, C, Y, N);
    else
        hipLaunchKernelGGL((k_combine<R, false>), dim3((unsigned)blocks), dim3(256), 0, st, S, C, Y, N);
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
            s = fma(rx, rx, s);
            s = fma(ry, ry, s);
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

// out[e] = sum over chunks of part[c][e]; one work-group per entry e
__global__ void __launch_bounds__(256) k_reduce_real(const double* __restrict__ part, int nchunk, int count,
                                                      double* __restrict__ out) {
    __shared__ double red[4];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += blockDim.x) s += part[(size_t)c * count + e];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[e] = s;
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
    hipLaunchKernelGGL(k_reduce_real, dim3(count), dim3(256), 0, st, part, chunks, count, out);
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

template <typename RI, typename RO>
__global__ void k_scale_modes(const cx<RI>* in, cx<RO>* out, const double* __restrict__ prec, long n, long count) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const double d = prec[e % n];
        const cx<RI> v = in[e];
        cx<RO> o;
        o.x = (RO)(d * (double)v.x);
        o.y = (RO)(d * (double)v.y);
        out[e] = o;
    }
}

template <typename R>
hipError_t launch_scale_modes(const cx<R>* in, cx<R>* out, const double* prec, long n, int nvec, hipStream_t st) {
    const long count = 2 * n * (long)nvec;
    hipLaunchKernelGGL((k_scale_modes<R, R>), dim3(grid_for(count)), dim3(256), 0, st, in, out, prec, n, count);
    return hipGetLastError();
}

hipError_t launch_scale_modes(const cx<float>* in, cx<double>* out, const double* prec, long n, int nvec,
                              hipStream_t st) {
    const long count = 2 * n * (long)nvec;
    hipLaunchKernelGGL((k_scale_modes<float, double>), dim3(grid_for(count)), dim3(256), 0, st, in, out, prec, n,
                       count);
    return hipGetLastError();
}

// y = a x + b y (complex a, b), FP64
__global__ void k_axpby(const cx<double>* __restrict__ x, cx<double>* __restrict__ y, double ar, double ai, double br,
                        double bi, long count) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const cx<double> u = x[e], v = y[e];
        cx<double> o;
        o.x = ar * u.x - ai * u.y + br * v.x - bi * v.y;
        o.y = ar * u.y + ai * u.x + br * v.y + bi * v.x;
        y[e] = o;
    }
}

hipError_t launch_axpby(const cx<double>* x, cx<double>* y, cx<double> a, cx<double> b, long count, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(count)), dim3(256), 0, st, x, y, a.x, a.y, b.x, b.y, count);
    return hipGetLastError();
}

// sum_e conj(a_e) b_e over count entries: per-work-group partial sums, then one work-group adds them
constexpr int kDotGroups = 1024;

__global__ void __launch_bounds__(256) k_dot_part(const cx<double>* __restrict__ a, const cx<double>* __restrict__ b,
                                                  long count, cx<double>* __restrict__ part) {
    __shared__ double rx[4], ry[4];
    double sx = 0.0, sy = 0.0;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x) {
        const cx<double> u = a[e], v = b[e];
        sx = fma(u.x, v.x, sx);
        sx = fma(u.y, v.y, sx);
        sy = fma(u.x, v.y, sy);
        sy = fma(-u.y, v.x, sy);
    }
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        rx[wid] = sx;
        ry[wid] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cx<double> o;
        o.x = rx[0] + rx[1] + rx[2] + rx[3];
        o.y = ry[0] + ry[1] + ry[2] + ry[3];
        part[blockIdx.x] = o;
    }
}

__global__ void __launch_bounds__(256) k_dot_final(const cx<double>* __restrict__ part, int nparts,
                                                   cx<double>* __restrict__ out) {
    __shared__ double rx[4], ry[4];
    double sx = 0.0, sy = 0.0;
    for (int e = threadIdx.x; e < nparts; e += blockDim.x) {
        sx += part[e].x;
        sy += part[e].y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        rx[wid] = sx;
        ry[wid] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out->x = rx[0] + rx[1] + rx[2] + rx[3];
        out->y = ry[0] + ry[1] + ry[2] + ry[3];
    }
}

hipError_t launch_dot(const cx<double>* a, const cx<double>* b, long count, cx<double>* part, cx<double>* out,
                      hipStream_t st) {
    long blocks = (count + 255) / 256;
    if (blocks > kDotGroups) blocks = kDotGroups;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_dot_part, dim3((unsigned)blocks), dim3(256), 0, st, a, b, count, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, part, (int)blocks, out);
    return hipGetLastError();
}

__global__ void k_sqrt(const double* __restrict__ in, double* __restrict__ out, long count) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count; e += (long)gridDim.x * blockDim.x)
        out[e] = sqrt(in[e]);
}

hipError_t launch_sqrt(const double* in, double* out, long count, hipStream_t st) {
    hipLaunchKernelGGL(k_sqrt, dim3(grid_for(count)), dim3(256), 0, st, in, out, count);
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

template <typename R>
__global__ void k_set_units(cx<R>* __restrict__ y, UnitList u) {
    const int c = threadIdx.x;
    if (c < u.count) {
        cx<R> o;
        o.x = (R)1;
        o.y = (R)0;
        y[u.idx[c]] = o;
    }
}

template <typename R>
hipError_t launch_set_units(cx<R>* y, const UnitList& u, hipStream_t st) {
    if (u.count < 1) return hipSuccess;
    hipLaunchKernelGGL((k_set_units<R>), dim3(1), dim3(PCX_MAX_BLOCK), 0, st, y, u);
    return hipGetLastError();
}

template <typename R, int BLK, bool HERM>
static hipError_t set_gram_lds() {
    hipError_t e = hipFuncSetAttribute((const void*)k_gram<R, BLK, HERM, 1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_gram<R, BLK, HERM, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}

hipError_t configure_block_kernels() {
    hipError_t e = hipSuccess;
#define G(R, B, H) \
    if (e == hipSuccess) e = set_gram_lds<R, B, H>()
    G(float, 1, false); G(float, 2, false); G(float, 3, false); G(float, 4, false);
    G(float, 1, true); G(float, 2, true); G(float, 3, true); G(float, 4, true);
    G(double, 1, false); G(double, 2, false); G(double, 3, false); G(double, 4, false);
    G(double, 1, true); G(double, 2, true); G(double, 3, true); G(double, 4, true);
#undef G
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_combine<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kCombineLds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_combine<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kCombineLds);
    return e;
}

template hipError_t launch_random<float>(cx<float>*, long, unsigned long long, double, hipStream_t);
template hipError_t launch_random<double>(cx<double>*, long, unsigned long long, double, hipStream_t);
template hipError_t launch_set_units<float>(cx<float>*, const UnitList&, hipStream_t);
template hipError_t launch_set_units<double>(cx<double>*, const UnitList&, hipStream_t);
template hipError_t launch_gram<float>(const ColSet&, const ColSet&, long, cx<double>*, int, cx<double>*, hipStream_t,
                                       bool);
template hipError_t launch_gram<double>(const ColSet&, const ColSet&, long, cx<double>*, int, cx<double>*, hipStream_t,
                                        bool);
template hipError_t launch_combine<float>(const ColSet&, const cx<double>*, const ColSet&, long, hipStream_t);
template hipError_t launch_combine<double>(const ColSet&, const cx<double>*, const ColSet&, long, hipStream_t);
template hipError_t launch_residual<float>(const ColSet&, const ColSet&, const double*, const double*, long,
                                           const ColSet&, double*, int, double*, hipStream_t);
template hipError_t launch_residual<double>(const ColSet&, const ColSet&, const double*, const double*, long,
                                            const ColSet&, double*, int, double*, hipStream_t);
template hipError_t launch_mask<float>(cx<float>*, const double*, long, int, hipStream_t);
template hipError_t launch_mask<double>(cx<double>*, const double*, long, int, hipStream_t);
template hipError_t launch_scale_modes<float>(const cx<float>*, cx<float>*, const double*, long, int, hipStream_t);
template hipError_t launch_scale_modes<double>(const cx<double>*, cx<double>*, const double*, long, int, hipStream_t);

}  // namespace pcx
