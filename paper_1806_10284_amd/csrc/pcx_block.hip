// Block-vector kernels for the LOBPCG driver: Gram products A^H B (FP64 accumulation),
// small-matrix combinations S C, residual + Lambda_q^{-1} preconditioner, conversions.
// Vectors are columns of length N stored contiguously; a ColSet lists up to 4 runs of columns.
#include "pcx_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>

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

// ------------------------------------------------------------------ Gram on the matrix cores
// The Hermitian layouts (B = [A] or [A | A'], every ka x ka half Hermitian) with ka <= kMfmaMaxA go
// through FP64 4x4x4 MFMA products with four blocks per instruction.  A complex inner product is
// a real one over a K index that runs over (row, real/imaginary part): with a_k = (Re a, Im a) and
// b_k = (Re b, Im b), Re(conj(a) b) = sum_k a_k b_k, and with a'_k = (-Im a, Re a),
// Im(conj(a) b) = sum_k a'_k b_k.  An instruction takes K = 4 (two rows) in each of its blocks,
// i.e. eight rows of one 4 x 4 tile of G, and the four blocks' partial sums are added at the end.
// Operand lane l holds element (m, k) of block q, m = l & 3 (the column within the tile),
// q = (l >> 2) & 3, k = l >> 4; result element (i, j) of block q sits in lane 16 i + 4 q + j.
// The partner k ^ 1 that a' needs sits in lane l ^ 16: one lane swap (v_permlane16_swap) and a
// sign flip turn a into a'.
//
// Rows reach LDS by direct global-to-LDS loads (16 bytes per lane, lane L written at 16 L of a
// 1 KB unit), so the number of bytes in flight is bounded by LDS, not by registers.  A unit holds
// one tile of four columns over 16 rows (FP64) or 32 rows (FP32), with the lanes' rows chosen so
// that the operand of lane l is
//   FP64: element 32 g + 16 (l >> 5) + (l & 15) of the unit, half (l >> 4) & 1,
//   FP32: 16-byte chunk 16 g + (l & 15) (rows 2 q, 2 q + 1 of column m), float l >> 4,
// for the group g of eight rows: a wave's operand read is 512 contiguous bytes (FP64) or 256
// (FP32), free of bank conflicts.  A stage is `sub` row blocks of all tiles; `slots` stages rotate
// through LDS, slots - 1 of them in flight while the waves multiply the oldest, with one barrier
// per stage.  Rows past the end and padding columns load from a zero block.
//
// Work split: 512 threads, eight waves, two per SIMD.  With two halves (NH = 2) waves 0-3 take
// half 0 and waves 4-7 half 1; within a half, the upper-triangle tile pairs (I, J >= I) are split
// at a tile row into two sets of about equal size (I < IS and I >= IS), and each set goes to two
// waves that alternate over the groups of eight rows (with one half, to four waves).  A wave
// reads the A and B tiles of its set for a group once, into registers, and issues the set's
// products fully unrolled (NT a template parameter), holding the real and imaginary accumulators
// of its pairs for the whole row chunk; while they run, the reads of the next group are in
// flight.  The waves of a set add their accumulators through LDS at the end.
#ifndef PCX_MFMA_LDS
#define PCX_MFMA_LDS (76 * 1024)
#endif
#ifndef PCX_MFMA_LDS1
#define PCX_MFMA_LDS1 (150 * 1024)
#endif
#ifndef PCX_DMA_UNITS
#define PCX_DMA_UNITS 16
#endif
#ifndef PCX_DMA_SLOTS
#define PCX_DMA_SLOTS 8
#endif
constexpr int kMfmaMaxNT = 12;
constexpr int kMfmaMaxA = 4 * kMfmaMaxNT;
constexpr int kMfmaLds = PCX_MFMA_LDS;         // LDS for the stage slots, two work-groups per CU
constexpr int kMfmaLds1 = PCX_MFMA_LDS1;       // the same, one work-group per CU
constexpr int kDmaUnits = PCX_DMA_UNITS;       // 1 KB units per stage aimed at
constexpr int kDmaSlots = PCX_DMA_SLOTS;       // most stage slots
constexpr int kMfmaThreads = 512;              // eight waves
constexpr int kMfmaWaves = kMfmaThreads / 64;
constexpr int kDmaMaxUPW = 3;                  // units per wave and stage (at most 24 per stage)

__device__ __align__(16) double g_dma_zero[2];   // never written: the zero block

// tile counts up to this run two work-groups per CU (the accumulators' registers allow it)
constexpr int kMfmaTwoGroupsNT = 5;

// first tile row of the second pair set: the smallest IS with at least half of the
// nt (nt + 1) / 2 pairs in rows I < IS
__host__ __device__ constexpr int mfma_split(int nt) {
    int is = 0, c = 0;
    while (2 * c < nt * (nt + 1) / 2) c += nt - is++;
    return is;
}
__host__ __device__ constexpr int mfma_set_pairs(int nt, int set) {
    int c = 0;
    for (int I = set ? mfma_split(nt) : 0; I < (set ? nt : mfma_split(nt)); ++I) c += nt - I;
    return c;
}

struct DmaShape {
    int sub, units, slot_bytes, slots, lds_bytes;
};
// nphase: waves that alternate over one half's groups of eight rows
__host__ __device__ inline int mfma_phases(int nh) { return nh == 2 ? 2 : 4; }
__host__ __device__ inline DmaShape dma_shape(int ka, int kb, bool f64) {
    DmaShape d;
    const int nt = (ka + 3) / 4, nh = kb / ka, ntiles = nh * nt;
    d.sub = kDmaUnits / ntiles < 1 ? 1 : kDmaUnits / ntiles;
    // every wave of a half gets the same number of groups: sub * (groups per row block) a
    // multiple of the phases
    if (f64 && mfma_phases(nh) == 4 && (d.sub & 1)) ++d.sub;
    while (d.sub > 1 && d.sub * ntiles > kMfmaWaves * kDmaMaxUPW) d.sub -= f64 && mfma_phases(nh) == 4 ? 2 : 1;
    if (d.sub < 1) d.sub = 1;
    d.units = d.sub * ntiles;
    d.slot_bytes = d.units * 1024;
    d.slots = (nt <= kMfmaTwoGroupsNT ? kMfmaLds : kMfmaLds1) / d.slot_bytes;
    if (d.slots > kDmaSlots) d.slots = kDmaSlots;
    if (d.slots < 2) d.slots = 2;
    // the final reduction: the other phases' partial sums of every pair of both sets, 16 lanes x
    // 16 bytes each
    const int ps = mfma_set_pairs(nt, 0) > mfma_set_pairs(nt, 1) ? mfma_set_pairs(nt, 0) : mfma_set_pairs(nt, 1);
    const int red = nh * 2 * (mfma_phases(nh) - 1) * ps * 256;
    d.lds_bytes = d.slots * d.slot_bytes > red ? d.slots * d.slot_bytes : red;
    return d;
}

DEV double flip_sign(double x, unsigned hi_mask) {
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    u ^= (unsigned long long)hi_mask << 32;
    return __longlong_as_double((long long)u);
}

// the value of lane l ^ 16: v_permlane16_swap of x with itself returns the even 16-lane rows'
// values in its first result and the odd rows' in its second
DEV unsigned swap16(unsigned x) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
}
DEV double swap16(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = swap16((unsigned)u), hi = swap16((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One 16-byte-per-lane global-to-LDS load: lane L's 16 bytes land at LDS byte lds_addr + 16 L
// (lds_addr wave-uniform).  Written as an instruction rather than the builtin so that the compiler
// does not order every later LDS read after it (it cannot tell which stage slot a read touches);
// the kernel waits for these loads itself (wait_then_barrier).  The load has no register result.
DEV void dma16(const void* src, unsigned lds_addr) {
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds_addr) : "memory", "m0");
}

// wait until at most n of this wave's global loads are outstanding (n wave-uniform; the counter
// holds at most 63, a larger n waits for 63) and its LDS reads are done, then the work-group barrier
DEV void wait_then_barrier(int n) {
#define W(k) \
    case k: __builtin_amdgcn_s_waitcnt(0x070 | ((k) & 15) | (((k) >> 4) << 14)); break
#define W8(k) W(k); W(k + 1); W(k + 2); W(k + 3); W(k + 4); W(k + 5); W(k + 6); W(k + 7)
    switch (n) {
        W8(0); W8(8); W8(16); W8(24); W8(32); W8(40); W8(48);
        W(56); W(57); W(58); W(59); W(60); W(61); W(62);
        default: __builtin_amdgcn_s_waitcnt(0x070 | 15 | (3 << 14)); break;
    }
#undef W8
#undef W
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <typename R, int NT, int NH>
__global__ void __launch_bounds__(kMfmaThreads) k_gram_mfma(ColSet B, int ka, long N, long rows_per_chunk, int sub,
                                                             int slots, cx<double>* __restrict__ part) {
    constexpr bool F64 = sizeof(R) == 8;
    constexpr int UR = F64 ? 16 : 32;                    // rows per unit
    constexpr int G = UR / 8;                            // groups of eight rows per unit
    constexpr int NPH = NH == 2 ? 2 : 4;                 // waves per set
    constexpr int ntiles = NH * NT;
    constexpr int PSMAX = mfma_set_pairs(NT, 0) > mfma_set_pairs(NT, 1) ? mfma_set_pairs(NT, 0) : mfma_set_pairs(NT, 1);
    extern __shared__ __align__(1024) char lds[];
    const int kb = NH * ka;
    const int U = sub * ntiles, slot_bytes = U * 1024, SR = sub * UR;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int hw = NH == 2 ? wave >> 2 : 0;
    const int set = NH == 2 ? (wave >> 1) & 1 : wave >> 2;
    const int ph = NH == 2 ? wave & 1 : wave & 3;
    const long r0 = (long)blockIdx.x * rows_per_chunk;
    const long r1 = min(N, r0 + rows_per_chunk);
    const int stages = (int)((r1 - r0 + SR - 1) / SR);

    // this wave's units u = wave + 8 i (row block u / ntiles, tile u % ntiles): the column this
    // lane loads and its row within the stage
    const int urow = F64 ? 8 * (lane >> 5) + 2 * ((lane >> 2) & 3) + ((lane >> 4) & 1)
                         : 8 * (lane >> 4) + 2 * ((lane >> 2) & 3);
    const int cw = (U - wave + kMfmaWaves - 1) / kMfmaWaves;
    const cx<R>* colp[kDmaMaxUPW];
    int srow[kDmaMaxUPW];
#pragma unroll
    for (int i = 0; i < kDmaMaxUPW; ++i) {
        const int u = wave + kMfmaWaves * i;
        colp[i] = nullptr;
        srow[i] = 0;
        if (u < U) {
            const int t = u % ntiles, h = t / NT, q = 4 * (t % NT) + (lane & 3);
            if (q < ka) colp[i] = col_ptr<const cx<R>>(B, h * ka + q, N);
            srow[i] = (u / ntiles) * UR + urow;
        }
    }
    const unsigned lds0 = __builtin_amdgcn_readfirstlane(
        (unsigned)(size_t)(__attribute__((address_space(3))) char*)lds);
    const void* zero = (const void*)g_dma_zero;
    auto issue = [&](int s) {
        const unsigned dst = lds0 + (unsigned)((s % slots) * slot_bytes) + (unsigned)(wave * 1024);
        const long rs = r0 + (long)s * SR;
#pragma unroll
        for (int i = 0; i < kDmaMaxUPW; ++i) {
            if (i < cw) {
                const long row = rs + srow[i];
                dma16((colp[i] && row < r1) ? (const void*)(colp[i] + row) : zero,
                      dst + (unsigned)(kMfmaWaves * i * 1024));
            }
        }
    };

    const unsigned neg = ((lane >> 4) & 1) ? 0u : 0x80000000u;   // a' = (-Im a, Re a)
    const int lo = F64 ? (16 * (lane >> 5) + (lane & 15)) * 16 + ((lane >> 4) & 1) * 8 : (lane & 15) * 16 + (lane >> 4) * 4;
    const int bofs = hw * NT * 1024;                              // this wave's half of B

    // The wave's groups of eight rows, in order: gps per stage (group ph + NPH j of the stage),
    // W in all.  A group that opens a stage first waits for that stage's loads and passes the
    // barrier, then queues the loads of a later stage into the slot every wave has finished with.
    const int gps = sub * G / NPH, W = stages * gps;
    auto open_stage = [&](int w) {
        const int s = w / gps;
        wait_then_barrier(min(slots - 2, stages - 1 - s) * cw);
        if (s + slots - 1 < stages) issue(s + slots - 1);
    };
    cx<double>* red = (cx<double>*)lds;    // final reduction: [half][set][phase - 1][pair][16 lanes]
    const int slot16 = (lane >> 4) * 4 + (lane & 3);

    // everything a wave does for the pair set SET: tile rows I in [IB, IE), B tiles J in [IB, NT)
    auto run = [&](auto set_tag) {
        constexpr int SET = decltype(set_tag)::value;
        constexpr int IS = mfma_split(NT);
        constexpr int IB = SET ? IS : 0, IE = SET ? NT : IS;
        constexpr int NA = IE - IB > 0 ? IE - IB : 1, NB = NT - IB > 0 ? NT - IB : 1;
        constexpr int PS = mfma_set_pairs(NT, SET) > 0 ? mfma_set_pairs(NT, SET) : 1;
        double accR[PS], accI[PS];
#pragma unroll
        for (int p = 0; p < PS; ++p) accR[p] = accI[p] = 0.0;

        // raw LDS reads of a group, then, after the products that overlap their latency, a' and b
        auto load = [&](int w, R* ra, R* rb) {
            const int s = w / gps, gg = ph + NPH * (w - s * gps);
            const char* pg = lds + (size_t)(s % slots) * slot_bytes + (size_t)(gg / G) * ntiles * 1024 +
                             (F64 ? 512 : 256) * (gg % G) + lo;
            // an empty set (NT = 1) reads the last tile, whose products it never issues
            constexpr int T0 = IB < NT ? IB : NT - 1;
#pragma unroll
            for (int t = 0; t < NA; ++t) ra[t] = *(const R*)(pg + 1024 * (T0 + t));
#pragma unroll
            for (int t = 0; t < NB; ++t) rb[t] = *(const R*)(pg + bofs + 1024 * (T0 + t));
        };
        auto finish = [&](const R* ra, const R* rb, double* a, double* a2, double* bv) {
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                a[t] = (double)ra[t];
                if (F64)
                    a2[t] = flip_sign(swap16(a[t]), neg);
                else
                    a2[t] = flip_sign((double)__uint_as_float(swap16(__float_as_uint((float)ra[t]))), neg);
            }
#pragma unroll
            for (int t = 0; t < NB; ++t) bv[t] = (double)rb[t];
        };
        auto product = [&](const double* a, const double* a2, const double* bv) {
            int p = 0;
#pragma unroll
            for (int I = IB; I < IE; ++I)
#pragma unroll
                for (int J = I; J < NT; ++J, ++p) {
                    accR[p] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I - IB], bv[J - IB], accR[p], 0, 0, 0);
                    accI[p] = __builtin_amdgcn_mfma_f64_4x4x4f64(a2[I - IB], bv[J - IB], accI[p], 0, 0, 0);
                }
        };

        R ra[NA], rb[NB];
        double a0[NA], b0[NA], c0[NB], a1[NA], b1[NA], c1[NB];   // two sets of (a, a', b)
        open_stage(0);
        load(0, ra, rb);
        finish(ra, rb, a0, b0, c0);
        // the reads are unconditional (past the last group they read the current one again), so
        // that no register copies, which would wait for them, join the branches
        for (int w = 0; w < W; w += 2) {
            const bool more1 = w + 1 < W;
            if (more1 && (w + 1) % gps == 0) open_stage(w + 1);
            load(more1 ? w + 1 : w, ra, rb);
            __builtin_amdgcn_sched_barrier(0);
            product(a0, b0, c0);
            __builtin_amdgcn_sched_barrier(0);
            if (!more1) break;
            finish(ra, rb, a1, b1, c1);
            const bool more2 = w + 2 < W;
            if (more2 && (w + 2) % gps == 0) open_stage(w + 2);
            load(more2 ? w + 2 : w + 1, ra, rb);
            __builtin_amdgcn_sched_barrier(0);
            product(a1, b1, c1);
            __builtin_amdgcn_sched_barrier(0);
            finish(ra, rb, a0, b0, c0);
        }

        // the four blocks of each accumulator, then the phases of the set through LDS (the stage
        // slots are free: the last wait had no load outstanding and every wave is past it)
#pragma unroll
        for (int p = 0; p < PS; ++p) {
            accR[p] += __shfl_xor(accR[p], 4, 64);
            accI[p] += __shfl_xor(accI[p], 4, 64);
            accR[p] += __shfl_xor(accR[p], 8, 64);
            accI[p] += __shfl_xor(accI[p], 8, 64);
        }
        wait_then_barrier(0);
        const size_t rbase = (size_t)((hw * 2 + SET) * (NPH - 1)) * PSMAX;
        if (ph > 0 && (lane & 12) == 0) {
#pragma unroll
            for (int p = 0; p < PS; ++p) {
                cx<double> v;
                v.x = accR[p];
                v.y = accI[p];
                red[(rbase + (size_t)(ph - 1) * PSMAX + p) * 16 + slot16] = v;
            }
        }
        wait_then_barrier(0);
        if (ph == 0 && (lane & 12) == 0 && mfma_set_pairs(NT, SET) > 0) {
            cx<double>* out = part + (size_t)blockIdx.x * ka * kb;
            int p = 0;
#pragma unroll
            for (int I = IB; I < IE; ++I)
#pragma unroll
                for (int J = I; J < NT; ++J, ++p) {
                    double re = accR[p], im = accI[p];
#pragma unroll
                    for (int f = 1; f < NPH; ++f) {
                        const cx<double> v = red[(rbase + (size_t)(f - 1) * PSMAX + p) * 16 + slot16];
                        re += v.x;
                        im += v.y;
                    }
                    const int ia = 4 * I + (lane >> 4), jb = 4 * J + (lane & 3);
                    if (ia < ka && jb < ka) {
                        cx<double> o;
                        o.x = re;
                        o.y = im;
                        out[(size_t)ia * kb + hw * ka + jb] = o;
                    }
                }
        }
    };

    for (int s = 0; s < min(slots - 1, stages); ++s) issue(s);
    if (set == 0)
        run(std::integral_constant<int, 0>{});
    else
        run(std::integral_constant<int, 1>{});
}

template <typename R, int NT, int NH>
static hipError_t gram_mfma_impl(const ColSet& B, int ka, long N, cx<double>* part, int chunks, long rpc,
                                 hipStream_t st) {
    const DmaShape d = dma_shape(ka, B.total(), sizeof(R) == 8);
    hipLaunchKernelGGL((k_gram_mfma<R, NT, NH>), dim3(chunks), dim3(kMfmaThreads), (size_t)d.lds_bytes, st, B, ka, N,
                       rpc, d.sub, d.slots, part);
    return hipGetLastError();
}

template <typename R, int NH>
static hipError_t gram_mfma_nh(const ColSet& B, int ka, long N, cx<double>* part, int chunks, long rpc,
                               hipStream_t st) {
    switch ((ka + 3) / 4) {
        case 1: return gram_mfma_impl<R, 1, NH>(B, ka, N, part, chunks, rpc, st);
        case 2: return gram_mfma_impl<R, 2, NH>(B, ka, N, part, chunks, rpc, st);
        case 3: return gram_mfma_impl<R, 3, NH>(B, ka, N, part, chunks, rpc, st);
        case 4: return gram_mfma_impl<R, 4, NH>(B, ka, N, part, chunks, rpc, st);
        case 5: return gram_mfma_impl<R, 5, NH>(B, ka, N, part, chunks, rpc, st);
        case 6: return gram_mfma_impl<R, 6, NH>(B, ka, N, part, chunks, rpc, st);
        case 7: return gram_mfma_impl<R, 7, NH>(B, ka, N, part, chunks, rpc, st);
        case 8: return gram_mfma_impl<R, 8, NH>(B, ka, N, part, chunks, rpc, st);
        case 9: return gram_mfma_impl<R, 9, NH>(B, ka, N, part, chunks, rpc, st);
        case 10: return gram_mfma_impl<R, 10, NH>(B, ka, N, part, chunks, rpc, st);
        case 11: return gram_mfma_impl<R, 11, NH>(B, ka, N, part, chunks, rpc, st);
        default: return gram_mfma_impl<R, 12, NH>(B, ka, N, part, chunks, rpc, st);
    }
}

// row chunks of the matrix-core Gram: one or two work-groups per CU (by the accumulators' registers)
inline int mfma_groups(int ka) { return (ka + 3) / 4 <= kMfmaTwoGroupsNT ? 512 : 256; }

template <typename R>
static hipError_t gram_mfma(const ColSet& B, int ka, long N, cx<double>* part, int chunks, long rpc,
                            hipStream_t st) {
    return B.total() == 2 * ka ? gram_mfma_nh<R, 2>(B, ka, N, part, chunks, rpc, st)
                               : gram_mfma_nh<R, 1>(B, ka, N, part, chunks, rpc, st);
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

// out = the sum of the chunks' partial Gram matrices (count entries each); the middle stage's
// kRedGroups rows sit after the chunks' rows in part
static hipError_t reduce_chunks(cx<double>* part, int chunks, int count, cx<double>* out, hipStream_t st) {
    cx<double>* mid = part + (size_t)chunks * count;
    hipLaunchKernelGGL(k_reduce_stage1, dim3((count + 255) / 256, kRedGroups), dim3(256), 0, st, part, chunks, count,
                       mid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_stage2, dim3((count + 255) / 256), dim3(256), 0, st, mid, count, out);
    return hipGetLastError();
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

// columns [c0, c0 + nc) of A (runs of columns of length N, complex R)
template <typename R>
static ColSet col_subset(const ColSet& A, int c0, int nc, long N) {
    ColSet s = colset(nullptr, 0);
    int q = 0, at = 0;
    for (int r = 0; r < kMaxSeg && nc > 0; ++r) {
        const int n = A.ncols[r];
        if (c0 < at + n) {
            const int off = c0 - at, take = std::min(n - off, nc);
            s.ptr[q] = (char*)A.ptr[r] + (size_t)off * N * sizeof(cx<R>);
            s.ncols[q] = take;
            ++q;
            c0 += take;
            nc -= take;
        }
        at += n;
    }
    return s;
}

// a tile of a Hermitian product into the full output: the tile's upper-triangle entries (local
// column >= local row, in each of its nh halves) at rows / columns gmap[] of the full ka x nh ka
// matrix
struct TileMap {
    int g[kMfmaMaxA];
};
__global__ void k_scatter_tile(const cx<double>* __restrict__ tile, int kp, int nh, TileMap gm, int ka,
                               cx<double>* __restrict__ out) {
    const int kbp = nh * kp;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kp * kbp; e += gridDim.x * blockDim.x) {
        const int r = e / kbp, cc = e % kbp, h = cc / kp, c = cc % kp;
        if (c >= r) out[(size_t)gm.g[r] * nh * ka + (size_t)h * ka + gm.g[c]] = tile[e];
    }
}

// Hermitian A^H [A | AA] for ka above the matrix-core kernel's width: the ka columns in groups of
// at most 24, one matrix-core product per pair of groups (the columns of both groups, and of their
// halves in B), each tile's upper triangle scattered into out.  Every group pair is read once, so
// the columns are read (groups - 1) times in all.
template <typename R>
static hipError_t gram_mfma_tiled(const ColSet& B, int ka, int nh, long N, cx<double>* part, int nchunk,
                                  cx<double>* out, hipStream_t st) {
    const int G = (ka + 23) / 24;
    int g0[8], gn[8];
    for (int g = 0, at = 0; g < G; ++g) {
        gn[g] = (ka - at + (G - g) - 1) / (G - g);
        g0[g] = at;
        at += gn[g];
    }
    for (int i = 0; i < G; ++i)
        for (int j = i + 1; j < G; ++j) {
            const int kp = gn[i] + gn[j];
            ColSet Bp = concat(col_subset<R>(B, g0[i], gn[i], N), col_subset<R>(B, g0[j], gn[j], N));
            if (nh == 2)
                Bp = concat(Bp, concat(col_subset<R>(B, ka + g0[i], gn[i], N), col_subset<R>(B, ka + g0[j], gn[j], N)));
            int segs = 0;
            for (int q = 0; q < kMaxSeg; ++q) segs += Bp.ncols[q] > 0;
            if (Bp.total() != nh * kp) return hipErrorInvalidValue;     // more runs than a ColSet holds
            (void)segs;
            const long groups = std::min<long>(nchunk, mfma_groups(kp));
            const DmaShape d = dma_shape(kp, nh * kp, sizeof(R) == 8);
            const long SR = (long)d.sub * (sizeof(R) == 8 ? 16 : 32);
            long rpc = (N + groups - 1) / groups;
            rpc = (rpc + SR - 1) / SR * SR;
            const int chunks = (int)((N + rpc - 1) / rpc);
            const int count = kp * nh * kp;
            cx<double>* tile = part + (size_t)(chunks + kRedGroups) * count;
            hipError_t e = gram_mfma<R>(Bp, kp, N, part, chunks, rpc, st);
            if (e == hipSuccess) e = reduce_chunks(part, chunks, count, tile, st);
            if (e != hipSuccess) return e;
            TileMap gm;
            for (int r = 0; r < gn[i]; ++r) gm.g[r] = g0[i] + r;
            for (int r = 0; r < gn[j]; ++r) gm.g[gn[i] + r] = g0[j] + r;
            hipLaunchKernelGGL(k_scatter_tile, dim3((count + 255) / 256), dim3(256), 0, st, tile, kp, nh, gm, ka, out);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

template <typename R>
hipError_t launch_gram(const ColSet& A, const ColSet& B, long N, cx<double>* part, int nchunk, cx<double>* out,
                       hipStream_t st, bool herm) {
    const int ka = A.total(), kb = B.total();
    if (ka < 1 || kb < 1 || ka > kMaxCols || kb > kMaxCols) return hipErrorInvalidValue;
    if (herm && kb != ka && kb != 2 * ka) return hipErrorInvalidValue;
    hipError_t e;
    int chunks;
    // the matrix-core kernel loads 16 bytes per lane: columns must start 16-byte aligned, and in FP32
    // (a row pair per load) have an even length
    bool dma_ok = sizeof(R) == 8 || N % 2 == 0;
    for (int q = 0; q < kMaxSeg; ++q)
        if (B.ncols[q] > 0 && ((size_t)B.ptr[q] & 15)) dma_ok = false;
    if (herm && dma_ok && ka > kMfmaMaxA && ka <= 2 * kMfmaMaxA && (kb == ka || kb == 2 * ka))
        return gram_mfma_tiled<R>(B, ka, kb / ka, N, part, nchunk, out, st);
    if (herm && dma_ok && ka <= kMfmaMaxA) {
        // matrix-core path: at most kMfmaGroups row chunks
        const long groups = std::min<long>(nchunk, mfma_groups(ka));
        const DmaShape d = dma_shape(ka, kb, sizeof(R) == 8);
        const long SR = (long)d.sub * (sizeof(R) == 8 ? 16 : 32);     // rows per stage
        long rpc = (N + groups - 1) / groups;
        rpc = (rpc + SR - 1) / SR * SR;
        chunks = (int)((N + rpc - 1) / rpc);
        e = gram_mfma<R>(B, ka, N, part, chunks, rpc, st);
        if (e != hipSuccess) return e;
        return reduce_chunks(part, chunks, ka * kb, out, st);
    }
    long rpc = (N + nchunk - 1) / nchunk;
    rpc = (rpc + kGramRows - 1) / kGramRows * kGramRows;
    chunks = (int)((N + rpc - 1) / rpc);
    // register tile: every thread of the group waits for the busiest, so the cost of a tile size
    // is (rounds of 256 pair-blocks) x BLK^2; the cheapest, larger BLK on ties (fewer LDS reads per
    // product).  A second round (two pair-blocks per thread) counts 2.5: half the group idles
    // through it and the doubled registers lower the occupancy (measured: the 36-column Hermitian
    // Rayleigh-Ritz product takes 207 us with BLK 3 in one round, 248 us with BLK 2 in two); beyond
    // 2 rounds the pair-blocks go to several work-groups per row chunk, each of which stages the
    // rows again, so those rounds count double
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
    return reduce_chunks(part, chunks, ka * kb, out, st);
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

// Y = S C on the matrix cores for ks <= kCombMaxK inputs and m <= 2 NTO outputs: the real
// product [Re S, Im S] C' in FP64 4x4x4 MFMA with four blocks of four rows each, i.e. 16 rows per
// instruction.  Real outputs are ordered (output column u, real/imaginary part); C' row
// (c, Re) = (Re C[c][u], Im C[c][u]) and row (c, Im) = (-Im C[c][u], Re C[c][u]).  A K step takes
// four input columns: operand lane l (block q = (l >> 2) & 3, row 4 q + (l & 3), k = l >> 4) loads
// the complex entry of column 4 s + k (16 bytes; a wave reads 16 rows of four columns) and feeds
// its real part to one product (K rows (c, Re)) and its imaginary part to a second one (K rows
// (c, Im)).  The B side (C' tiles of 4 K x 4 outputs, the same for the four blocks) is staged in
// LDS once per work-group and read with four lanes on each address.  A wave takes kCombRT row
// tiles at a time, so each C' tile read serves kCombRT products, with NTO accumulators per row
// tile, and the S loads run kCombAhead K steps ahead of the products.
// Result lane l holds row 4 q + (l >> 4)'s output 4 t + (l & 3) of block q.
#ifndef PCX_COMB_RT
#define PCX_COMB_RT 2
#endif
#ifndef PCX_COMB_AHEAD
#define PCX_COMB_AHEAD 2
#endif
constexpr int kCombMaxK = 48;                      // inputs of the one-block-per-SIMD-pair variant
constexpr int kCombMaxK2 = 96;                     // inputs of the large variant (up to 98 KB of LDS)
constexpr int kCombRT = PCX_COMB_RT;               // row tiles per wave and pass
constexpr int kCombAhead = PCX_COMB_AHEAD;         // K steps the S loads run ahead

template <typename R, int NTO, int KMAX>
__global__ void __launch_bounds__(256) k_combine_mfma(ColSet S, const cx<double>* __restrict__ C, int ldc, ColSet Y,
                                                       long N) {
    constexpr int CR = kCombRT, AH = kCombAhead;
    __shared__ double cp[(KMAX / 4) * 2 * NTO * 16];        // C' tiles [K step][Re, Im][output tile][k][j]
    __shared__ const cx<R>* scol[KMAX];
    __shared__ cx<R>* ycol[2 * NTO];
    const int ks = S.total(), m = Y.total();
    const int nks = (ks + 3) / 4;                            // K steps (four complex columns each)
    const int tid = threadIdx.x, lane = tid & 63;
    for (int c = tid; c < ks; c += blockDim.x) scol[c] = col_ptr<const cx<R>>(S, c, N);
    for (int c = tid; c < m; c += blockDim.x) ycol[c] = col_ptr<cx<R>>(Y, c, N);
    for (int e = tid; e < nks * 2 * NTO * 16; e += blockDim.x) {
        const int s = e / (2 * NTO * 16), rem = e % (2 * NTO * 16);
        const int p = rem / (NTO * 16), t = (rem / 16) % NTO, k = (rem / 4) % 4, j = rem % 4;
        const int c = 4 * s + k, o = 4 * t + j, u = o >> 1, pp = o & 1;
        double v = 0.0;
        if (c < ks && u < m) {
            const cx<double> cc = C[(size_t)c * ldc + u];
            v = p == 0 ? (pp == 0 ? cc.x : cc.y) : (pp == 0 ? -cc.y : cc.x);
        }
        cp[e] = v;
    }
    __syncthreads();

    const int q = (lane >> 2) & 3, k = lane >> 4;
    const int wave = tid >> 6, nwave = blockDim.x >> 6;
    const double* cpl = cp + (size_t)(k * 4 + (lane & 3));        // B lane (k, j) of a tile
    const long span = 16L * CR;
    for (long base = ((long)blockIdx.x * nwave + wave) * span; base < N; base += (long)gridDim.x * nwave * span) {
        double acc[CR][NTO];
#pragma unroll
        for (int r = 0; r < CR; ++r)
#pragma unroll
            for (int t = 0; t < NTO; ++t) acc[r][t] = 0.0;
        long row[CR];
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const long rr = base + 16 * r + 4 * q + (lane & 3);
            row[r] = rr < N ? rr : N - 1;                          // tail rows read a valid row
        }
        // the ring of loaded S entries: slot (s mod (AH + 1)); padding columns read column ks - 1
        // (their C' rows are zero)
        cx<R> ring[AH + 1][CR];
        auto load = [&](int s, cx<R>* v) {
            const cx<R>* col = scol[min(4 * s + k, ks - 1)];
#pragma unroll
            for (int r = 0; r < CR; ++r) v[r] = col[row[r]];
        };
#pragma unroll
        for (int a = 0; a < AH; ++a)
            if (a < nks) load(a, ring[a]);
        for (int s0 = 0; s0 < nks; s0 += AH + 1) {
#pragma unroll
            for (int d = 0; d <= AH; ++d) {
                const int s = s0 + d;
                if (s >= nks) break;
                if (s + AH < nks) load(s + AH, ring[(d + AH) % (AH + 1)]);
                const double* cs = cpl + (size_t)s * 2 * NTO * 16;
#pragma unroll
                for (int t = 0; t < NTO; ++t) {
                    const double bre = cs[t * 16], bim = cs[(NTO + t) * 16];
#pragma unroll
                    for (int r = 0; r < CR; ++r) {
                        acc[r][t] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)ring[d][r].x, bre, acc[r][t], 0, 0, 0);
                        acc[r][t] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)ring[d][r].y, bim, acc[r][t], 0, 0, 0);
                    }
                }
            }
        }
        // lane l: row 4 q + (l >> 4) of the tile, real output 4 t + (l & 3)
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const long rr = base + 16 * r + 4 * q + (lane >> 4);
            if (rr >= N) continue;
#pragma unroll
            for (int t = 0; t < NTO; ++t) {
                const int o = 4 * t + (lane & 3), u = o >> 1;
                if (u < m) ((R*)ycol[u])[2 * rr + (o & 1)] = (R)acc[r][t];
            }
        }
    }
}

template <typename R, int NTO>
static hipError_t combine_mfma_impl(const ColSet& S, const cx<double>* C, int ldc, const ColSet& Y, long N,
                                    hipStream_t st) {
    long blocks = (N + 16L * kCombRT * 4 - 1) / (16L * kCombRT * 4);
    if (blocks > 2048) blocks = 2048;
    if (S.total() <= kCombMaxK)
        hipLaunchKernelGGL((k_combine_mfma<R, NTO, kCombMaxK>), dim3((unsigned)blocks), dim3(256), 0, st, S, C, ldc,
                           Y, N);
    else
        hipLaunchKernelGGL((k_combine_mfma<R, NTO, kCombMaxK2>), dim3((unsigned)blocks), dim3(256), 0, st, S, C,
                           ldc, Y, N);
    return hipGetLastError();
}



template <typename R>
static hipError_t combine_mfma_chunk(const ColSet& S, const cx<double>* C, int ldc, const ColSet& Y, long N,
                                     hipStream_t st) {
    switch ((Y.total() + 1) / 2) {
        case 1: return combine_mfma_impl<R, 1>(S, C, ldc, Y, N, st);
        case 2: return combine_mfma_impl<R, 2>(S, C, ldc, Y, N, st);
        case 3: return combine_mfma_impl<R, 3>(S, C, ldc, Y, N, st);
        case 4: return combine_mfma_impl<R, 4>(S, C, ldc, Y, N, st);
        case 5: return combine_mfma_impl<R, 5>(S, C, ldc, Y, N, st);
        case 6: return combine_mfma_impl<R, 6>(S, C, ldc, Y, N, st);
        case 7: return combine_mfma_impl<R, 7>(S, C, ldc, Y, N, st);
        case 8: return combine_mfma_impl<R, 8>(S, C, ldc, Y, N, st);
        case 9: return combine_mfma_impl<R, 9>(S, C, ldc, Y, N, st);
        case 10: return combine_mfma_impl<R, 10>(S, C, ldc, Y, N, st);
        case 11: return combine_mfma_impl<R, 11>(S, C, ldc, Y, N, st);
        case 12: return combine_mfma_impl<R, 12>(S, C, ldc, Y, N, st);
        case 13: return combine_mfma_impl<R, 13>(S, C, ldc, Y, N, st);
        case 14: return combine_mfma_impl<R, 14>(S, C, ldc, Y, N, st);
        case 15: return combine_mfma_impl<R, 15>(S, C, ldc, Y, N, st);
        default: return combine_mfma_impl<R, 16>(S, C, ldc, Y, N, st);
    }
}

// Y = S C for up to kCombMaxK2 inputs: the outputs in chunks of at most 32 columns (each chunk reads
// S again), the coefficient block of a chunk taken in place (row stride m)
template <typename R>
static hipError_t combine_mfma(const ColSet& S, const cx<double>* C, const ColSet& Y, long N, hipStream_t st) {
    const int m = Y.total();
    const int nc = (m + 31) / 32, per = (m + nc - 1) / nc;
    for (int u0 = 0; u0 < m; u0 += per) {
        const int mc = std::min(per, m - u0);
        const hipError_t e = combine_mfma_chunk<R>(S, C + u0, m, col_subset<R>(Y, u0, mc, N), N, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename R>
hipError_t launch_combine(const ColSet& S, const cx<double>* C, const ColSet& Y, long N, hipStream_t st) {
    if (S.total() < 1 || Y.total() < 1 || S.total() > kMaxCols || Y.total() > kMaxCols) return hipErrorInvalidValue;
    if (S.total() <= kCombMaxK2) return combine_mfma<R>(S, C, Y, N, st);
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
__global__ void __launch_bounds__(256) k_residual(ColSet X, ColSet AX, Shifts theta,
                                                   const double* __restrict__ prec, long n, ColSet W,
                                                   long rows_per_chunk, double* __restrict__ part) {
    // grid (chunks, columns): one column of one row chunk per work-group, so the loads of all
    // columns are in flight together rather than one column after another behind a reduction
    __shared__ double red[4];
    const int ka = X.total();
    const int j = blockIdx.y;
    const long N = 2 * n;
    const long r0 = (long)blockIdx.x * rows_per_chunk;
    const long r1 = min(N, r0 + rows_per_chunk);
    const cx<R>* x = col_ptr<const cx<R>>(X, j, N);
    const cx<R>* ax = col_ptr<const cx<R>>(AX, j, N);
    cx<R>* w = col_ptr<cx<R>>(W, j, N);
    const double th = theta.v[j];
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
    if (X.total() > PCX_MAX_BLOCK) return hipErrorInvalidValue;
    Shifts sh;
    for (int j = 0; j < X.total(); ++j) sh.v[j] = theta[j];
    long rpc = (N + nchunk - 1) / nchunk;
    rpc = (rpc + 255) / 256 * 256;
    const int chunks = (int)((N + rpc - 1) / rpc);
    if (X.total() < 1) return hipSuccess;
    hipLaunchKernelGGL((k_residual<R>), dim3(chunks, X.total()), dim3(256), 0, st, X, AX, sh, prec, n, W, rpc, part);
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

template <typename R, int NT, int NH>
static hipError_t set_mfma_lds_one() {
    return hipFuncSetAttribute((const void*)k_gram_mfma<R, NT, NH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024);
}
template <typename R, int... NT>
static hipError_t set_mfma_lds_list(std::integer_sequence<int, NT...>) {
    hipError_t e = hipSuccess;
    ((e = e == hipSuccess ? set_mfma_lds_one<R, NT + 1, 1>() : e), ...);
    ((e = e == hipSuccess ? set_mfma_lds_one<R, NT + 1, 2>() : e), ...);
    return e;
}
template <typename R>
static hipError_t set_mfma_lds() {
    return set_mfma_lds_list<R>(std::make_integer_sequence<int, kMfmaMaxNT>{});
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
    if (e == hipSuccess) e = set_mfma_lds<float>();
    if (e == hipSuccess) e = set_mfma_lds<double>();
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
