// Per-plane tables and the per-mode mixing W of the fixed-size plane kernels (Section 5.1 and the
// twiddles of Algorithms 5.1 / 5.2), shared by the LDS-staged and the register-resident kernels.
// LT: any layout with the LDS arrays twz, twy, twb, twc (precision R) and halfz, rowz, lamy, d10
// (complex FP64), a01, p10 (FP64) of the plane.
#pragma once

#include "pcx_dev.h"

namespace pcx {

// Fills the per-plane tables of plane i; returns Lambda_1(i).
template <typename R, int N2, int N3, int NT, typename LT>
DEV cx<double> p3_setup(const Grid& g, const KSel& ks, const DeviceTables& tb, int i, const LT& L) {
    const double tx = (ks.kap[0] + (double)i) / (double)g.n1;
    const cx<double> L0 = lam_of_turn(tx, 1.0 / g.dlt[0]);
    const cx<R>* twz_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[2] : (const cx<R>*)tb.tw32[2];
    const cx<R>* twy_g = sizeof(R) == 8 ? (const cx<R>*)tb.tw64[1] : (const cx<R>*)tb.tw32[1];
    const double phi2 = (ks.kap[1] - (double)g.s1 * tx) / (double)N2;
    const double Ai =
        ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ((ks.kap[1] - (double)g.s1 * tx) / (double)N2)) / (double)N3;
    // three independent groups of entries, each on its own wavefront when the work-group has three
    // (their FP64 sines and cosines then run side by side instead of one after another)
    constexpr bool kSpread = NT >= 192;
    const int grp = kSpread ? (int)threadIdx.x >> 6 : 0;
    const int t0 = kSpread ? (int)threadIdx.x & 63 : (int)threadIdx.x;
    constexpr int kStep = kSpread ? 64 : NT;
    if (grp == 0) {
        for (int q = t0; q < N3; q += kStep) {
            L.twz[q] = twz_g[q];
            L.halfz[q] = tb.halfz[q];
            L.twc[q] = cis_turns<R>((double)q * Ai);
        }
    }
    if (grp == (kSpread ? 1 : 0)) {
        for (int j = t0; j < N2; j += kStep) {
            L.twy[j] = twy_g[j];
            L.twb[j] = cis_turns<R>((double)j * phi2);
        }
    }
    if (grp == (kSpread ? 2 : 0)) {
        for (int j = t0; j < N2; j += kStep) {
            const double ty = ((ks.kap[1] + (double)j) - (double)g.s1 * tx) / (double)N2;
            const cx<double> L1 = lam_of_turn(ty, 1.0 / g.dlt[1]);
            const cx<double> D = L1 - L0;
            L.lamy[j] = L1;
            L.d10[j] = D;
            L.a01[j] = abs2(L0) + abs2(L1);
            L.p10[j] = abs2(D);
            const double p3 = ((ks.kap[2] - (double)g.s2 * tx) - (double)g.s3 * ty) / (double)N3;
            double s, c;
            sincospi(p3, &s, &c);
            L.rowz[j] = mk<double>(c, s);
        }
    }
    return L0;
}

// W (3 x 2) of mode (j, k) in precision R.  Code 0 (the paper's basis) from the per-row tables:
//   W[l,0] = sum_{m != l} conj(L_m)(L_m - L_l) / Lp,  W[:,1] = sqrt(Lq) conj(L2 - L1, L0 - L2, L1 - L0) / Lp
// with the differences and the sums Lq, Lp^2 in FP64; other codes through w_row_code.
template <typename R, int N2, int N3, typename LT>
DEV void p3_w(const LT& L, cx<double> L0, int j, int k, int code, double idz, cx<R> w[3][2]) {
    const cx<double> h = cmul(L.halfz[k], L.rowz[j]);
    const cx<double> L2 = lam_from_halfturn(h.y, h.x, idz);
    const cx<double> L1 = L.lamy[j];
    if (code == 0) {
        const cx<double> D10 = L.d10[j];
        const cx<double> D20 = L2 - L0, D21 = L2 - L1;
        const double lq = L.a01[j] + abs2(L2);
        const double lp2 = L.p10[j] + abs2(D20) + abs2(D21);
        const R inv = rsqrt_r((R)lp2);
        const R sc = sqrt_r((R)lq) * inv;
        const cx<R> c0 = conjc(cvt<R>(L0)), c1 = conjc(cvt<R>(L1)), c2 = conjc(cvt<R>(L2));
        const cx<R> d10 = cvt<R>(D10), d20 = cvt<R>(D20), d21 = cvt<R>(D21);
        w[0][0] = cscale(cmul(c1, d10) + cmul(c2, d20), inv);
        w[1][0] = cscale(cmul(c2, d21) - cmul(c0, d10), inv);
        w[2][0] = cscale(mk<R>((R)0, (R)0) - cmul(c0, d20) - cmul(c1, d21), inv);
        w[0][1] = cscale(conjc(d21), sc);
        w[1][1] = cscale(mk<R>((R)0, (R)0) - conjc(d20), sc);
        w[2][1] = cscale(conjc(d10), sc);
    } else {
#pragma unroll
        for (int l = 0; l < 3; ++l) w_row_code<R>(L0, L1, L2, code, l, &w[l][0], &w[l][1]);
    }
}

// exp(2 pi i c phi3(i, j)) = twc[c] * exp(-2 pi i ((c j s3) mod N2 N3) / (N2 N3)), rot = the table of
// (N2 N3)-th roots, s3m = s3 mod N2 N3 in [0, N2 N3)
template <typename R, int N2, int N3, typename LT>
DEV cx<R> p3_ztw(const LT& L, const cx<R>* __restrict__ rot, int c, int j, int s3m) {
    constexpr int M = N2 * N3;
    return cmul(L.twc[c], rot[(c * j * s3m) % M]);
}

// W of mode e of plane i: from the grid's table (layout [2l + c][n], zero on the masked mode) when
// there is one, else formed here (zero on the masked mode).
template <typename R, int N2, int N3, bool WT, typename LT>
DEV void mode_w(const cx<R>* __restrict__ wt, long n, long m, const LT& L, cx<double> L0, int j, int k, int code,
                double idz, cx<R> w[3][2]) {
    if constexpr (WT) {
#pragma unroll
        for (int q = 0; q < 6; ++q) w[q >> 1][q & 1] = wt[(long)q * n + m];
        return;
    }
    if (code == kMasked) {
#pragma unroll
        for (int q = 0; q < 6; ++q) w[q >> 1][q & 1] = mk<R>((R)0, (R)0);
        return;
    }
    p3_w<R, N2, N3>(L, L0, j, k, code, idz, w);
}

}  // namespace pcx
