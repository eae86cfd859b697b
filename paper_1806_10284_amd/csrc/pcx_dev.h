// Device-side helpers shared by the matvec kernels: complex arithmetic, radix butterflies, the
// curl symbols Lambda_d (Section 4.2) and the mixing matrix W of Section 5.1.
#pragma once

#include "pcx_internal.h"

namespace pcx {

#define DEV __device__ __forceinline__

// ------------------------------------------------------------------ complex helpers
template <typename R>
DEV cx<R> mk(R a, R b) {
    cx<R> z;
    z.x = a;
    z.y = b;
    return z;
}
template <typename R>
DEV cx<R> operator+(cx<R> a, cx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R>
DEV cx<R> operator-(cx<R> a, cx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R>
DEV cx<R> cmul(cx<R> a, cx<R> b) { return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <typename R>
DEV cx<R> cmulc(cx<R> a, cx<R> b) { return mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }  // a * conj(b)
template <typename R>
DEV cx<R> cscale(cx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }
template <typename R>
DEV cx<R> times_i(cx<R> a, int sign) { return sign > 0 ? mk<R>(-a.y, a.x) : mk<R>(a.y, -a.x); }  // sign*i*a
template <typename R>
DEV cx<R> conjc(cx<R> a) { return mk<R>(a.x, -a.y); }

template <typename R, typename S>
DEV cx<R> cvt(cx<S> a) { return mk<R>((R)a.x, (R)a.y); }

DEV void sincospi_r(double x, double* s, double* c) { sincospi(x, s, c); }
DEV void sincospi_r(float x, float* s, float* c) { sincospif(x, s, c); }

// exp(2 pi i * turns) with the turn reduced in FP64 first
template <typename R>
DEV cx<R> cis_turns(double turns) {
    double r = turns - rint(turns);
    R s, c;
    sincospi_r((R)(2.0 * r), &s, &c);
    return mk<R>(c, s);
}

// ------------------------------------------------------------------ radix butterflies
// y_q = sum_r x_r exp(sign 2 pi i r q / RAD)
template <typename R, int RAD>
struct Bfly;

template <typename R>
struct Bfly<R, 2> {
    static DEV void run(cx<R>* v, int) {
        cx<R> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <typename R>
struct Bfly<R, 4> {
    static DEV void run(cx<R>* v, int s) {
        cx<R> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = times_i(v[1] - v[3], s);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + d;
        v[3] = b - d;
    }
};

template <typename R>
struct Bfly<R, 3> {
    static DEV void run(cx<R>* v, int s) {
        const R c1 = (R)-0.5;
        const R s1 = (R)0.86602540378443864676;
        cx<R> t = v[1] + v[2];
        cx<R> d = times_i(v[1] - v[2], s);
        cx<R> m = v[0] + cscale(t, c1);
        v[0] = v[0] + t;
        v[1] = m + cscale(d, s1);
        v[2] = m - cscale(d, s1);
    }
};

template <typename R>
struct Bfly<R, 5> {
    static DEV void run(cx<R>* v, int s) {
        const R c1 = (R)0.30901699437494742410;   // cos(2 pi / 5)
        const R c2 = (R)-0.80901699437494742410;  // cos(4 pi / 5)
        const R s1 = (R)0.95105651629515357212;   // sin(2 pi / 5)
        const R s2 = (R)0.58778525229247312917;   // sin(4 pi / 5)
        cx<R> t1 = v[1] + v[4], t2 = v[2] + v[3];
        cx<R> d1 = times_i(v[1] - v[4], s), d2 = times_i(v[2] - v[3], s);
        cx<R> a = v[0] + cscale(t1, c1) + cscale(t2, c2);
        cx<R> b = v[0] + cscale(t1, c2) + cscale(t2, c1);
        cx<R> p = cscale(d1, s1) + cscale(d2, s2);
        cx<R> q = cscale(d1, s2) - cscale(d2, s1);
        v[0] = v[0] + t1 + t2;
        v[1] = a + p;
        v[4] = a - p;
        v[2] = b + q;
        v[3] = b - q;
    }
};

template <typename R>
struct Bfly<R, 8> {
    static DEV void run(cx<R>* v, int s) {
        const R h = (R)0.70710678118654752440;
        cx<R> e[4] = {v[0], v[2], v[4], v[6]};
        cx<R> o[4] = {v[1], v[3], v[5], v[7]};
        Bfly<R, 4>::run(e, s);
        Bfly<R, 4>::run(o, s);
        // o_q *= exp(s 2 pi i q / 8)
        cx<R> o1 = cscale(o[1] + times_i(o[1], s), h);
        cx<R> o2 = times_i(o[2], s);
        cx<R> o3 = cscale(times_i(o[3], s) - o[3], h);
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + o1;
        v[5] = e[1] - o1;
        v[2] = e[2] + o2;
        v[6] = e[2] - o2;
        v[3] = e[3] + o3;
        v[7] = e[3] - o3;
    }
};

// ------------------------------------------------------------------ per-mode symbols (FP64)
// exp(i 2 pi t) - 1 = 2 s (-s + i c) with (s, c) = (sin, cos)(pi t)
DEV cx<double> lam_from_halfturn(double s, double c, double inv_delta) {
    return mk<double>(-2.0 * s * s * inv_delta, 2.0 * s * c * inv_delta);
}
DEV cx<double> lam_of_turn(double t, double inv_delta) {
    double r = t - rint(t);
    double s, c;
    sincospi(r, &s, &c);
    return lam_from_halfturn(s, c, inv_delta);
}

DEV double abs2(cx<double> a) { return a.x * a.x + a.y * a.y; }

// Basis choice per mode (Section 5.1 reading): 0 = the paper's basis (reference vector 1),
// 1..3 = fallback reference vector e_{code-1}, kMasked = no range space (Gamma mode).
constexpr unsigned char kMasked = 255;

DEV unsigned char mix_code(cx<double> L0, cx<double> L1, cx<double> L2) {
    const double a0 = abs2(L0), a1 = abs2(L1), a2 = abs2(L2);
    const double Lq = a0 + a1 + a2;
    const double Lp2 = abs2(L0 - L1) + abs2(L0 - L2) + abs2(L1 - L2);
    if (Lp2 >= kMixTau * Lq) return 0;
    const double mn = fmin(a0, fmin(a1, a2)) * (1.0 + 1e-8);
    return (unsigned char)(1 + ((a0 <= mn) ? 0 : ((a1 <= mn) ? 1 : 2)));
}

DEV double rsqrt_r(double x) { return 1.0 / sqrt(x); }
DEV float rsqrt_r(float x) { return rsqrtf(x); }
DEV double sqrt_r(double x) { return sqrt(x); }
DEV float sqrt_r(float x) { return sqrtf(x); }

// Row l of W in precision R for the basis `code` (not kMasked), from FP64 symbols:
//   code 0: W[:,0] = (Lq 1 - Lambda conj(Ls)) / Lp, W[:,1] = sqrt(Lq) (1 x conj Lambda) / Lp,
//           evaluated without cancellation as W[l,0] = sum_{m != l} conj(L_m)(L_m - L_l) / Lp and
//           W[:,1] = sqrt(Lq) conj(L2 - L1, L0 - L2, L1 - L0) / Lp, Lp^2 = sum |L_a - L_b|^2,
//           the differences taken in FP64;
//   code 1+m: the same with 1 replaced by e_m: W[l,0] = (delta_lm Lq - L_l conj(L_m)) / d,
//           W[:,1] = sqrt(Lq) (e_m x conj Lambda) / d, d^2 = Lq - |L_m|^2 = sum_{l != m} |L_l|^2.
template <typename R>
DEV void w_row_code(cx<double> L0, cx<double> L1, cx<double> L2, int code, int l, cx<R>* w1, cx<R>* w2) {
    const double a0 = abs2(L0), a1 = abs2(L1), a2 = abs2(L2);
    const R sq = sqrt_r((R)(a0 + a1 + a2));
    const cx<R> zero = mk<R>((R)0, (R)0);
    if (code == 0) {
        const cx<double> D10 = L1 - L0, D20 = L2 - L0, D21 = L2 - L1;
        const R inv = rsqrt_r((R)(abs2(D10) + abs2(D20) + abs2(D21)));
        const cx<R> d10 = cvt<R>(D10), d20 = cvt<R>(D20), d21 = cvt<R>(D21);
        cx<R> c1, c2;
        if (l == 0) {
            c1 = cmul(conjc(cvt<R>(L1)), d10) + cmul(conjc(cvt<R>(L2)), d20);
            c2 = conjc(d21);
        } else if (l == 1) {
            c1 = cmul(conjc(cvt<R>(L2)), d21) - cmul(conjc(cvt<R>(L0)), d10);
            c2 = zero - conjc(d20);
        } else {
            c1 = zero - cmul(conjc(cvt<R>(L0)), d20) - cmul(conjc(cvt<R>(L1)), d21);
            c2 = conjc(d10);
        }
        *w1 = cscale(c1, inv);
        *w2 = cscale(c2, sq * inv);
    } else {
        const int m = code - 1;
        const double d2 = (m == 0) ? a1 + a2 : (m == 1 ? a0 + a2 : a0 + a1);
        const R inv = rsqrt_r((R)d2);
        const cx<R> Ll = cvt<R>((l == 0) ? L0 : (l == 1 ? L1 : L2));
        const cx<R> Lm = cvt<R>((m == 0) ? L0 : (m == 1 ? L1 : L2));
        const cx<R> v0 = conjc(cvt<R>(L0)), v1 = conjc(cvt<R>(L1)), v2 = conjc(cvt<R>(L2));
        cx<R> cr;
        if (m == 0) cr = (l == 0) ? zero : (l == 1 ? zero - v2 : v1);
        else if (m == 1) cr = (l == 0) ? v2 : (l == 1 ? zero : zero - v0);
        else cr = (l == 0) ? zero - v1 : (l == 1 ? v0 : zero);
        *w1 = cscale(l == m ? mk<R>((R)d2, (R)0) : zero - cmulc(Ll, Lm), inv);
        *w2 = cscale(cr, sq * inv);
    }
}

// The wave vector of this work-group: the grid's own, or in a multi-k launch (blockIdx.y =
// k * nvk + v) the k-th kappa and its n-byte block of mode codes.
struct KSel {
    double kap[3];
    const unsigned char* codes;
};

DEV KSel select_k(const Grid& g, long n) {
    KSel s;
    if (g.nvk > 0) {
        const int kk = (int)blockIdx.y / g.nvk;
        s.kap[0] = g.kaps[3 * kk];
        s.kap[1] = g.kaps[3 * kk + 1];
        s.kap[2] = g.kaps[3 * kk + 2];
        s.codes = g.codes + (long)kk * n;
    } else {
        s.kap[0] = g.kap[0];
        s.kap[1] = g.kap[1];
        s.kap[2] = g.kap[2];
        s.codes = g.codes;
    }
    return s;
}

}  // namespace pcx
