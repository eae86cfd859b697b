// The discrete curl C of Section 3 and its adjoint as real-space stencils, for the magnetic-field
// side of the SVD C = P_r Sigma_r Q_r^* (Section 5.1, eq. SVD): the H-field eigenvectors are
// h = P_r y = C Q_r Sigma_r^{-1} y, and the H-field operator C B^{-1} C^* has the same nonzero
// eigenvalues as the GEP (P_r^* C B^{-1} C^* P_r = A_r).
//
// (C_d f)(p) = (f(p + e_d) - f(p)) / delta_d, where a neighbour that leaves the box
// [0, n1) x [0, n2) x [0, n3) is brought back by the lattice vectors (grid units L1 = (n1, 0, 0),
// L2 = (s1, n2, 0), L3 = (s2, s3, n3)) and picks up exp(i 2 pi kappa_l) per L_l taken off (the
// quasi-periodic condition of Section 1.2, eq. quasi_periodic); C = [[0, -C3, C2], [C3, 0, -C1],
// [-C2, C1, 0]] (Section 3).  The adjoint uses the backward neighbour with the inverse reduction:
// (C_d^* g)(p) = (exp(i 2 pi kappa . t) g(q) - g(p)) / delta_d, q = p - e_d reduced into the box
// with t lattice vectors added.  Layout: the e-layout, component l at [l n, (l + 1) n), index
// a + n1 (b + n2 c).  One thread per grid point and vector computes the three output components.
#include "pcx_dev.h"

namespace pcx {

namespace {

struct CurlGrid {
    int n1, n2, n3, s1, s2, s3;
    double kap[3];
    double idl[3];    // 1 / delta_d
};

// brings (a, b, c) into the box: subtracts t3 L3, then t2 L2, then t1 L1 (floor divisions), and
// returns the phase turns kappa . t
DEV double reduce(const CurlGrid& g, int& a, int& b, int& c) {
    double turns = 0.0;
    int t = c >= g.n3 ? 1 : (c < 0 ? -1 : 0);
    if (t) {
        c -= t * g.n3;
        b -= t * g.s3;
        a -= t * g.s2;
        turns += t * g.kap[2];
    }
    t = (b >= 0) ? b / g.n2 : -((-b + g.n2 - 1) / g.n2);
    if (t) {
        b -= t * g.n2;
        a -= t * g.s1;
        turns += t * g.kap[1];
    }
    t = (a >= 0) ? a / g.n1 : -((-a + g.n1 - 1) / g.n1);
    if (t) {
        a -= t * g.n1;
        turns += t * g.kap[0];
    }
    return turns;
}

// f at the neighbour p + sgn e_d of (a, b, c), with its Bloch phase (conjugated for sgn < 0 so that
// the backward difference is the adjoint of the forward one)
template <typename R>
DEV cx<R> neighbour(const CurlGrid& g, const cx<R>* __restrict__ f, int a, int b, int c, int d, int sgn) {
    if (d == 0) a += sgn;
    else if (d == 1) b += sgn;
    else c += sgn;
    const bool inside = a >= 0 && a < g.n1 && b >= 0 && b < g.n2 && c >= 0 && c < g.n3;
    double turns = 0.0;
    if (!inside) turns = reduce(g, a, b, c);
    cx<R> v = f[(long)a + (long)g.n1 * ((long)b + (long)g.n2 * c)];
    if (!inside) {
        // forward neighbour: exp(+i 2 pi kappa . t); backward: the reduction of p - e_d added
        // lattice vectors (t < 0), and the adjoint takes exp(+i 2 pi kappa . t) of that reduction
        const cx<R> ph = cis_turns<R>(turns);
        v = cmul(v, ph);
    }
    return v;
}

template <typename R, bool ADJ>
__global__ void __launch_bounds__(256) k_curl(CurlGrid g, const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                              long nvec) {
    const long n = (long)g.n1 * g.n2 * g.n3;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nvec * n; e += (long)gridDim.x * blockDim.x) {
        const long v = e / n, p = e % n;
        const int a = (int)(p % g.n1), b = (int)((p / g.n1) % g.n2), c = (int)(p / ((long)g.n1 * g.n2));
        const cx<R>* f = in + v * 3 * n;
        // D[l][d] = (C_d f_l)(p) or (C_d^* f_l)(p) for the (l, d) pairs the curl needs
        auto D = [&](int l, int d) {
            const cx<R>* fl = f + (long)l * n;
            const cx<R> x = neighbour<R>(g, fl, a, b, c, d, ADJ ? -1 : +1);
            const cx<R> diff = x - fl[p];
            return cscale(diff, (R)g.idl[d]);
        };
        cx<R> o0, o1, o2;
        if (!ADJ) {
            // C = [[0, -C3, C2], [C3, 0, -C1], [-C2, C1, 0]]
            o0 = D(2, 1) - D(1, 2);
            o1 = D(0, 2) - D(2, 0);
            o2 = D(1, 0) - D(0, 1);
        } else {
            // C^* = [[0, C3^*, -C2^*], [-C3^*, 0, C1^*], [C2^*, -C1^*, 0]]
            o0 = D(1, 2) - D(2, 1);
            o1 = D(2, 0) - D(0, 2);
            o2 = D(0, 1) - D(1, 0);
        }
        cx<R>* ov = out + v * 3 * n;
        ov[p] = o0;
        ov[n + p] = o1;
        ov[2 * n + p] = o2;
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_scale3(const R* __restrict__ s, cx<R>* __restrict__ x, long n3, long nvec) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < nvec * n3; e += (long)gridDim.x * blockDim.x)
        x[e] = cscale(x[e], s[e % n3]);
}

unsigned blocks_for(long work) {
    long b = (work + 255) / 256;
    if (b > 16384) b = 16384;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

template <typename R>
hipError_t launch_curl(const Grid& gg, const cx<R>* in, cx<R>* out, int nvec, bool adjoint, hipStream_t st) {
    CurlGrid g;
    g.n1 = gg.n1; g.n2 = gg.n2; g.n3 = gg.n3;
    g.s1 = gg.s1; g.s2 = gg.s2; g.s3 = gg.s3;
    for (int l = 0; l < 3; ++l) {
        g.kap[l] = gg.kap[l];
        g.idl[l] = 1.0 / gg.dlt[l];
    }
    const long work = (long)nvec * gg.n1 * gg.n2 * gg.n3;
    if (adjoint)
        hipLaunchKernelGGL((k_curl<R, true>), dim3(blocks_for(work)), dim3(256), 0, st, g, in, out, (long)nvec);
    else
        hipLaunchKernelGGL((k_curl<R, false>), dim3(blocks_for(work)), dim3(256), 0, st, g, in, out, (long)nvec);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_scale3(const R* s, cx<R>* x, long n3, int nvec, hipStream_t st) {
    hipLaunchKernelGGL((k_scale3<R>), dim3(blocks_for(n3 * nvec)), dim3(256), 0, st, s, x, n3, (long)nvec);
    return hipGetLastError();
}

template hipError_t launch_curl<float>(const Grid&, const cx<float>*, cx<float>*, int, bool, hipStream_t);
template hipError_t launch_curl<double>(const Grid&, const cx<double>*, cx<double>*, int, bool, hipStream_t);
template hipError_t launch_scale3<float>(const float*, cx<float>*, long, int, hipStream_t);
template hipError_t launch_scale3<double>(const double*, cx<double>*, long, int, hipStream_t);

}  // namespace pcx
