// Small dense Hermitian linear algebra for the Rayleigh-Ritz step (host, FP64, row-major).
//
// herm_eig: Householder reduction of a Hermitian matrix to a real symmetric tridiagonal one
// (a unitary similarity followed by a diagonal phase), then the implicit QL iteration with
// Wilkinson shifts (the classical tridiagonal QL algorithm) accumulating the eigenvectors.
#include "pcx_dense.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace pcx {

void hermitize(int k, std::vector<zc>& A) {
    for (int i = 0; i < k; ++i) {
        A[(size_t)i * k + i] = zc(A[(size_t)i * k + i].real(), 0.0);
        for (int j = i + 1; j < k; ++j) {
            const zc a = 0.5 * (A[(size_t)i * k + j] + std::conj(A[(size_t)j * k + i]));
            A[(size_t)i * k + j] = a;
            A[(size_t)j * k + i] = std::conj(a);
        }
    }
}

// complex products in plain real arithmetic (no special-value handling: every entry here is finite)
static inline zc cmul(zc a, zc b) {
    return zc(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}
static inline zc cjmul(zc a, zc b) {   // conj(a) * b
    return zc(a.real() * b.real() + a.imag() * b.imag(), a.real() * b.imag() - a.imag() * b.real());
}
static inline zc mulcj(zc a, zc b) {   // a * conj(b)
    return zc(a.real() * b.real() + a.imag() * b.imag(), a.imag() * b.real() - a.real() * b.imag());
}

// sqrt(a^2 + b^2), scaled only where the squares could leave the double range
static inline double pyth(double a, double b) {
    const double m = std::max(std::fabs(a), std::fabs(b));
    if (m > 1e-150 && m < 1e150) return std::sqrt(a * a + b * b);
    return std::hypot(a, b);
}

// one plane rotation of the QL iteration: columns i and i + 1 of the eigenvector matrix Z become
// (c z_i - s z_{i+1}, s z_i + c z_{i+1})
struct Rot {
    double c, s;
    int i;
};

// implicit QL on the symmetric tridiagonal (d diagonal, e[i] = T(i+1, i)); the eigenvector matrix
// is the product of the recorded rotations (applied later to the wanted columns only)
static bool tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e, std::vector<Rot>& rots) {
    rots.clear();
    if (n == 0) return true;
    e.resize(n);
    e[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            if (++iter > 200) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = pyth(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = pyth(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                rots.push_back({c, s, i});
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

bool herm_eig(int k, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V, int ncols) {
    if (ncols < 0 || ncols > k) ncols = k;
    hermitize(k, A);
    // Householder reduction A = Q T Q^H, Q = H_0 H_1 ... with H_j = I - 2 v_j v_j^H acting on the
    // indices above j; each step updates only the trailing block A[j+1:, j+1:]
    std::vector<zc> R((size_t)k * k, zc(0, 0));   // row j: v_j (zero below index j + 1)
    std::vector<char> has(k, 0);
    std::vector<zc> p(k), q(k);
    for (int j = 0; j + 2 < k; ++j) {
        zc* aj = &A[(size_t)j * k];                 // row j holds conj of column j
        double xn2 = 0.0;
        for (int i = j + 1; i < k; ++i) xn2 += std::norm(aj[i]);
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const zc x0 = std::conj(aj[j + 1]);          // A[j+1][j]
        const double ax0 = std::abs(x0);
        const zc ph = ax0 > 0 ? x0 / ax0 : zc(1, 0);
        const zc alpha = -ph * xn;                   // reflect x = A[j+1:, j] onto alpha e_1
        zc* v = &R[(size_t)j * k];
        for (int i = j + 1; i < k; ++i) v[i] = std::conj(aj[i]);
        v[j + 1] -= alpha;
        double vn2 = 0.0;
        for (int i = j + 1; i < k; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double vi = 1.0 / std::sqrt(vn2);
        for (int i = j + 1; i < k; ++i) v[i] *= vi;
        has[j] = 1;
        // H A22 H = A22 - 2 (v q^H + q v^H), p = A22 v, K = v^H p (real), q = p - K v
        for (int i = j + 1; i < k; ++i) {
            const zc* ai = &A[(size_t)i * k];
            double sr = 0.0, si = 0.0;
            for (int c = j + 1; c < k; ++c) {
                sr += ai[c].real() * v[c].real() - ai[c].imag() * v[c].imag();
                si += ai[c].real() * v[c].imag() + ai[c].imag() * v[c].real();
            }
            p[i] = zc(sr, si);
        }
        double K = 0.0;
        for (int i = j + 1; i < k; ++i) K += cjmul(v[i], p[i]).real();
        for (int i = j + 1; i < k; ++i) q[i] = p[i] - K * v[i];
        for (int i = j + 1; i < k; ++i) {
            zc* ai = &A[(size_t)i * k];
            const zc vi2 = 2.0 * v[i], qi2 = 2.0 * q[i];
            for (int c = j + 1; c < k; ++c) ai[c] -= mulcj(vi2, q[c]) + mulcj(qi2, v[c]);
        }
        // the reduced column and row: alpha e_1
        A[(size_t)(j + 1) * k + j] = alpha;
        aj[j + 1] = std::conj(alpha);
    }
    // phases that make the sub-diagonal real and non-negative
    std::vector<zc> dph(k, zc(1, 0));
    std::vector<double> d(k), e(std::max(k, 1), 0.0);
    for (int i = 0; i < k; ++i) d[i] = A[(size_t)i * k + i].real();
    for (int i = 0; i + 1 < k; ++i) {
        const zc s = A[(size_t)(i + 1) * k + i];
        const double as = std::abs(s);
        e[i] = as;
        dph[i + 1] = as > 0 ? dph[i] * s / as : dph[i];
    }
    std::vector<Rot> rots;
    rots.reserve((size_t)4 * k * k);
    if (!tridiag_ql(k, d, e, rots)) return false;
    std::vector<int> idx(k);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    w.resize(k);
    for (int c = 0; c < k; ++c) w[c] = d[idx[c]];
    // Z = G_1 G_2 ... G_N, so Z[:, wanted] = G_1 (G_2 (... (G_N E))) with E the unit columns:
    // the rotations in reverse order on a k x ncols block (row m: entries of row m of Z)
    std::vector<double> Zw((size_t)k * ncols, 0.0);
    for (int c = 0; c < ncols; ++c) Zw[(size_t)idx[c] * ncols + c] = 1.0;
    for (size_t t = rots.size(); t-- > 0;) {
        const Rot& g = rots[t];
        double* zi = &Zw[(size_t)g.i * ncols];
        double* zj = zi + ncols;
        for (int c = 0; c < ncols; ++c) {
            const double a0 = zi[c], a1 = zj[c];
            zi[c] = g.c * a0 + g.s * a1;
            zj[c] = g.c * a1 - g.s * a0;
        }
    }
    // eigenvector c = Q diag(dph) Z[:, idx[c]]: the phases, then H_{k-3}, ..., H_0 in turn
    std::vector<zc> X((size_t)ncols * k);           // row c: eigenvector c
    for (int c = 0; c < ncols; ++c) {
        zc* x = &X[(size_t)c * k];
        for (int m = 0; m < k; ++m) x[m] = dph[m] * Zw[(size_t)m * ncols + c];
    }
    for (int j = k - 3; j >= 0; --j) {
        if (!has[j]) continue;
        const zc* v = &R[(size_t)j * k];
        for (int c = 0; c < ncols; ++c) {
            zc* x = &X[(size_t)c * k];
            double sr = 0.0, si = 0.0;
            for (int i = j + 1; i < k; ++i) {
                sr += v[i].real() * x[i].real() + v[i].imag() * x[i].imag();
                si += v[i].real() * x[i].imag() - v[i].imag() * x[i].real();
            }
            const zc s2(2.0 * sr, 2.0 * si);
            for (int i = j + 1; i < k; ++i) x[i] -= cmul(s2, v[i]);
        }
    }
    V.assign((size_t)k * ncols, zc(0, 0));
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < ncols; ++c) V[(size_t)i * ncols + c] = X[(size_t)c * k + i];
    return true;
}

bool cholesky(int k, const std::vector<zc>& G, std::vector<zc>& L, double rel_tol) {
    L.assign((size_t)k * k, zc(0, 0));
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) dmax = std::max(dmax, G[(size_t)i * k + i].real());
    if (!(dmax > 0.0)) return false;
    for (int j = 0; j < k; ++j) {
        double dj = G[(size_t)j * k + j].real();
        for (int m = 0; m < j; ++m) dj -= std::norm(L[(size_t)j * k + m]);
        if (!(dj > rel_tol * dmax)) return false;
        const double ljj = std::sqrt(dj);
        L[(size_t)j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            zc s = G[(size_t)i * k + j];
            for (int m = 0; m < j; ++m) s -= mulcj(L[(size_t)i * k + m], L[(size_t)j * k + m]);
            L[(size_t)i * k + j] = s / ljj;
        }
    }
    return true;
}

void solve_LH(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int i = k - 1; i >= 0; --i) {
        zc* xi = &X[(size_t)i * m];
        for (int j = i + 1; j < k; ++j) {
            const zc l = L[(size_t)j * k + i];
            const zc* xj = &X[(size_t)j * m];
            for (int c = 0; c < m; ++c) xi[c] -= cjmul(l, xj[c]);
        }
        const double inv = L[(size_t)i * k + i].real();
        for (int c = 0; c < m; ++c) xi[c] /= inv;
    }
}

void solve_L(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int i = 0; i < k; ++i) {
        zc* xi = &X[(size_t)i * m];
        for (int j = 0; j < i; ++j) {
            const zc l = L[(size_t)i * k + j];
            const zc* xj = &X[(size_t)j * m];
            for (int c = 0; c < m; ++c) xi[c] -= cmul(l, xj[c]);
        }
        const double inv = L[(size_t)i * k + i].real();
        for (int c = 0; c < m; ++c) xi[c] /= inv;
    }
}

bool rayleigh_ritz(int k, std::vector<zc> GA, std::vector<zc> GB, int want, double chol_tol,
                   std::vector<double>& theta, std::vector<zc>& C) {
    hermitize(k, GA);
    hermitize(k, GB);
    // scale the basis columns to unit norm so the Cholesky tolerance measures linear dependence
    std::vector<double> sc(k);
    for (int i = 0; i < k; ++i) {
        const double dii = GB[(size_t)i * k + i].real();
        if (!(dii > 0.0)) return false;
        sc[i] = 1.0 / std::sqrt(dii);
    }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            GA[(size_t)i * k + j] *= sc[i] * sc[j];
            GB[(size_t)i * k + j] *= sc[i] * sc[j];
        }
    std::vector<zc> L;
    if (!cholesky(k, GB, L, chol_tol)) return false;
    std::vector<zc> Y, H;
    solve_L(k, L, GA, k, Y);                    // Y = L^{-1} GA
    std::vector<zc> Yh((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Yh[(size_t)i * k + j] = std::conj(Y[(size_t)j * k + i]);
    solve_L(k, L, Yh, k, H);                    // H = L^{-1} Y^H = L^{-1} GA L^{-H}
    std::vector<double> w;
    std::vector<zc> V;
    if (!herm_eig(k, H, w, V, want)) return false;
    solve_LH(k, L, V, want, C);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < want; ++c) C[(size_t)i * want + c] *= sc[i];
    theta.assign(w.begin(), w.begin() + want);
    return true;
}

// C with Y C orthonormal for the Gram matrix G = Y^H Y (Cholesky QR on unit-scaled columns,
// eigenvalue-based fallback when the columns are nearly dependent)
void orthonormalizer(int m, std::vector<zc> G, std::vector<zc>& C) {
    hermitize(m, G);
    std::vector<double> sc(m);
    for (int i = 0; i < m; ++i) {
        const double dii = G[(size_t)i * m + i].real();
        sc[i] = dii > 0 ? 1.0 / std::sqrt(dii) : 0.0;
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) G[(size_t)i * m + j] *= sc[i] * sc[j];
    std::vector<zc> L, I((size_t)m * m, zc(0, 0));
    for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
    if (cholesky(m, G, L, 1e-14)) {
        solve_LH(m, L, I, m, C);
    } else {
        std::vector<double> w;
        std::vector<zc> V;
        herm_eig(m, G, w, V);
        const double wmax = std::max(w.empty() ? 1.0 : w.back(), 1e-300);
        C.assign((size_t)m * m, zc(0, 0));
        for (int c = 0; c < m; ++c) {
            const double dc = 1.0 / std::sqrt(std::max(w[c], 1e-14 * wmax));
            for (int r = 0; r < m; ++r) C[(size_t)r * m + c] = V[(size_t)r * m + c] * dc;
        }
    }
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < m; ++c) C[(size_t)i * m + c] *= sc[i];
}

}  // namespace pcx

// Host-only self-test hooks for the dense routines (interleaved complex, row-major).
static std::vector<pcx::zc> load_cx(int n, const double* a) {
    std::vector<pcx::zc> A((size_t)n);
    for (int i = 0; i < n; ++i) A[i] = pcx::zc(a[2 * i], a[2 * i + 1]);
    return A;
}

static void store_cx(const std::vector<pcx::zc>& A, double* a) {
    for (size_t i = 0; i < A.size(); ++i) {
        a[2 * i] = A[i].real();
        a[2 * i + 1] = A[i].imag();
    }
}

// all k eigenvalues; v: k x ncols eigenvectors of the lowest ncols
extern "C" int pcxd_herm_eig_cols(int k, const double* a, int ncols, double* w, double* v) {
    std::vector<double> ww;
    std::vector<pcx::zc> V;
    if (!pcx::herm_eig(k, load_cx(k * k, a), ww, V, ncols)) return -1;
    for (int i = 0; i < k; ++i) w[i] = ww[i];
    store_cx(V, v);
    return 0;
}

extern "C" int pcxd_herm_eig(int k, const double* a, double* w, double* v) {
    return pcxd_herm_eig_cols(k, a, k, w, v);
}

// lowest `want` pairs of the pencil (ga, gb); c: k x want
extern "C" int pcxd_rayleigh_ritz(int k, const double* ga, const double* gb, int want, double* theta, double* c) {
    std::vector<double> th;
    std::vector<pcx::zc> C;
    if (!pcx::rayleigh_ritz(k, load_cx(k * k, ga), load_cx(k * k, gb), want, 1e-14, th, C)) return -1;
    for (int i = 0; i < want; ++i) theta[i] = th[i];
    store_cx(C, c);
    return 0;
}
