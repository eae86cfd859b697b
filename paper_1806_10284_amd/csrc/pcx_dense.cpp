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

// implicit QL on the symmetric tridiagonal (d diagonal, e[i] = T(i+1, i)), rotating the columns of Z
static bool tridiag_ql(int n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z) {
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
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            bool deflated = false;
            for (; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
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
                for (int q = 0; q < n; ++q) {
                    f = Z[(size_t)q * n + i + 1];
                    Z[(size_t)q * n + i + 1] = s * Z[(size_t)q * n + i] + c * f;
                    Z[(size_t)q * n + i] = c * Z[(size_t)q * n + i] - s * f;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

bool herm_eig(int k, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V) {
    hermitize(k, A);
    // Q accumulates the Householder reflections: A = Q T Q^H
    std::vector<zc> Q((size_t)k * k, zc(0, 0));
    for (int i = 0; i < k; ++i) Q[(size_t)i * k + i] = 1.0;
    std::vector<zc> v(k), p(k), q(k);
    for (int j = 0; j + 2 < k; ++j) {
        // x = A[j+1:, j]
        double xn2 = 0.0;
        for (int i = j + 1; i < k; ++i) xn2 += std::norm(A[(size_t)i * k + j]);
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const zc x0 = A[(size_t)(j + 1) * k + j];
        const double ax0 = std::abs(x0);
        const zc ph = ax0 > 0 ? x0 / ax0 : zc(1, 0);
        const zc alpha = -ph * xn;                 // reflect x onto alpha e_1
        // v = x - alpha e1, normalised
        for (int i = 0; i < k; ++i) v[i] = 0.0;
        for (int i = j + 1; i < k; ++i) v[i] = A[(size_t)i * k + j];
        v[j + 1] -= alpha;
        double vn2 = 0.0;
        for (int i = j + 1; i < k; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        const double vi = 1.0 / std::sqrt(vn2);
        for (int i = j + 1; i < k; ++i) v[i] *= vi;
        // H = I - 2 v v^H ;  A <- H A H via p = A v, K = v^H p, q = p - K v ; A -= 2 (v q^H + q v^H)
        for (int i = 0; i < k; ++i) {
            zc s = 0.0;
            for (int c = j + 1; c < k; ++c) s += A[(size_t)i * k + c] * v[c];
            p[i] = s;
        }
        zc K = 0.0;
        for (int i = j + 1; i < k; ++i) K += std::conj(v[i]) * p[i];
        for (int i = 0; i < k; ++i) q[i] = p[i] - K * v[i];
        for (int i = 0; i < k; ++i)
            for (int c = 0; c < k; ++c)
                A[(size_t)i * k + c] -= 2.0 * (v[i] * std::conj(q[c]) + q[i] * std::conj(v[c]));
        // Q <- Q H
        for (int i = 0; i < k; ++i) {
            zc s = 0.0;
            for (int c = j + 1; c < k; ++c) s += Q[(size_t)i * k + c] * v[c];
            for (int c = j + 1; c < k; ++c) Q[(size_t)i * k + c] -= 2.0 * s * std::conj(v[c]);
        }
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
    std::vector<double> Z((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) Z[(size_t)i * k + i] = 1.0;
    if (!tridiag_ql(k, d, e, Z)) return false;
    std::vector<int> idx(k);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    w.resize(k);
    V.assign((size_t)k * k, zc(0, 0));
    // V = Q diag(dph) Z
    for (int c = 0; c < k; ++c) {
        const int src = idx[c];
        w[c] = d[src];
        for (int i = 0; i < k; ++i) {
            zc s = 0.0;
            for (int m = 0; m < k; ++m) s += Q[(size_t)i * k + m] * dph[m] * Z[(size_t)m * k + src];
            V[(size_t)i * k + c] = s;
        }
    }
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
            for (int m = 0; m < j; ++m) s -= L[(size_t)i * k + m] * std::conj(L[(size_t)j * k + m]);
            L[(size_t)i * k + j] = s / ljj;
        }
    }
    return true;
}

void solve_LH(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int c = 0; c < m; ++c)
        for (int i = k - 1; i >= 0; --i) {
            zc s = X[(size_t)i * m + c];
            for (int j = i + 1; j < k; ++j) s -= std::conj(L[(size_t)j * k + i]) * X[(size_t)j * m + c];
            X[(size_t)i * m + c] = s / L[(size_t)i * k + i].real();
        }
}

void solve_L(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int c = 0; c < m; ++c)
        for (int i = 0; i < k; ++i) {
            zc s = X[(size_t)i * m + c];
            for (int j = 0; j < i; ++j) s -= L[(size_t)i * k + j] * X[(size_t)j * m + c];
            X[(size_t)i * m + c] = s / L[(size_t)i * k + i].real();
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
    if (!herm_eig(k, H, w, V)) return false;
    std::vector<zc> Vw((size_t)k * want);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < want; ++c) Vw[(size_t)i * want + c] = V[(size_t)i * k + c];
    solve_LH(k, L, Vw, want, C);
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

// Host-only self-test hook for the dense routines (interleaved complex, row-major).
extern "C" int pcxd_herm_eig(int k, const double* a, double* w, double* v) {
    std::vector<pcx::zc> A((size_t)k * k);
    for (size_t i = 0; i < A.size(); ++i) A[i] = pcx::zc(a[2 * i], a[2 * i + 1]);
    std::vector<double> ww;
    std::vector<pcx::zc> V;
    if (!pcx::herm_eig(k, A, ww, V)) return -1;
    for (int i = 0; i < k; ++i) w[i] = ww[i];
    for (size_t i = 0; i < V.size(); ++i) {
        v[2 * i] = V[i].real();
        v[2 * i + 1] = V[i].imag();
    }
    return 0;
}
