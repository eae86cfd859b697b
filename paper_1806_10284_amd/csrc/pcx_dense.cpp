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

// implicit QL on the symmetric tridiagonal (d diagonal, e[i] = T(i+1, i)): the published method of
// Bowdler, Martin, Reinsch and Wilkinson ("The QR and QL algorithms for symmetric matrices",
// Numer. Math. 11, 1968), with the shift from the eigenvalue of the leading 2 x 2 block nearer
// d[l] and the bulge chased upwards by plane rotations.  The eigenvector matrix is the product of
// the recorded rotations (applied later to the wanted columns only).
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

// Matrices in split form (real and imaginary parts in separate row-major arrays), so that the
// row operations below are plain real loops the compiler vectorises.
struct SMat {
    int rows = 0, cols = 0;
    std::vector<double> re, im;
    SMat() = default;
    SMat(int r, int c) : rows(r), cols(c), re((size_t)r * c, 0.0), im((size_t)r * c, 0.0) {}
    double* rr(int i) { return re.data() + (size_t)i * cols; }
    double* ri(int i) { return im.data() + (size_t)i * cols; }
    const double* rr(int i) const { return re.data() + (size_t)i * cols; }
    const double* ri(int i) const { return im.data() + (size_t)i * cols; }
};

static SMat split(int r, int c, const std::vector<zc>& A) {
    SMat S(r, c);
    for (size_t e = 0; e < (size_t)r * c; ++e) {
        S.re[e] = A[e].real();
        S.im[e] = A[e].imag();
    }
    return S;
}

static std::vector<zc> join(const SMat& S) {
    std::vector<zc> A((size_t)S.rows * S.cols);
    for (size_t e = 0; e < A.size(); ++e) A[e] = zc(S.re[e], S.im[e]);
    return A;
}

// sum_c a[c] b[c] over n entries (complex, a conjugated when CONJ)
template <bool CONJ>
static inline void dotc(int n, const double* ar, const double* ai, const double* br, const double* bi, double& sr,
                        double& si) {
    double xr = 0.0, xi = 0.0;
    {
        // the order of the additions is free (lets the loop run on vector registers)
#pragma clang fp reassociate(on)
        for (int c = 0; c < n; ++c) {
            if (CONJ) {
                xr += ar[c] * br[c] + ai[c] * bi[c];
                xi += ar[c] * bi[c] - ai[c] * br[c];
            } else {
                xr += ar[c] * br[c] - ai[c] * bi[c];
                xi += ar[c] * bi[c] + ai[c] * br[c];
            }
        }
    }
    sr = xr;
    si = xi;
}

// y[c] -= s x[c] over n entries (complex s)
static inline void axpy_sub(int n, double sr, double si, const double* xr, const double* xi, double* yr, double* yi) {
    for (int c = 0; c < n; ++c) {
        const double a = xr[c], b = xi[c];
        yr[c] -= sr * a - si * b;
        yi[c] -= sr * b + si * a;
    }
}

// Householder reduction and QL on a split Hermitian matrix; V (k x ncols, split) holds the
// eigenvectors of the ncols lowest eigenvalues
static bool herm_eig_split(int k, SMat A, std::vector<double>& w, SMat& V, int ncols) {
    if (ncols < 0 || ncols > k) ncols = k;
    // hermitize
    for (int i = 0; i < k; ++i) {
        A.ri(i)[i] = 0.0;
        for (int j = i + 1; j < k; ++j) {
            const double r = 0.5 * (A.rr(i)[j] + A.rr(j)[i]), m = 0.5 * (A.ri(i)[j] - A.ri(j)[i]);
            A.rr(i)[j] = r;
            A.ri(i)[j] = m;
            A.rr(j)[i] = r;
            A.ri(j)[i] = -m;
        }
    }
    // A = Q T Q^H, Q = H_0 H_1 ... with H_j = I - 2 v_j v_j^H acting on the indices above j; each
    // step updates only the trailing block A[j+1:, j+1:], and only its lower triangle (the matrix
    // stays Hermitian, so the upper one is implied)
    SMat R(k, k);                                   // row j: v_j (zero below index j + 1)
    std::vector<char> has(k, 0);
    std::vector<double> pr(k), pi(k), qr(k), qi(k);
    for (int j = 0; j + 2 < k; ++j) {
        const int o = j + 1, n = k - o;
        // x = A[j+1:, j], the column below the diagonal
        double* vr = R.rr(j) + o;
        double* vi = R.ri(j) + o;
        double xn2 = 0.0;
        for (int i = 0; i < n; ++i) {
            vr[i] = A.rr(o + i)[j];
            vi[i] = A.ri(o + i)[j];
            xn2 += vr[i] * vr[i] + vi[i] * vi[i];
        }
        const double xn = std::sqrt(xn2);
        if (xn == 0.0) continue;
        const zc x0(vr[0], vi[0]);
        const double ax0 = std::abs(x0);
        const zc ph = ax0 > 0 ? zc(x0.real() / ax0, x0.imag() / ax0) : zc(1, 0);
        const zc alpha = -ph * xn;                  // reflect x onto alpha e_1
        vr[0] -= alpha.real();
        vi[0] -= alpha.imag();
        double vn2 = 0.0;
        for (int i = 0; i < n; ++i) vn2 += vr[i] * vr[i] + vi[i] * vi[i];
        if (vn2 == 0.0) continue;
        const double vs = 1.0 / std::sqrt(vn2);
        for (int i = 0; i < n; ++i) {
            vr[i] *= vs;
            vi[i] *= vs;
        }
        has[j] = 1;
        // H A22 H = A22 - 2 (v q^H + q v^H), p = A22 v, K = v^H p (real), q = p - K v; p from the
        // lower triangle: row i's entries left of the diagonal act on v (a dot product) and, as
        // the conjugate column, add to p below them (an axpy)
        for (int i = 0; i < n; ++i) pr[i] = pi[i] = 0.0;
        for (int i = 0; i < n; ++i) {
            const double* ar = A.rr(o + i) + o;
            const double* ai = A.ri(o + i) + o;
            double sr, si;
            dotc<false>(i, ar, ai, vr, vi, sr, si);                 // sum_{c < i} A[i][c] v[c]
            pr[i] += sr + ar[i] * vr[i];
            pi[i] += si + ar[i] * vi[i];
            const double wr = vr[i], wi = vi[i];
            for (int c = 0; c < i; ++c) {                           // p[c] += conj(A[i][c]) v[i]
                pr[c] += ar[c] * wr + ai[c] * wi;
                pi[c] += ar[c] * wi - ai[c] * wr;
            }
        }
        double K = 0.0;
        for (int i = 0; i < n; ++i) K += vr[i] * pr[i] + vi[i] * pi[i];
        for (int i = 0; i < n; ++i) {
            qr[i] = pr[i] - K * vr[i];
            qi[i] = pi[i] - K * vi[i];
        }
        for (int i = 0; i < n; ++i) {
            double* ar = A.rr(o + i) + o;
            double* ai = A.ri(o + i) + o;
            const double v2r = 2.0 * vr[i], v2i = 2.0 * vi[i], q2r = 2.0 * qr[i], q2i = 2.0 * qi[i];
            // a[c] -= 2 v_i conj(q_c) + 2 q_i conj(v_c), c <= i
            for (int c = 0; c <= i; ++c) {
                ar[c] -= v2r * qr[c] + v2i * qi[c] + q2r * vr[c] + q2i * vi[c];
                ai[c] -= v2i * qr[c] - v2r * qi[c] + q2i * vr[c] - q2r * vi[c];
            }
        }
        // the reduced column: alpha e_1
        A.rr(o)[j] = alpha.real();
        A.ri(o)[j] = alpha.imag();
    }
    // phases that make the sub-diagonal real and non-negative
    std::vector<zc> dph(k, zc(1, 0));
    std::vector<double> d(k), e(std::max(k, 1), 0.0);
    for (int i = 0; i < k; ++i) d[i] = A.rr(i)[i];
    for (int i = 0; i + 1 < k; ++i) {
        const zc s(A.rr(i + 1)[i], A.ri(i + 1)[i]);
        const double as = std::abs(s);
        e[i] = as;
        dph[i + 1] = as > 0 ? dph[i] * zc(s.real() / as, s.imag() / as) : dph[i];
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
    // eigenvector c = Q diag(dph) Z[:, idx[c]]: the phases, then H_{k-3}, ..., H_0 in turn (X:
    // row c holds eigenvector c)
    SMat X(ncols, k);
    for (int c = 0; c < ncols; ++c)
        for (int m = 0; m < k; ++m) {
            const double z = Zw[(size_t)m * ncols + c];
            X.rr(c)[m] = dph[m].real() * z;
            X.ri(c)[m] = dph[m].imag() * z;
        }
    for (int j = k - 3; j >= 0; --j) {
        if (!has[j]) continue;
        const int o = j + 1, n = k - o;
        const double* vr = R.rr(j) + o;
        const double* vi = R.ri(j) + o;
        for (int c = 0; c < ncols; ++c) {
            double* xr = X.rr(c) + o;
            double* xi = X.ri(c) + o;
            double sr, si;
            dotc<true>(n, vr, vi, xr, xi, sr, si);          // v^H x
            axpy_sub(n, 2.0 * sr, 2.0 * si, vr, vi, xr, xi);  // x -= 2 (v^H x) v
        }
    }
    V = SMat(k, ncols);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < ncols; ++c) {
            V.rr(i)[c] = X.rr(c)[i];
            V.ri(i)[c] = X.ri(c)[i];
        }
    return true;
}

bool herm_eig(int k, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V, int ncols) {
    if (ncols < 0 || ncols > k) ncols = k;
    SMat Vs;
    if (!herm_eig_split(k, split(k, k, A), w, Vs, ncols)) return false;
    V = join(Vs);
    return true;
}

// G = L L^H on split matrices
static bool cholesky_split(int k, const SMat& G, SMat& L, double rel_tol) {
    L = SMat(k, k);
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) dmax = std::max(dmax, G.rr(i)[i]);
    if (!(dmax > 0.0)) return false;
    for (int j = 0; j < k; ++j) {
        double dj = G.rr(j)[j];
        for (int m = 0; m < j; ++m) dj -= L.rr(j)[m] * L.rr(j)[m] + L.ri(j)[m] * L.ri(j)[m];
        if (!(dj > rel_tol * dmax)) return false;
        const double ljj = std::sqrt(dj), inv = 1.0 / ljj;
        L.rr(j)[j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            // L[i][j] = (G[i][j] - sum_m L[i][m] conj(L[j][m])) / L[j][j]
            double sr, si;
            dotc<true>(j, L.rr(j), L.ri(j), L.rr(i), L.ri(i), sr, si);   // sum conj(L[j][m]) L[i][m]
            L.rr(i)[j] = (G.rr(i)[j] - sr) * inv;
            L.ri(i)[j] = (G.ri(i)[j] - si) * inv;
        }
    }
    return true;
}

// X = L^{-1} B (B: k x m), split
static SMat solve_L_split(int k, const SMat& L, const SMat& B) {
    SMat X = B;
    const int m = B.cols;
    for (int i = 0; i < k; ++i) {
        double* xr = X.rr(i);
        double* xi = X.ri(i);
        for (int j = 0; j < i; ++j) axpy_sub(m, L.rr(i)[j], L.ri(i)[j], X.rr(j), X.ri(j), xr, xi);
        const double inv = 1.0 / L.rr(i)[i];
        for (int c = 0; c < m; ++c) {
            xr[c] *= inv;
            xi[c] *= inv;
        }
    }
    return X;
}

// H = Y L^{-H} where H is Hermitian (Y = L^{-1} G with G Hermitian, so H = L^{-1} G L^{-H}): the
// lower triangle row by row from H L^H = Y, the upper one by conjugate symmetry -- a third of
// the work of a second full triangular solve
static SMat congruence_split(int k, const SMat& L, const SMat& Y) {
    SMat H(k, k);
    for (int i = 0; i < k; ++i) {
        double* hr = H.rr(i);
        double* hi = H.ri(i);
        for (int j = 0; j <= i; ++j) {
            double sr, si;
            dotc<true>(j, L.rr(j), L.ri(j), hr, hi, sr, si);   // sum over m < j of conj(L[j][m]) H[i][m]
            const double inv = 1.0 / L.rr(j)[j];
            hr[j] = (Y.rr(i)[j] - sr) * inv;
            hi[j] = (Y.ri(i)[j] - si) * inv;
        }
    }
    for (int i = 0; i < k; ++i) {
        H.ri(i)[i] = 0.0;
        for (int j = 0; j < i; ++j) {
            H.rr(j)[i] = H.rr(i)[j];
            H.ri(j)[i] = -H.ri(i)[j];
        }
    }
    return H;
}

// X = L^{-H} B (B: k x m), split
static SMat solve_LH_split(int k, const SMat& L, const SMat& B) {
    SMat X = B;
    const int m = B.cols;
    for (int i = k - 1; i >= 0; --i) {
        double* xr = X.rr(i);
        double* xi = X.ri(i);
        for (int j = i + 1; j < k; ++j) axpy_sub(m, L.rr(j)[i], -L.ri(j)[i], X.rr(j), X.ri(j), xr, xi);
        const double inv = 1.0 / L.rr(i)[i];
        for (int c = 0; c < m; ++c) {
            xr[c] *= inv;
            xi[c] *= inv;
        }
    }
    return X;
}

bool cholesky(int k, const std::vector<zc>& G, std::vector<zc>& L, double rel_tol) {
    SMat Ls;
    const bool ok = cholesky_split(k, split(k, k, G), Ls, rel_tol);
    L = ok ? join(Ls) : std::vector<zc>((size_t)k * k, zc(0, 0));
    return ok;
}

void solve_LH(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = join(solve_LH_split(k, split(k, k, L), split(k, m, B)));
}

void solve_L(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = join(solve_L_split(k, split(k, k, L), split(k, m, B)));
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
    SMat L;
    if (!cholesky_split(k, split(k, k, GB), L, chol_tol)) return false;
    const SMat Y = solve_L_split(k, L, split(k, k, GA));      // Y = L^{-1} GA
    const SMat H = congruence_split(k, L, Y);                // H = Y L^{-H} = L^{-1} GA L^{-H}
    std::vector<double> w;
    SMat V;
    if (!herm_eig_split(k, H, w, V, want)) return false;
    const SMat Cs = solve_LH_split(k, L, V);
    C.resize((size_t)k * want);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < want; ++c) C[(size_t)i * want + c] = zc(Cs.rr(i)[c], Cs.ri(i)[c]) * sc[i];
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
