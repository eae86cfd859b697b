// Block LOBPCG on the nullspace-free operator A_r (Section 5.2, eq. NFSEP).
//
// The paper solves A_r y = lambda y by inverse Lanczos with CG inner solves; here the same
// operator drives a block LOBPCG (Knyazev) with
//   * the preconditioner Lambda_q^{-1} on both y-blocks (the Sigma_r^{-2} scaling: by the
//     bound kappa(Q_r* B^{-1} Q_r) <= kappa(B^{-1}) of Section 5.2 the preconditioned operator
//     has condition number at most eps_max / eps_min),
//   * Gram matrices accumulated in FP64 on the device and the Rayleigh-Ritz step solved in
//     FP64 on the host (Cholesky of the basis Gram matrix + cyclic Jacobi),
//   * an optional FP32 phase (FP32 storage and matvecs) followed by an FP64 phase that
//     refines the same block to the requested residual.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pcx_host.h"

namespace pcx {

using zc = std::complex<double>;

// ---------------------------------------------------------------- small dense linear algebra (row-major)

// Hermitian eigen-decomposition by cyclic Jacobi: A = V diag(w) V^H, w ascending.
static void jacobi_eigh(int k, std::vector<zc> A, std::vector<double>& w, std::vector<zc>& V) {
    V.assign((size_t)k * k, zc(0, 0));
    for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
    for (int i = 0; i < k; ++i) A[(size_t)i * k + i] = zc(A[(size_t)i * k + i].real(), 0.0);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < k; ++p) {
            dia += std::norm(A[(size_t)p * k + p]);
            for (int q = p + 1; q < k; ++q) off += std::norm(A[(size_t)p * k + q]);
        }
        if (off <= 1e-32 * dia || off == 0.0) break;
        for (int p = 0; p < k; ++p) {
            for (int q = p + 1; q < k; ++q) {
                const zc apq = A[(size_t)p * k + q];
                const double mag = std::abs(apq);
                if (mag == 0.0) continue;
                const double app = A[(size_t)p * k + p].real(), aqq = A[(size_t)q * k + q].real();
                const zc e = apq / mag;
                const double th = 0.5 * std::atan2(2.0 * mag, aqq - app);
                const double c = std::cos(th), s = std::sin(th);
                const zc eb = std::conj(e);
                // A <- A G with G = [[c, s], [-s conj(e), c conj(e)]] on columns p, q
                for (int r = 0; r < k; ++r) {
                    const zc x = A[(size_t)r * k + p], y = A[(size_t)r * k + q];
                    A[(size_t)r * k + p] = c * x - s * eb * y;
                    A[(size_t)r * k + q] = s * x + c * eb * y;
                }
                // A <- G^H A on rows p, q
                for (int r = 0; r < k; ++r) {
                    const zc x = A[(size_t)p * k + r], y = A[(size_t)q * k + r];
                    A[(size_t)p * k + r] = c * x - s * e * y;
                    A[(size_t)q * k + r] = s * x + c * e * y;
                }
                A[(size_t)p * k + q] = 0.0;
                A[(size_t)q * k + p] = 0.0;
                A[(size_t)p * k + p] = zc(A[(size_t)p * k + p].real(), 0.0);
                A[(size_t)q * k + q] = zc(A[(size_t)q * k + q].real(), 0.0);
                for (int r = 0; r < k; ++r) {
                    const zc x = V[(size_t)r * k + p], y = V[(size_t)r * k + q];
                    V[(size_t)r * k + p] = c * x - s * eb * y;
                    V[(size_t)r * k + q] = s * x + c * eb * y;
                }
            }
        }
    }
    std::vector<int> idx(k);
    for (int i = 0; i < k; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(),
              [&](int a, int b) { return A[(size_t)a * k + a].real() < A[(size_t)b * k + b].real(); });
    w.resize(k);
    std::vector<zc> Vs((size_t)k * k);
    for (int c = 0; c < k; ++c) {
        w[c] = A[(size_t)idx[c] * k + idx[c]].real();
        for (int r = 0; r < k; ++r) Vs[(size_t)r * k + c] = V[(size_t)r * k + idx[c]];
    }
    V.swap(Vs);
}

// G = L L^H, L lower triangular; false if a pivot is not safely positive.
static bool cholesky(int k, const std::vector<zc>& G, std::vector<zc>& L, double rel_tol) {
    L.assign((size_t)k * k, zc(0, 0));
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) dmax = std::max(dmax, G[(size_t)i * k + i].real());
    if (!(dmax > 0.0)) return false;
    for (int j = 0; j < k; ++j) {
        double d = G[(size_t)j * k + j].real();
        for (int m = 0; m < j; ++m) d -= std::norm(L[(size_t)j * k + m]);
        if (!(d > rel_tol * dmax)) return false;
        const double ljj = std::sqrt(d);
        L[(size_t)j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            zc s = G[(size_t)i * k + j];
            for (int m = 0; m < j; ++m) s -= L[(size_t)i * k + m] * std::conj(L[(size_t)j * k + m]);
            L[(size_t)i * k + j] = s / ljj;
        }
    }
    return true;
}

// X = L^{-H} B  (B: k x m), back substitution with the upper triangular L^H
static void solve_LH(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int c = 0; c < m; ++c) {
        for (int i = k - 1; i >= 0; --i) {
            zc s = X[(size_t)i * m + c];
            for (int j = i + 1; j < k; ++j) s -= std::conj(L[(size_t)j * k + i]) * X[(size_t)j * m + c];
            X[(size_t)i * m + c] = s / L[(size_t)i * k + i].real();
        }
    }
}

// X = L^{-1} B (B: k x m), forward substitution
static void solve_L(int k, const std::vector<zc>& L, const std::vector<zc>& B, int m, std::vector<zc>& X) {
    X = B;
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < k; ++i) {
            zc s = X[(size_t)i * m + c];
            for (int j = 0; j < i; ++j) s -= L[(size_t)i * k + j] * X[(size_t)j * m + c];
            X[(size_t)i * m + c] = s / L[(size_t)i * k + i].real();
        }
    }
}

static void hermitize(int k, std::vector<zc>& A) {
    for (int i = 0; i < k; ++i) {
        A[(size_t)i * k + i] = zc(A[(size_t)i * k + i].real(), 0.0);
        for (int j = i + 1; j < k; ++j) {
            const zc a = 0.5 * (A[(size_t)i * k + j] + std::conj(A[(size_t)j * k + i]));
            A[(size_t)i * k + j] = a;
            A[(size_t)j * k + i] = std::conj(a);
        }
    }
}

// Rayleigh-Ritz for the pencil (GA, GB): lowest `want` pairs; C is k x want with C^H GB C = I.
static bool rayleigh_ritz(int k, std::vector<zc> GA, std::vector<zc> GB, int want, double chol_tol,
                          std::vector<double>& theta, std::vector<zc>& C) {
    hermitize(k, GA);
    hermitize(k, GB);
    std::vector<zc> L;
    if (!cholesky(k, GB, L, chol_tol)) return false;
    std::vector<zc> Y, H, Ht;
    solve_L(k, L, GA, k, Y);                 // Y = L^{-1} GA
    std::vector<zc> Yh((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) Yh[(size_t)i * k + j] = std::conj(Y[(size_t)j * k + i]);
    solve_L(k, L, Yh, k, Ht);                // Ht = L^{-1} Y^H = (Y L^{-H})^H = H^H = H
    hermitize(k, Ht);
    std::vector<double> w;
    std::vector<zc> V;
    jacobi_eigh(k, Ht, w, V);
    std::vector<zc> Vw((size_t)k * want);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < want; ++c) Vw[(size_t)i * want + c] = V[(size_t)i * k + c];
    solve_LH(k, L, Vw, want, C);
    theta.assign(w.begin(), w.begin() + want);
    return true;
}

// ---------------------------------------------------------------- the solver

template <typename R>
struct Blocks {
    cx<R>* X; cx<R>* AX; cx<R>* W; cx<R>* AW; cx<R>* P; cx<R>* AP;
    cx<R>* T1; cx<R>* T2; cx<R>* T3; cx<R>* T4;
};

struct Solver {
    Plan* p;
    const double* kappa;
    int nev, b;
    long n, N;
    pcx_opts o;
    pcx_stats st;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool pending_event = false;
    double* prec = nullptr;              // device, n
    cx<double>* gram_part = nullptr;     // device
    int gram_chunks = 0;
    cx<double>* dev_small = nullptr;     // device: gram output, then C matrices
    double* dev_theta = nullptr;         // device, b
    double* res_part = nullptr;          // device
    double* res_out = nullptr;           // device, b
    std::vector<double> theta;           // host
    std::vector<double> resid;           // host, relative residuals of the current block

    int sync() {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: stream");
        if (pending_event) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) st.seconds_matvec += ms * 1e-3;
            pending_event = false;
        }
        return PCX_OK;
    }

    template <typename R>
    int matvec(const cx<R>* in, cx<R>* out, int m) {
        (void)hipEventRecord(ev0, p->stream);
        int rc = p->apply(Plan::OP_AR, kappa, sizeof(R) == 8 ? PCX_FP64 : PCX_FP32, in, out, m);
        (void)hipEventRecord(ev1, p->stream);
        pending_event = true;
        st.matvecs += m;
        if (sizeof(R) == 4) st.matvecs_fp32 += m;
        return rc;
    }

    // G (ka x kb) = A^H B on the host
    template <typename R>
    int gram(const ColSet& A, const ColSet& B, std::vector<zc>& G) {
        const int ka = A.total(), kb = B.total();
        hipError_t e = launch_gram<R>(A, B, N, gram_part, gram_chunks, dev_small, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: gram");
        G.resize((size_t)ka * kb);
        e = hipMemcpyAsync(G.data(), dev_small, sizeof(zc) * ka * kb, hipMemcpyDeviceToHost, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: gram copy");
        return sync();
    }

    // Y = S C with C (ks x m) from the host
    template <typename R>
    int combine(const ColSet& S, const std::vector<zc>& C, const ColSet& Y) {
        hipError_t e = hipMemcpyAsync(dev_small, C.data(), sizeof(zc) * C.size(), hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: coefficient copy");
        e = launch_combine<R>(S, (const cx<double>*)dev_small, Y, N, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: combine");
        // the coefficient buffer is reused by the next call: keep the host ahead by at most one launch
        return sync();
    }

    // Cholesky-QR (SVQB fallback) of the b columns of `Y`, result into `T`; then swap.
    template <typename R>
    int orthonormalize(cx<R>*& Y, cx<R>*& T) {
        std::vector<zc> G;
        int rc = gram<R>(colset(Y, b), colset(Y, b), G);
        if (rc) return rc;
        std::vector<zc> L, C, I((size_t)b * b, zc(0, 0));
        for (int i = 0; i < b; ++i) I[(size_t)i * b + i] = 1.0;
        hermitize(b, G);
        if (cholesky(b, G, L, 1e-14)) {
            solve_LH(b, L, I, b, C);
        } else {
            std::vector<double> w;
            std::vector<zc> V;
            jacobi_eigh(b, G, w, V);
            const double wmax = std::max(w.back(), 1e-300);
            C.assign((size_t)b * b, zc(0, 0));
            for (int c = 0; c < b; ++c) {
                const double d = 1.0 / std::sqrt(std::max(w[c], 1e-14 * wmax));
                for (int r = 0; r < b; ++r) C[(size_t)r * b + c] = V[(size_t)r * b + c] * d;
            }
        }
        rc = combine<R>(colset(Y, b), C, colset(T, b));
        if (rc) return rc;
        std::swap(Y, T);
        return PCX_OK;
    }

    template <typename R>
    int residuals(Blocks<R>& B) {
        hipError_t e = hipMemcpyAsync(dev_theta, theta.data(), sizeof(double) * b, hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: theta copy");
        e = launch_residual<R>(colset(B.X, b), colset(B.AX, b), dev_theta, o.precondition ? prec : nullptr, n,
                               colset(B.W, b), res_part, gram_chunks, res_out, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: residual");
        std::vector<double> r2(b);
        e = hipMemcpyAsync(r2.data(), res_out, sizeof(double) * b, hipMemcpyDeviceToHost, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: residual copy");
        int rc = sync();
        if (rc) return rc;
        resid.resize(b);
        for (int j = 0; j < b; ++j) resid[j] = std::sqrt(std::max(r2[j], 0.0)) / std::max(std::fabs(theta[j]), 1e-300);
        return PCX_OK;
    }

    // Rayleigh-Ritz on the b columns of X alone (start of a phase)
    template <typename R>
    int rr_block(Blocks<R>& B) {
        std::vector<zc> GA, GB;
        int rc = gram<R>(colset(B.X, b), colset(B.AX, b), GA);
        if (rc) return rc;
        rc = gram<R>(colset(B.X, b), colset(B.X, b), GB);
        if (rc) return rc;
        std::vector<zc> C;
        if (!rayleigh_ritz(b, GA, GB, b, 1e-14, theta, C)) return fail(PCX_E_NOCONV, "pcx_solve: start block is singular");
        if ((rc = combine<R>(colset(B.X, b), C, colset(B.T1, b)))) return rc;
        if ((rc = combine<R>(colset(B.AX, b), C, colset(B.T2, b)))) return rc;
        std::swap(B.X, B.T1);
        std::swap(B.AX, B.T2);
        return PCX_OK;
    }

    // one phase of LOBPCG at precision R, starting from the b columns in B.X
    template <typename R>
    int phase(Blocks<R>& B, double tol, int max_iter, int& iters) {
        int rc;
        hipError_t e = launch_mask<R>(B.X, prec, n, b, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: mask");
        for (int pass = 0; pass < 2; ++pass)
            if ((rc = orthonormalize<R>(B.X, B.T1))) return rc;
        if ((rc = matvec<R>(B.X, B.AX, b))) return rc;
        if ((rc = rr_block<R>(B))) return rc;
        bool hasP = false;
        const double chol_tol = sizeof(R) == 8 ? 1e-13 : 1e-9;
        double best = 1e300;
        int stall = 0;
        for (;;) {
            if ((rc = residuals<R>(B))) return rc;
            bool all = true;
            double worst = 0;
            for (int j = 0; j < nev; ++j) {
                all = all && resid[j] <= tol;
                worst = std::max(worst, resid[j]);
            }
            if (o.verbose)
                fprintf(stderr, "pcx lobpcg %s it %d: theta0 %.12g worst residual %.3e\n", sizeof(R) == 8 ? "fp64" : "fp32",
                        iters, theta[0], worst);
            if (all || iters >= max_iter) return PCX_OK;
            // a reduced-precision phase ends when its residual stops improving (rounding floor)
            if (worst < 0.9 * best) {
                best = worst;
                stall = 0;
            } else if (sizeof(R) == 4 && ++stall >= 8) {
                return PCX_OK;
            }
            ++iters;
            ++st.iterations;
            if (sizeof(R) == 4) ++st.iterations_fp32;
            // W <- W - X (X^H W), twice, then orthonormalise W
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<zc> G, C((size_t)2 * b * b, zc(0, 0));
                if ((rc = gram<R>(colset(B.X, b), colset(B.W, b), G))) return rc;
                for (int r = 0; r < b; ++r)
                    for (int c = 0; c < b; ++c) C[(size_t)r * b + c] = -G[(size_t)r * b + c];
                for (int r = 0; r < b; ++r) C[(size_t)(b + r) * b + r] = 1.0;
                if ((rc = combine<R>(colset(B.X, b, B.W, b), C, colset(B.T1, b)))) return rc;
                std::swap(B.W, B.T1);
            }
            if ((rc = orthonormalize<R>(B.W, B.T1))) return rc;
            if ((rc = matvec<R>(B.W, B.AW, b))) return rc;
            // Rayleigh-Ritz on S = [X W P]
            std::vector<double> th;
            std::vector<zc> C;
            int k = 0;
            for (int tryP = hasP ? 1 : 0; tryP >= 0; --tryP) {
                k = tryP ? 3 * b : 2 * b;
                ColSet S = tryP ? colset(B.X, b, B.W, b, B.P, b) : colset(B.X, b, B.W, b);
                // B-set = [S | AS]: build with up to 4 runs; AS runs follow
                ColSet BS;
                if (tryP) {
                    // [X W P AX] and [AW AP] as two gram calls to stay within 4 runs
                    std::vector<zc> G1, G2;
                    if ((rc = gram<R>(S, colset(B.X, b, B.W, b, B.P, b), G1))) return rc;
                    if ((rc = gram<R>(S, colset(B.AX, b, B.AW, b, B.AP, b), G2))) return rc;
                    std::vector<zc> GB((size_t)k * k), GA((size_t)k * k);
                    for (size_t q = 0; q < GB.size(); ++q) { GB[q] = G1[q]; GA[q] = G2[q]; }
                    if (rayleigh_ritz(k, GA, GB, b, chol_tol, th, C)) break;
                } else {
                    std::vector<zc> G;
                    BS = colset(B.X, b, B.W, b, B.AX, b);
                    BS.ptr[3] = B.AW;
                    BS.ncols[3] = b;
                    BS.nseg = 4;
                    if ((rc = gram<R>(S, BS, G))) return rc;
                    std::vector<zc> GB((size_t)k * k), GA((size_t)k * k);
                    for (int r = 0; r < k; ++r)
                        for (int c = 0; c < k; ++c) {
                            GB[(size_t)r * k + c] = G[(size_t)r * 2 * k + c];
                            GA[(size_t)r * k + c] = G[(size_t)r * 2 * k + k + c];
                        }
                    if (rayleigh_ritz(k, GA, GB, b, chol_tol, th, C)) break;
                    return fail(PCX_E_NOCONV, "pcx_solve: Rayleigh-Ritz basis became singular");
                }
            }
            // [X' | P'] = S [C | C_P], C_P = C with the X rows zeroed
            std::vector<zc> C2((size_t)k * 2 * b, zc(0, 0));
            for (int r = 0; r < k; ++r)
                for (int c = 0; c < b; ++c) {
                    C2[(size_t)r * 2 * b + c] = C[(size_t)r * b + c];
                    if (r >= b) C2[(size_t)r * 2 * b + b + c] = C[(size_t)r * b + c];
                }
            ColSet S = k == 3 * b ? colset(B.X, b, B.W, b, B.P, b) : colset(B.X, b, B.W, b);
            ColSet AS = k == 3 * b ? colset(B.AX, b, B.AW, b, B.AP, b) : colset(B.AX, b, B.AW, b);
            if ((rc = combine<R>(S, C2, colset(B.T1, b, B.T3, b)))) return rc;
            if ((rc = combine<R>(AS, C2, colset(B.T2, b, B.T4, b)))) return rc;
            std::swap(B.X, B.T1);
            std::swap(B.P, B.T3);
            std::swap(B.AX, B.T2);
            std::swap(B.AP, B.T4);
            theta = th;
            hasP = true;
        }
    }
};

template <typename R>
static Blocks<R> carve(void* base, int b, long N) {
    cx<R>* q = (cx<R>*)base;
    const size_t s = (size_t)b * N;
    Blocks<R> B;
    B.X = q; B.AX = q + s; B.W = q + 2 * s; B.AW = q + 3 * s; B.P = q + 4 * s; B.AP = q + 5 * s;
    B.T1 = q + 6 * s; B.T2 = q + 7 * s; B.T3 = q + 8 * s; B.T4 = q + 9 * s;
    return B;
}

}  // namespace pcx

using namespace pcx;

extern "C" void pcx_opts_default(pcx_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = PCX_MODE_FP64;
    o->block = 0;
    o->max_iter = 400;
    o->tol = 1e-9;
    o->tol_fp32 = 1e-3;
    o->seed = 12345;
    o->precondition = 1;
    o->verbose = 0;
}

extern "C" int pcx_solve(pcx_plan* pp, const double kappa[3], int nev, const pcx_opts* opts, double* lambda,
                         void* y_out, void* x_out, pcx_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    Plan* p = (Plan*)pp;
    if (!p || !kappa || !lambda) return fail(PCX_E_ARG, "pcx_solve: null pointer");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_solve: permittivity not set");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "pcx_solve: non-finite kappa");
    Solver S;
    S.p = p;
    S.kappa = kappa;
    if (opts) S.o = *opts;
    else pcx_opts_default(&S.o);
    std::memset(&S.st, 0, sizeof(S.st));
    const long n = p->n, N = 2 * n;
    S.n = n;
    S.N = N;
    if (nev < 1) return fail(PCX_E_ARG, "pcx_solve: nev must be >= 1");
    int b = S.o.block > 0 ? S.o.block : nev + std::max(2, nev / 4);
    if (b < nev) return fail(PCX_E_ARG, "pcx_solve: block (%d) smaller than nev (%d)", b, nev);
    if (b > PCX_MAX_BLOCK || 3L * b > N - 2) return fail(PCX_E_ARG, "pcx_solve: block %d too large for this grid", b);
    if (S.o.mode < PCX_MODE_FP64 || S.o.mode > PCX_MODE_FP32) return fail(PCX_E_ARG, "pcx_solve: bad mode");
    if (!(S.o.tol > 0) || S.o.max_iter < 1) return fail(PCX_E_ARG, "pcx_solve: bad tolerance or max_iter");
    if (b > p->max_vectors) return fail(PCX_E_ARG, "pcx_solve: block %d exceeds the plan's max_vectors", b);
    S.nev = nev;
    S.b = b;
    const bool use32 = S.o.mode != PCX_MODE_FP64;
    const bool use64 = S.o.mode != PCX_MODE_FP32;
    int rc;
    if (use64 && (rc = p->check_fits(PCX_FP64))) return rc;
    if (use32 && (rc = p->check_fits(PCX_FP32))) return rc;

    // storage: FP64 blocks, then FP32 blocks
    const size_t bytes64 = use64 ? 10 * (size_t)b * N * sizeof(cx<double>) : 0;
    const size_t bytes32 = use32 ? 10 * (size_t)b * N * sizeof(cx<float>) : 0;
    if ((rc = p->grow(&p->lob_mem, &p->lob_cap, bytes64 + bytes32))) return rc;
    if ((rc = p->grow(&p->prec, &p->prec_cap, n * sizeof(double)))) return rc;
    S.gram_chunks = (int)std::min<long>(1024, std::max<long>(1, N / 1024));
    const size_t gp = (size_t)S.gram_chunks * (3 * b) * (3 * b) * sizeof(cx<double>);
    const size_t rp = (size_t)S.gram_chunks * b * sizeof(double);
    if ((rc = p->grow(&p->gram_part, &p->gram_part_cap, gp + rp))) return rc;
    const size_t small = (size_t)(3 * b) * (4 * b) * sizeof(cx<double>) + 2 * b * sizeof(double) + 1024;
    if ((rc = p->grow(&p->small_mem, &p->small_cap, std::max<size_t>(small, 1 << 16)))) return rc;
    S.prec = (double*)p->prec;
    S.gram_part = (cx<double>*)p->gram_part;
    S.res_part = (double*)((char*)p->gram_part + gp);
    S.dev_small = (cx<double>*)p->small_mem;
    S.dev_theta = (double*)((char*)p->small_mem + (size_t)(3 * b) * (4 * b) * sizeof(cx<double>));
    S.res_out = S.dev_theta + b;
    (void)hipEventCreate(&S.ev0);
    (void)hipEventCreate(&S.ev1);

    const Grid g = p->grid(kappa);
    hipError_t e = launch_precond_diag(g, p->tables, S.prec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_solve: preconditioner");

    Blocks<double> B64{};
    Blocks<float> B32{};
    if (use64) B64 = carve<double>(p->lob_mem, b, N);
    if (use32) B32 = carve<float>((char*)p->lob_mem + bytes64, b, N);
    int iters = 0;
    rc = PCX_OK;
    if (use32) {
        e = launch_random<float>(B32.X, (long)b * N, S.o.seed, p->stream);
        if (e != hipSuccess) rc = hip_fail(e, "pcx_solve: random start");
        const double tol32 = S.o.mode == PCX_MODE_FP32 ? S.o.tol : std::max(S.o.tol, S.o.tol_fp32);
        if (!rc) rc = S.phase<float>(B32, tol32, S.o.max_iter, iters);
        if (!rc && use64) {
            e = launch_convert(B32.X, B64.X, (long)b * N, p->stream);
            if (e != hipSuccess) rc = hip_fail(e, "pcx_solve: convert");
        }
    } else {
        e = launch_random<double>(B64.X, (long)b * N, S.o.seed, p->stream);
        if (e != hipSuccess) rc = hip_fail(e, "pcx_solve: random start");
    }
    if (!rc && use64) rc = S.phase<double>(B64, S.o.tol, S.o.max_iter, iters);
    if (!rc) {
        for (int j = 0; j < nev; ++j) lambda[j] = S.theta[j];
        int conv = 0;
        for (int j = 0; j < nev; ++j) {
            if (j < PCX_MAX_BLOCK) S.st.residual[j] = S.resid[j];
            if (S.resid[j] <= S.o.tol) ++conv;
        }
        S.st.converged = conv;
        // outputs: y (FP64), x = B^{-1} Q_r Sigma_r y
        if (y_out) {
            if (use64) e = hipMemcpyAsync(y_out, B64.X, sizeof(cx<double>) * nev * N, hipMemcpyDeviceToDevice, p->stream);
            else e = launch_convert(B32.X, (cx<double>*)y_out, (long)nev * N, p->stream);
            if (e != hipSuccess) rc = hip_fail(e, "pcx_solve: y output");
        }
        if (!rc && x_out) {
            if (use64) {
                rc = p->apply(Plan::OP_EIGVEC, kappa, PCX_FP64, B64.X, x_out, nev);
            } else {
                // promote to FP64 through the T1 block, then map
                cx<double>* tmp = (cx<double>*)y_out;
                if (!tmp) rc = fail(PCX_E_ARG, "pcx_solve: FP32 mode needs y_out to return x_out");
                else rc = p->apply(Plan::OP_EIGVEC, kappa, PCX_FP64, tmp, x_out, nev);
            }
        }
        if (!rc) rc = S.sync();
        if (!rc && conv < nev) rc = fail(PCX_E_NOCONV, "pcx_solve: %d of %d bands converged after %d iterations", conv, nev, iters);
    }
    (void)hipEventDestroy(S.ev0);
    (void)hipEventDestroy(S.ev1);
    S.st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S.st;
    return rc;
}
