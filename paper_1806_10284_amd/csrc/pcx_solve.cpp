// Block LOBPCG on the nullspace-free operator A_r (Section 5.2, eq. NFSEP).
//
// The paper solves A_r y = lambda y by inverse Lanczos with CG inner solves; here the same
// operator drives a block LOBPCG (Knyazev) with
//   * a preconditioner: Lambda_q^{-1} on both y-blocks (the Sigma_r^{-2} scaling: by the bound
//     kappa(Q_r* B^{-1} Q_r) <= kappa(B^{-1}) of Section 5.2 the preconditioned operator has
//     condition number at most eps_max / eps_min), or by default the approximate inverse
//     Sigma_r^{-1} Q_r* B Q_r Sigma_r^{-1} (the same FFT operator with eps for 1/eps between two
//     Lambda_q^{-1} scalings), whose preconditioned spectrum lies in [1, (eps_max + eps_min)^2 /
//     (4 eps_max eps_min)],
//   * Gram matrices accumulated in FP64 on the device and the Rayleigh-Ritz step solved in
//     FP64 on the host (Cholesky of the basis Gram matrix, Householder tridiagonalisation and
//     implicit QL),
//   * one host synchronisation per iteration: the new directions enter the Rayleigh-Ritz basis
//     without orthogonalisation against X, so the residual norms and the basis Gram matrix reach
//     the host together,
//   * an optional FP32 phase (FP32 storage and matvecs) followed by an FP64 phase that
//     refines the same block to the requested residual.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <type_traits>
#include <vector>

#include "pcx_dense.h"
#include "pcx_host.h"

#ifndef PCX_FLOOR_FACTOR
#define PCX_FLOOR_FACTOR 1024
#endif
#ifndef PCX_FP32_STALL
#define PCX_FP32_STALL 12
#endif

namespace pcx {

// iterations without a 10% drop of the worst residual that end a reduced-precision phase
constexpr int kFp32Stall = PCX_FP32_STALL;
// the same for the FP64 phase (then the solve reports the bands it did not converge)
constexpr int kFp64Stall = 40;
// FP64 absolute residual floor in units of eps ||A_r||
constexpr double kFloor = PCX_FLOOR_FACTOR;
// Rayleigh-Ritz: smallest accepted Cholesky pivot of the unit-scaled basis Gram matrix (relative to
// its largest), else the step is retried without P.  FP32 columns carry ~6e-8 relative rounding,
// amplified in the Ritz coefficients by 1 / sqrt(pivot); a 1e-9 bound let a nearly dependent P
// through and the implicitly updated A S drift until Ritz values went negative (FCC 64^3, the
// approximate-inverse preconditioner); 1e-6 keeps the amplification below 1e3.  In FP64 a 1e-13
// bound let a P through that had become nearly dependent once the residuals reached ~1e-10 (SC
// sphere at Gamma, started from the eigenvectors of the neighbouring path point): the Ritz vectors
// lost accuracy and the residuals climbed back to 1e-4; 1e-11 drops that P (the cold solves of the
// same path take the same iterations with either bound).
constexpr double kCholTol32 = 1e-6;
constexpr double kCholTol64 = 1e-11;

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
    cx<double>* dev_small = nullptr;     // device: the small area (coefficient slots, theta)
    double* res_part = nullptr;          // device
    static constexpr int kSlots = 8;
    zc* pinned = nullptr;                // host, kSlots * slot_elems
    zc* host_gram = nullptr;             // host (pinned), gram results
    double* host_res = nullptr;          // host (pinned), b
    // the device's addresses of host_gram and host_res: the final reduction kernels store the Gram
    // matrix and the residual norms straight into pinned host memory (one copy fewer per host
    // synchronisation: about 9 us of a 21 us round trip on MI355X)
    cx<double>* gram_map = nullptr;
    double* res_map = nullptr;
    cx<double>* dev_slots = nullptr;     // device, kSlots * slot_elems
    size_t slot_elems = 0;
    int slot_next = 0;
    std::vector<double> theta;           // host
    std::vector<double> resid;           // host, relative residuals of the current block
    std::vector<double> rabs;            // host, absolute residual norms ||A_r x - theta x||
    double anorm = 0;                    // ||A_r|| <= max Lambda_q / min eps
    // columns [pre_lo, pre_hi) get the approximate-inverse preconditioner: the span of the
    // columns open at the previous convergence check (the others have converged; should one
    // reopen, its W is still the Lambda_q^{-1}-preconditioned residual)
    int pre_lo = 0, pre_hi = 0;
    // one plane wave with Lambda_q far below the others (next to Gamma): its bands go to zero and
    // the FP64 phase applies the preconditioner in FP64 (FP32 rounding of the preconditioned
    // residual, dominated by that mode, stalls and then upsets those bands near 1e-9)
    bool near_gamma = false;

    // Band j has converged when its relative residual is below tol or, for eigenvalues so close
    // to zero (next to Gamma) that tol |theta| is below what the arithmetic can resolve, when its
    // absolute residual is at the working-precision floor c eps ||A_r||: c = 1024 in FP64 (the
    // level where LOBPCG's basis stops improving next to Gamma, ~1e-13 ||A_r||), c = 1 in FP32
    // (the matvec's own rounding).  The eigenvalue error of such a band is ~ residual^2 / gap.
    // In the FP64 phase the floor applies only to bands whose tol |theta| lies four orders below it
    // (the bands that go to zero next to Gamma, which cannot reach tol; point 30 of the FCC path
    // then takes 44 iterations instead of 136), inside the iteration only next to Gamma and in the
    // final verdict everywhere: every other band must reach tol itself (at 64^3 the FP64 floor,
    // ~1.4e-8, lies above tol |theta| ~ 1e-9 of ordinary bands, which do reach tol).  The FP32
    // phase accepts any band at its floor (refinement follows).
    template <typename R>
    bool at_floor(int j, double tol) const {
        const double floor = (sizeof(R) == 8 ? kFloor * 1.1102230246251565e-16 : 5.9604644775390625e-08) * anorm;
        if (rabs[j] > floor) return false;
        return sizeof(R) == 4 || tol * std::fabs(theta[j]) < 1e-4 * floor;
    }
    template <typename R>
    bool converged(int j, double tol, bool final_verdict = false) const {
        if (resid[j] <= tol) return true;
        if (!at_floor<R>(j, tol)) return false;
        return sizeof(R) == 4 || final_verdict || near_gamma;
    }

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

    // G (ka x kb) = A^H B on the host, in two halves: gram_async queues the product and its copy
    // into pinned host memory, gram_read takes it after a stream synchronisation.  herm: B = [A]
    // or [A | AA] with each ka x ka half Hermitian; the device computes the upper part and the
    // lower part is mirrored here.
    template <typename R>
    int gram_async(const ColSet& A, const ColSet& B, bool herm) {
        const int ka = A.total(), kb = B.total();
        (void)ka;
        (void)kb;
        const hipError_t e = launch_gram<R>(A, B, N, gram_part, gram_chunks, gram_map, p->stream, herm);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: gram");
        return PCX_OK;
    }

    void gram_read(int ka, int kb, std::vector<zc>& G, bool herm) {
        G.assign(host_gram, host_gram + (size_t)ka * kb);
        if (!herm) return;
        for (int h = 0; h < kb / ka; ++h)
            for (int i = 0; i < ka; ++i) {
                zc* row = G.data() + (size_t)i * kb + (size_t)h * ka;
                row[i] = zc(row[i].real(), 0.0);
                for (int j = 0; j < i; ++j) row[j] = std::conj(G[(size_t)j * kb + (size_t)h * ka + i]);
            }
    }

    template <typename R>
    int gram(const ColSet& A, const ColSet& B, std::vector<zc>& G, bool herm = false) {
        int rc = gram_async<R>(A, B, herm);
        if (!rc) rc = sync();
        if (!rc) gram_read(A.total(), B.total(), G, herm);
        return rc;
    }

    // Y = S C with C (ks x m) from the host.  The coefficients go through a ring of pinned host
    // slots into matching device slots; stream order keeps each device slot alive until its
    // combine has run, and a slot is reused only after several stream synchronisations.
    int stage(const std::vector<zc>& C, const cx<double>** dst) {
        if (C.size() > slot_elems) return fail(PCX_E_ARG, "pcx_solve: coefficient block too large");
        const int q = slot_next;
        slot_next = (slot_next + 1) % kSlots;
        std::copy(C.begin(), C.end(), pinned + (size_t)q * slot_elems);
        cx<double>* d = dev_slots + (size_t)q * slot_elems;
        hipError_t e = hipMemcpyAsync(d, pinned + (size_t)q * slot_elems, sizeof(zc) * C.size(),
                                      hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: coefficient copy");
        *dst = d;
        return PCX_OK;
    }
    template <typename R>
    int combine_staged(const ColSet& S, const cx<double>* C, const ColSet& Y) {
        hipError_t e = launch_combine<R>(S, C, Y, N, p->stream);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve: combine");
    }
    template <typename R>
    int combine(const ColSet& S, const std::vector<zc>& C, const ColSet& Y) {
        const cx<double>* d = nullptr;
        int rc = stage(C, &d);
        return rc ? rc : combine_staged<R>(S, d, Y);
    }
    // Y1 = S1 C and Y2 = S2 C from one staged copy of C
    template <typename R>
    int combine2(const ColSet& S1, const ColSet& Y1, const ColSet& S2, const ColSet& Y2, const std::vector<zc>& C) {
        const cx<double>* d = nullptr;
        int rc = stage(C, &d);
        if (!rc) rc = combine_staged<R>(S1, d, Y1);
        if (!rc) rc = combine_staged<R>(S2, d, Y2);
        return rc;
    }

    // Cholesky-QR (SVQB fallback) of the b columns of `Y`, result into `T`; then swap.
    template <typename R>
    int orthonormalize(cx<R>*& Y, cx<R>*& T, int m) {
        std::vector<zc> G, C;
        int rc = gram<R>(colset(Y, m), colset(Y, m), G, true);
        if (rc) return rc;
        orthonormalizer(m, G, C);
        rc = combine<R>(colset(Y, m), C, colset(T, m));
        if (rc) return rc;
        std::swap(Y, T);
        return PCX_OK;
    }

    // W[pre_lo, pre_lo + npre) <- D A_r(eps) D r with D = Lambda_q^{-1} (the residual kernel has
    // applied the inner D), in FP32 also in the FP64 phase away from Gamma: the preconditioner only
    // shapes the search direction (the Rayleigh-Ritz step and the residuals stay in the phase's
    // precision), and the FP32 kernels take about half the time of the FP64 ones.  AW is free
    // until the next matvec and holds the intermediate vectors.
    template <typename R>
    int precondition_inverse(Blocks<R>& B, int npre) {
        hipError_t e;
        cx<R>* w0 = B.W + (size_t)pre_lo * N;
        if (sizeof(R) == 8 && near_gamma) {
            cx<R>* t0 = B.AW + (size_t)pre_lo * N;
            if (int rc = p->apply(Plan::OP_AR_EPS, kappa, PCX_FP64, w0, t0, npre)) return rc;
            st.precond_applies += npre;
            e = launch_scale_modes<R>(t0, w0, prec, n, npre, p->stream);
            return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve: preconditioner scaling");
        }
        // FP64 phase on the register kernels: FP64 in and out, rounding to FP32 on the way in and the
        // outer D on the way out, in place
        if (sizeof(R) == 8) {
            bool done = false;
            if (int rc = p->precond_mixed(kappa, w0, w0, prec, npre, &done)) return rc;
            if (done) {
                st.precond_applies += npre;
                st.precond_applies_fp32 += npre;
                return PCX_OK;
            }
        }
        // FP64 phase: AW (b columns of complex128) holds the FP32 input and output side by side;
        // FP32 phase: W itself is the input and AW the output
        cx<float>* tin = sizeof(R) == 8 ? (cx<float>*)(void*)B.AW : (cx<float>*)(void*)w0;
        cx<float>* tout = sizeof(R) == 8 ? tin + (size_t)npre * N : (cx<float>*)(void*)B.AW;
        if (sizeof(R) == 8) {
            e = launch_convert((const cx<double>*)(const void*)w0, tin, (long)npre * N, p->stream);
            if (e != hipSuccess) return hip_fail(e, "pcx_solve: preconditioner input");
        }
        if (int rc = p->apply(Plan::OP_AR_EPS, kappa, PCX_FP32, tin, tout, npre)) return rc;
        st.precond_applies += npre;
        st.precond_applies_fp32 += npre;
        if (sizeof(R) == 8)
            e = launch_scale_modes(tout, (cx<double>*)(void*)w0, prec, n, npre, p->stream);
        else
            e = launch_scale_modes<float>(tout, (cx<float>*)(void*)w0, prec, n, npre, p->stream);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve: preconditioner scaling");
    }

    // queues W <- prec (AX - X theta) and the residual norms of the b Ritz pairs (read after the
    // next stream synchronisation by read_residuals)
    template <typename R>
    int residuals_async(Blocks<R>& B) {
        hipError_t e = launch_residual<R>(colset(B.X, b), colset(B.AX, b), theta.data(), o.precondition ? prec : nullptr, n,
                               colset(B.W, b), res_part, gram_chunks, res_map, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: residual");
        const int npre = pre_hi - pre_lo;
        if (o.precondition == PCX_PRECOND_INVERSE && npre > 0) {
            if (int rc = precondition_inverse<R>(B, npre)) return rc;
        }
        return PCX_OK;
    }

    void read_residuals() {
        resid.resize(b);
        rabs.resize(b);
        for (int j = 0; j < b; ++j) {
            rabs[j] = std::sqrt(std::max(host_res[j], 0.0));
            resid[j] = rabs[j] / std::max(std::fabs(theta[j]), 1e-300);
        }
    }

    // residual norms of the b Ritz pairs, W <- prec (AX - X theta); with wg, also the Gram matrix
    // [X | W]^H W (2b x b) of the new W, under the same stream synchronisation
    template <typename R>
    int residuals(Blocks<R>& B, std::vector<zc>* wg = nullptr) {
        if (int rc = residuals_async<R>(B)) return rc;
        // [X | W]^H W as the right half of the Hermitian [X | W]^H [X | W]: the 2b columns are staged
        // once (the plain product would stage W twice)
        const ColSet XW = colset(B.X, b, B.W, b);
        int rc = wg ? gram_async<R>(XW, XW, true) : PCX_OK;
        if (!rc) rc = sync();
        if (rc) return rc;
        if (wg) {
            std::vector<zc> full;
            gram_read(2 * b, 2 * b, full, true);
            wg->resize((size_t)2 * b * b);
            for (int r = 0; r < 2 * b; ++r)
                std::copy(full.begin() + (size_t)r * 2 * b + b, full.begin() + (size_t)(r + 1) * 2 * b,
                          wg->begin() + (size_t)r * b);
        }
        read_residuals();
        return PCX_OK;
    }

    // Rayleigh-Ritz on the b columns of X alone (start of a phase)
    template <typename R>
    int rr_block(Blocks<R>& B) {
        std::vector<zc> G, GA((size_t)b * b), GB((size_t)b * b);
        int rc = gram<R>(colset(B.X, b), colset(B.X, b, B.AX, b), G, true);   // X^H [X | AX]
        if (rc) return rc;
        for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c) {
                GB[(size_t)r * b + c] = G[(size_t)r * 2 * b + c];
                GA[(size_t)r * b + c] = G[(size_t)r * 2 * b + b + c];
            }
        std::vector<zc> C;
        if (!rayleigh_ritz(b, GA, GB, b, 1e-14, theta, C)) return fail(PCX_E_NOCONV, "pcx_solve: start block is singular");
        if ((rc = combine2<R>(colset(B.X, b), colset(B.T1, b), colset(B.AX, b), colset(B.T2, b), C))) return rc;
        std::swap(B.X, B.T1);
        std::swap(B.AX, B.T2);
        return PCX_OK;
    }

    // one phase of LOBPCG at precision R, starting from the b columns in B.X.  ortho_passes:
    // Cholesky-QR passes over the start block before its Rayleigh-Ritz step; none for the FP32
    // phase's Ritz vectors (orthonormal to FP32 rounding, so the Rayleigh-Ritz step's unit-scaled
    // Cholesky of their Gram matrix is well conditioned and leaves them orthonormal in FP64)
    template <typename R>
    int phase(Blocks<R>& B, double tol, int max_iter, int& iters, bool refine_after, int ortho_passes = 2) {
        int rc;
        hipError_t e = launch_mask<R>(B.X, prec, n, b, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: mask");
        for (int pass = 0; pass < ortho_passes; ++pass)
            if ((rc = orthonormalize<R>(B.X, B.T1, b))) return rc;
        if ((rc = matvec<R>(B.X, B.AX, b))) return rc;
        if ((rc = rr_block<R>(B))) return rc;
        pre_lo = 0;
        pre_hi = b;
        int np = 0;                       // columns of P (the previous active set)
        const double chol_tol = sizeof(R) == 8 ? kCholTol64 : kCholTol32;
        double best = 1e300;
        int stall = 0;
        std::vector<zc> G;                       // [X | W]^H W, (2b) x b
        // the convergence verdict on the residuals of the current X: 1 = leave the phase
        auto verdict = [&]() -> bool {
            bool all = true;
            double worst = 0;                    // over the bands still open
            int jw = -1;
            for (int j = 0; j < nev; ++j) {
                const bool cj = converged<R>(j, tol);
                all = all && cj;
                if (!cj && resid[j] >= worst) {
                    worst = resid[j];
                    jw = j;
                }
            }
            if (o.verbose) {
                int open = 0;
                for (int j = 0; j < b; ++j) open += !converged<R>(j, tol);
                fprintf(stderr, "pcx lobpcg %s it %d: theta0 %.12g worst residual %.3e (band %d), %d of %d columns open\n",
                        sizeof(R) == 8 ? "fp64" : "fp32", iters, theta[0], worst, jw, open, b);
            }
            if (all || iters >= max_iter) return true;
            // a reduced-precision phase ends when its residual stops improving (rounding floor)
            // and leaves at least half of the iterations to the refinement
            if (worst < 0.9 * best) {
                best = worst;
                stall = 0;
            } else if (++stall >= (sizeof(R) == 4 ? kFp32Stall : kFp64Stall) &&
                       (sizeof(R) == 8 || worst < 1e-2 || st.iterations_fp32 >= 40)) {
                // FP32: the rounding floor (or bands it cannot resolve at all, next to Gamma),
                // refinement follows; FP64: stagnation at the floor of a band the tolerance cannot
                // reach, stop before the basis loses orthogonality
                return true;
            }
            return sizeof(R) == 4 && refine_after && st.iterations_fp32 >= max_iter / 2;
        };
        // soft locking: only columns whose residual is above tol expand the basis
        auto open_columns = [&]() {
            std::vector<int> act;
            for (int j = 0; j < b; ++j)
                if (!converged<R>(j, tol)) act.push_back(j);
            return act;
        };
        // Rayleigh-Ritz on S = [X W P] (W: na columns at Wa); without P if the basis is too
        // ill-conditioned.  have_g: G already holds S^H [S | AS] of the basis with P.  Returns
        // false when it fails also without P.
        auto rayleigh_ritz_step = [&](cx<R>* Wa, int na, bool have_g, std::vector<zc>& GS, std::vector<double>& th,
                                      std::vector<zc>& C, bool& withP) -> int {
            withP = np > 0;
            for (;;) {
                const int k = b + na + (withP ? np : 0);
                const ColSet S = withP ? colset(B.X, b, Wa, na, B.P, np) : colset(B.X, b, Wa, na);
                const ColSet AS = withP ? colset(B.AX, b, B.AW, na, B.AP, np) : colset(B.AX, b, B.AW, na);
                if (!have_g)
                    if (int rc2 = gram<R>(S, concat(S, AS), GS, true)) return rc2;     // S^H [S | AS]
                have_g = false;
                std::vector<zc> GB((size_t)k * k), GA((size_t)k * k);
                for (int r = 0; r < k; ++r)
                    for (int c = 0; c < k; ++c) {
                        GB[(size_t)r * k + c] = GS[(size_t)r * 2 * k + c];
                        GA[(size_t)r * k + c] = GS[(size_t)r * 2 * k + k + c];
                    }
                // A_r is positive semi-definite: a negative Ritz value means the pencil is no longer
                // consistent (nearly dependent basis), handled like a failed factorisation
                if (rayleigh_ritz(k, GA, GB, b, chol_tol, th, C) && th[0] > -1e-8 * std::fabs(th[b - 1])) return PCX_OK;
                if (!withP) return 1;
                withP = false;
            }
        };
        // [X' | P'] = S [C | C_P], C_P = the columns act of C with the X rows zeroed
        auto update = [&](cx<R>* Wa, int na, bool withP, const std::vector<zc>& C,
                          const std::vector<int>& act) -> int {
            const int k = b + na + (withP ? np : 0);
            const int nn = (int)act.size();
            const int m = b + nn;
            std::vector<zc> C2((size_t)k * m, zc(0, 0));
            for (int r = 0; r < k; ++r) {
                for (int c = 0; c < b; ++c) C2[(size_t)r * m + c] = C[(size_t)r * b + c];
                if (r >= b)
                    for (int c = 0; c < nn; ++c) C2[(size_t)r * m + b + c] = C[(size_t)r * b + act[c]];
            }
            const ColSet S = withP ? colset(B.X, b, Wa, na, B.P, np) : colset(B.X, b, Wa, na);
            const ColSet AS = withP ? colset(B.AX, b, B.AW, na, B.AP, np) : colset(B.AX, b, B.AW, na);
            if (int rc2 = combine2<R>(S, colset(B.T1, b, B.T3, nn), AS, colset(B.T2, b, B.T4, nn), C2)) return rc2;
            std::swap(B.X, B.T1);
            std::swap(B.P, B.T3);
            std::swap(B.AX, B.T2);
            std::swap(B.AP, B.T4);
            np = nn;
            return PCX_OK;
        };
        // One stream synchronisation per iteration: the preconditioned residuals of the columns
        // open at the previous check, [pre_lo, pre_hi), enter the basis as they are (no
        // orthogonalisation against X; the Rayleigh-Ritz step scales the basis to unit columns),
        // their A_r product and the Gram matrix S^H [S | AS] are queued behind the residual kernel,
        // and the residual norms and the Gram matrix reach the host together.  Should the pencil
        // fail to factor also without P, the phase continues with two synchronisations per
        // iteration: W orthonormalised against X on the host first (throughout, on request).
        // At weak contrast (eps_max <= 2 eps_min) the approximate-inverse preconditioner is close to
        // the exact inverse, so the preconditioned residual of a nearly converged column lies
        // mostly in span X and the plain basis [X W P] is nearly dependent: there W is
        // orthonormalised against X in every iteration (vacuum hexagonal 6 x 6 x 8 at A: 78
        // iterations with it, 108 without, and no convergence under other rounding)
        bool two_sync = o.orthonormalize_w != 0 || p->eps_max <= 2.0 * p->eps_min;
        for (;;) {
            if (!two_sync) {
                if ((rc = residuals_async<R>(B))) return rc;
                const int na = pre_hi - pre_lo;
                cx<R>* Wa = B.W + (size_t)pre_lo * N;
                if ((rc = matvec<R>(Wa, B.AW, na))) return rc;
                std::vector<zc> GS;
                {
                    const ColSet S = np > 0 ? colset(B.X, b, Wa, na, B.P, np) : colset(B.X, b, Wa, na);
                    const ColSet AS = np > 0 ? colset(B.AX, b, B.AW, na, B.AP, np) : colset(B.AX, b, B.AW, na);
                    if ((rc = gram<R>(S, concat(S, AS), GS, true))) return rc;
                }
                read_residuals();
                if (verdict()) return PCX_OK;
                std::vector<double> th;
                std::vector<zc> C;
                bool withP = false;
                rc = rayleigh_ritz_step(Wa, na, true, GS, th, C, withP);
                if (rc < 0) return rc;
                if (rc > 0) {           // the unorthogonalised basis is too ill-conditioned
                    if (o.verbose) fprintf(stderr, "pcx lobpcg: plain basis singular, W orthonormalised from here on\n");
                    ++st.orth_fallbacks;
                    two_sync = true;
                    continue;
                }
                ++iters;
                ++st.iterations;
                if (sizeof(R) == 4) ++st.iterations_fp32;
                const std::vector<int> act = open_columns();
                if ((rc = update(Wa, na, withP, C, act))) return rc;
                theta = th;
                pre_lo = act.empty() ? 0 : act.front();
                pre_hi = act.empty() ? 0 : act.back() + 1;
                continue;
            }
            if ((rc = residuals<R>(B, &G))) return rc;   // W <- prec (AX - X theta) for all b columns
            if (verdict()) return PCX_OK;
            ++iters;
            ++st.iterations;
            if (sizeof(R) == 4) ++st.iterations_fp32;
            const std::vector<int> act = open_columns();
            const int na = (int)act.size();
            pre_lo = na ? act.front() : 0;
            pre_hi = na ? act.back() + 1 : 0;
            // W_act <- (W_act - X G) R^{-1} with one Gram product and one combination:
            // [X | W]^H W (taken with the residuals) gives G = X^H W_act and W_act^H W_act, and the
            // projected Gram matrix W_act^H W_act - G^H G (X has orthonormal columns) gives R
            // (Cholesky-QR, SVQB fallback)
            {
                std::vector<zc> M((size_t)na * na), Cw;
                for (int r = 0; r < na; ++r)
                    for (int c = 0; c < na; ++c) {
                        zc v = G[(size_t)(b + act[r]) * b + act[c]];
                        for (int q = 0; q < b; ++q)
                            v -= std::conj(G[(size_t)q * b + act[r]]) * G[(size_t)q * b + act[c]];
                        M[(size_t)r * na + c] = v;
                    }
                orthonormalizer(na, M, Cw);
                std::vector<zc> C((size_t)(2 * b) * na, zc(0, 0));
                for (int c = 0; c < na; ++c)
                    for (int r = 0; r < na; ++r) {
                        const zc w = Cw[(size_t)r * na + c];
                        C[(size_t)(b + act[r]) * na + c] = w;
                        for (int q = 0; q < b; ++q) C[(size_t)q * na + c] -= G[(size_t)q * b + act[r]] * w;
                    }
                if ((rc = combine<R>(colset(B.X, b, B.W, b), C, colset(B.T1, na)))) return rc;
                std::swap(B.W, B.T1);
            }
            if ((rc = matvec<R>(B.W, B.AW, na))) return rc;
            std::vector<double> th;
            std::vector<zc> C, GS;
            bool withP = false;
            rc = rayleigh_ritz_step(B.W, na, false, GS, th, C, withP);
            if (rc < 0) return rc;
            if (rc > 0) return fail(PCX_E_NOCONV, "pcx_solve: Rayleigh-Ritz basis became singular");
            if ((rc = update(B.W, na, withP, C, act))) return rc;
            theta = th;
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

namespace pcx {

int gram_chunks_for(long N) { return (int)std::min<long>(1024, std::max<long>(1, N / 512)); }

// Grows the plan's eigensolver storage for a block of b columns: the LOBPCG blocks (ten b-column
// blocks per precision), the Gram partial sums and residual partials, the small device area (Gram
// output, coefficient slots, theta, residuals), the pinned host staging and Lambda_q^{-1}.
int solver_reserve(Plan* p, int b, bool use32, bool use64) {
    const long n = p->n, N = 2 * n;
    const size_t bytes64 = use64 ? 10 * (size_t)b * N * sizeof(cx<double>) : 0;
    const size_t bytes32 = use32 ? 10 * (size_t)b * N * sizeof(cx<float>) : 0;
    int rc;
    if ((rc = p->grow(&p->lob_mem, &p->lob_cap, bytes64 + bytes32))) return rc;
    if ((rc = p->grow(&p->prec, &p->prec_cap, n * sizeof(double)))) return rc;
    const int chunks = gram_chunks_for(N);
    const size_t gp = (size_t)(chunks + 32) * (3 * b) * (6 * b) * sizeof(cx<double>);
    const size_t rp = (size_t)chunks * b * sizeof(double);
    if ((rc = p->grow(&p->gram_part, &p->gram_part_cap, gp + rp))) return rc;
    const size_t gram_out = (size_t)(3 * b) * (6 * b) * sizeof(cx<double>);
    const size_t slots = Solver::kSlots * (size_t)(3 * b) * (2 * b) * sizeof(cx<double>);
    const size_t small = gram_out + slots + 2 * b * sizeof(double) + 1024;
    if ((rc = p->grow(&p->small_mem, &p->small_cap, std::max<size_t>(small, 1 << 16)))) return rc;
    const size_t pinned_bytes = slots + gram_out + 2 * b * sizeof(double);
    if (p->pinned_cap < pinned_bytes) {
        if (p->pinned) (void)hipHostFree(p->pinned);
        p->pinned = nullptr;
        p->pinned_cap = 0;
        hipError_t e = hipHostMalloc(&p->pinned, pinned_bytes, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve: pinned staging");
        p->pinned_cap = pinned_bytes;
    }
    return PCX_OK;
}

// The block size pcx_solve chooses for nev bands at most (the near-Gamma guard is the larger one,
// and a block ending inside a cluster of Lambda_q grows by up to 16 columns).
int solver_max_block(int nev, const pcx_opts* o) {
    if (o && o->block > 0) return o->block;
    return nev + std::max(4, (nev + 1) / 2) + 16;
}

}  // namespace pcx

extern "C" void pcx_opts_default(pcx_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = PCX_MODE_FP64;
    o->block = 0;
    o->max_iter = 400;
    o->tol = 1e-9;
    o->tol_fp32 = 1e-3;
    o->seed = 12345;
    o->precondition = PCX_PRECOND_INVERSE;
    o->verbose = 0;
    o->y0 = nullptr;
    o->n_y0 = 0;
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
    // Lambda_q^{-1} per mode (the preconditioner), also on the host for the start block
    int rc0 = p->grow(&p->prec, &p->prec_cap, n * sizeof(double));
    if (rc0) return rc0;
    {
        Grid g0;
        if ((rc0 = p->grid_for(kappa, &g0))) return rc0;
        hipError_t e0 = launch_precond_diag(g0, p->tables, (double*)p->prec, p->stream);
        if (e0 != hipSuccess) return hip_fail(e0, "pcx_solve: preconditioner");
    }
    std::vector<double> hp(n);
    if (hipMemcpyAsync(hp.data(), p->prec, n * sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return fail(PCX_E_DEVICE, "pcx_solve: preconditioner copy");
    std::vector<long> modes(n);
    for (long q = 0; q < n; ++q) modes[q] = q;
    const long nsort = std::min<long>(n, PCX_MAX_BLOCK);
    std::partial_sort(modes.begin(), modes.begin() + nsort, modes.end(), [&](long a, long c) { return hp[a] > hp[c]; });
    // Block guard: small (the dense block work grows as the square of the block; at 64^3 with 10
    // bands block 12 solves in 0.72x the time of block 15), except next to Gamma, where one plane
    // wave has Lambda_q far below the others (its two bands go to zero) and the small guard
    // stalls above the tolerance: there the larger guard.
    int guard = std::max(2, (nev + 4) / 5);
    {
        const long ref = std::min<long>(nsort - 1, std::max<long>(1, (nev + 1) / 2));
        if (hp[modes[0]] > 0 && hp[modes[ref]] > 0 && hp[modes[0]] > 10.0 * hp[modes[ref]]) {
            guard = std::max(4, (nev + 1) / 2);
            S.near_gamma = true;
        }
    }
    int b = S.o.block > 0 ? S.o.block : nev + guard;
    if (S.o.block <= 0) {
        // The block's last column must not fall inside a cluster of eigenvalues: LOBPCG converges a
        // wanted band at the rate set by the gap between it and the first eigenvalue outside the
        // block, so a block edge inside a (near-)degenerate cluster next to the wanted bands stalls
        // them (vacuum BCC 6^3 at Gamma, bands 4..7 at 73.267 next to eight at 73.292: 400
        // iterations without converging at block 10, 10 iterations at block 24).  The clusters of the
        // homogeneous medium are those of Lambda_q (each plane wave twice): for weak contrast
        // (eps_max <= 2 eps_min), extend the block until the first plane wave outside it lies 5% above
        // the last one inside, by at most 16 columns (with 1%, a vacuum cubic 6^3 problem whose
        // block ended 3% below the next plane wave kept two bands open after 108 iterations under
        // a different rounding of the Rayleigh-Ritz step); at higher contrast the clusters of Lambda_q
        // split and the extension only costs time (the 510-problem gyroid figure, eps 3..30: 35.5 s
        // instead of 31 s), so there the block only avoids separating the two polarisations of one
        // plane wave.
        const bool weak = p->eps_max <= 2.0 * p->eps_min;
        long cap = std::min<long>({(long)p->max_vectors, (long)PCX_MAX_BLOCK, (N - 2) / 3,
                                   (long)b + (weak ? 16 : (b % 2)), 2 * nsort - 1});
        if (p->block_cap > 0) cap = std::min<long>(cap, p->block_cap);
        while (b < cap) {
            const double in = hp[modes[(b - 1) / 2]], out = hp[modes[b / 2]];   // 1 / Lambda_q
            if (out <= 0.0 || in <= 0.0 || in >= (weak ? 1.05 : 1.01) * out) break;
            ++b;
        }
    }
    if (b < nev) return fail(PCX_E_ARG, "pcx_solve: block (%d) smaller than nev (%d)", b, nev);
    if (b > PCX_MAX_BLOCK || 3L * b > N - 2) return fail(PCX_E_ARG, "pcx_solve: block %d too large for this grid", b);
    if (S.o.mode < PCX_MODE_FP64 || S.o.mode > PCX_MODE_FP32) return fail(PCX_E_ARG, "pcx_solve: bad mode");
    if (S.o.precondition < PCX_PRECOND_NONE || S.o.precondition > PCX_PRECOND_INVERSE)
        return fail(PCX_E_ARG, "pcx_solve: bad preconditioner %d", S.o.precondition);
    if (S.o.orthonormalize_w != 0 && S.o.orthonormalize_w != 1)
        return fail(PCX_E_ARG, "pcx_solve: orthonormalize_w must be 0 or 1");
    if (!(S.o.tol > 0) || S.o.max_iter < 1) return fail(PCX_E_ARG, "pcx_solve: bad tolerance or max_iter");
    if (b > p->max_vectors) return fail(PCX_E_ARG, "pcx_solve: block %d exceeds the plan's max_vectors", b);
    if (S.o.n_y0 < 0 || S.o.n_y0 > b || (S.o.n_y0 > 0 && !S.o.y0))
        return fail(PCX_E_ARG, "pcx_solve: warm start needs 0 <= n_y0 <= block (%d) and y0", b);
    S.nev = nev;
    S.b = b;
    const bool use32 = S.o.mode != PCX_MODE_FP64;
    const bool use64 = S.o.mode != PCX_MODE_FP32;
    int rc;
    if (use64 && (rc = p->check_fits(PCX_FP64))) return rc;
    if (use32 && (rc = p->check_fits(PCX_FP32))) return rc;

    // the autotuner's kernel choice for this grid (once per process and grid; plans with an explicit
    // variant keep it); the FP32 kernels also serve the FP64 phase's preconditioner
    if (use32 || S.o.precondition == PCX_PRECOND_INVERSE) autotune_default(p, kappa, PCX_FP32, b);
    if (use64) autotune_default(p, kappa, PCX_FP64, b);
    if ((rc = solver_reserve(p, b, use32, use64))) return rc;
    const size_t bytes64 = use64 ? 10 * (size_t)b * N * sizeof(cx<double>) : 0;
    S.gram_chunks = gram_chunks_for(N);
    const size_t gp = (size_t)(S.gram_chunks + 32) * (3 * b) * (6 * b) * sizeof(cx<double>);
    const size_t gram_out = (size_t)(3 * b) * (6 * b) * sizeof(cx<double>);
    S.slot_elems = (size_t)(3 * b) * (2 * b);
    const size_t slots = Solver::kSlots * S.slot_elems * sizeof(cx<double>);
    S.pinned = (zc*)p->pinned;
    S.host_gram = (zc*)((char*)p->pinned + slots);
    S.host_res = (double*)((char*)p->pinned + slots + gram_out) + b;
    S.prec = (double*)p->prec;
    S.gram_part = (cx<double>*)p->gram_part;
    S.res_part = (double*)((char*)p->gram_part + gp);
    S.dev_small = (cx<double>*)p->small_mem;
    S.dev_slots = (cx<double>*)((char*)p->small_mem + gram_out);
    {
        // the pinned block is mapped into the device's address space (hipHostMalloc)
        char* pin_dev = nullptr;
        if (hipHostGetDevicePointer((void**)&pin_dev, p->pinned, 0) != hipSuccess || !pin_dev)
            return fail(PCX_E_DEVICE, "pcx_solve: pinned staging is not mapped on the device");
        S.gram_map = (cx<double>*)(pin_dev + ((char*)S.host_gram - (char*)p->pinned));
        S.res_map = (double*)(pin_dev + ((char*)S.host_res - (char*)p->pinned));
    }
    (void)hipEventCreate(&S.ev0);
    (void)hipEventCreate(&S.ev1);

    hipError_t e = hipSuccess;
    Blocks<double> B64{};
    Blocks<float> B32{};
    if (use64) B64 = carve<double>(p->lob_mem, b, N);
    if (use32) B32 = carve<float>((char*)p->lob_mem + bytes64, b, N);
    // start block: the plane waves of the smallest Lambda_q (the homogeneous-medium eigenvectors,
    // both polarisations) plus a small seeded random perturbation
    const long nm = std::min<long>(n, (b + 1) / 2);
    {
        double dmin = 0;                  // smallest nonzero 1 / Lambda_q
        for (long q = 0; q < n; ++q)
            if (hp[q] > 0 && (dmin == 0 || hp[q] < dmin)) dmin = hp[q];
        S.anorm = dmin > 0 ? 1.0 / (dmin * p->eps_min) : 0.0;
    }
    // start block, with the caller's vectors y0 in its first columns when `warm`
    auto seed_block = [&](auto* X, bool warm) -> int {
        using C = typename std::remove_pointer<decltype(X)>::type;
        hipError_t e2 = launch_random(X, (long)b * N, S.o.seed, 1e-3, p->stream);
        if (e2 != hipSuccess) return hip_fail(e2, "pcx_solve: random start");
        // unit entries of the plane waves, written by a kernel (indices passed by value)
        UnitList units;
        units.count = b;
        for (int c = 0; c < b; ++c) units.idx[c] = (long long)c * N + (c % 2) * n + modes[(c / 2) % nm];
        e2 = launch_set_units(X, units, p->stream);
        if (e2 != hipSuccess) return hip_fail(e2, "pcx_solve: start block");
        if (warm && S.o.n_y0 > 0) {
            const long cnt = (long)S.o.n_y0 * N;
            if (std::is_same<C, cx<double>>::value)
                e2 = hipMemcpyAsync((void*)X, S.o.y0, cnt * sizeof(cx<double>), hipMemcpyDeviceToDevice, p->stream);
            else
                e2 = launch_convert((const cx<double>*)S.o.y0, (cx<float>*)(void*)X, cnt, p->stream);
            if (e2 != hipSuccess) return hip_fail(e2, "pcx_solve: warm start");
        }
        return S.sync();
    };
    int iters = 0;
    rc = PCX_OK;
    if (use32) {
        rc = seed_block(B32.X, true);
        const double tol32 = S.o.mode == PCX_MODE_FP32 ? S.o.tol : std::max(S.o.tol, S.o.tol_fp32);
        if (!rc) rc = S.phase<float>(B32, tol32, S.o.max_iter, iters, use64);
        if (!rc && use64) {
            e = launch_convert(B32.X, B64.X, (long)b * N, p->stream);
            if (e != hipSuccess) rc = hip_fail(e, "pcx_solve: convert");
        }
    } else {
        rc = seed_block(B64.X, true);
    }
    if (!rc && use64) rc = S.phase<double>(B64, S.o.tol, S.o.max_iter, iters, false, use32 ? 0 : 2);
    if (!rc && use64 && (use32 || S.o.n_y0 > 0) && iters < S.o.max_iter) {
        // an FP64 phase that stopped on stagnation with bands open, after an FP32 phase or from
        // the caller's vectors, is solved again in FP64 alone from the plain start block (seen
        // next to Gamma at high contrast, FP32+refine: started from the FP32 block, the near-zero
        // bands' residuals first fall to ~1e-7 and then climb back; SC sphere at Gamma started
        // from the eigenvectors of the neighbouring path point: the residuals reach 2.5e-10, then
        // climb back to 1e-4 and stall); at most once, within the same iteration budget
        bool open = false;
        for (int j = 0; j < nev; ++j) open = open || !S.converged<double>(j, S.o.tol, true);
        if (open) {
            ++S.st.restarts;
            rc = seed_block(B64.X, false);
            if (!rc) rc = S.phase<double>(B64, S.o.tol, S.o.max_iter, iters, false);
        }
    }
    if (!rc) {
        for (int j = 0; j < nev; ++j) lambda[j] = S.theta[j];
        int conv = 0;
        for (int j = 0; j < nev; ++j) {
            if (j < PCX_MAX_BLOCK) S.st.residual[j] = S.resid[j];
            if (use64 ? S.converged<double>(j, S.o.tol, true) : S.converged<float>(j, S.o.tol, true)) {
                ++conv;
                if (S.resid[j] > S.o.tol) S.st.floor_mask |= 1ull << j;
            }
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
