// The paper's own eigen-driver (Section 5.2): inverse Lanczos on the nullspace-free operator with
// conjugate-gradient inner solves, on the same A_r kernels as the LOBPCG solver.
//
// A_r = Sigma_r M Sigma_r with M = Q_r^* B^{-1} Q_r, so A_r^{-1} = Sigma_r^{-1} M^{-1} Sigma_r^{-1}.
// M is Hermitian positive definite on the modes with Lambda_q > 0 with condition number at most
// eps_max / eps_min (the bound of Section 5.2), which is why the paper runs CG on it without a
// preconditioner.  A product with M is the A_r kernels between two Lambda_q^{-1/2} scalings.
// Lanczos runs on A_r^{-1} from one seeded start vector with full reorthogonalisation (classical
// Gram-Schmidt twice per step); the largest Ritz values theta of the tridiagonal matrix give the
// smallest eigenvalues lambda = 1 / theta of A_r.  Everything is FP64; the reorthogonalisation
// uses the Gram and combination kernels of the block solver, CG a two-stage inner-product kernel
// and small axpby kernels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "pcx_dense.h"
#include "pcx_host.h"

using namespace pcx;

namespace {

struct Lanczos {
    Plan* p = nullptr;
    const double* kappa = nullptr;
    long n = 0, N = 0;
    hipStream_t st = nullptr;
    pcx_lanczos_opts o{};
    pcx_lanczos_stats stats{};
    void* mem = nullptr;
    cx<double>* V = nullptr;                 // (max_steps + 1) basis columns
    cx<double> *x = nullptr, *r = nullptr, *pp = nullptr, *q = nullptr, *tmp = nullptr, *w = nullptr, *rhs = nullptr;
    double* sqd = nullptr;                   // Lambda_q^{-1/2} per mode (0 on the masked mode)
    double* prec = nullptr;                  // Lambda_q^{-1}
    cx<double>* part = nullptr;              // Gram or inner-product partial sums
    cx<double>* small = nullptr;             // Gram output, then coefficient columns
    int chunks = 0;

    ~Lanczos() {
        if (mem) (void)hipFree(mem);
    }

    int sync() {
        hipError_t e = hipStreamSynchronize(st);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve_lanczos: stream");
    }

    // A^H b for the columns of A (ka of them) against one vector b, to the host
    int gram(const ColSet& A, const cx<double>* b, std::vector<zc>& out) {
        const int ka = A.total();
        hipError_t e = launch_gram<double>(A, colset(const_cast<cx<double>*>(b), 1), N, part, chunks, small, st, false);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: gram");
        out.resize(ka);
        e = hipMemcpyAsync(out.data(), small, sizeof(zc) * ka, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: gram copy");
        return sync();
    }

    int dot(const cx<double>* a, const cx<double>* b, zc* out) {
        hipError_t e = launch_dot(a, b, N, part, small, st);
        if (e == hipSuccess) e = hipMemcpyAsync(out, small, sizeof(zc), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: inner product");
        return sync();
    }

    int axpby(const cx<double>* xv, cx<double>* yv, zc a, zc b) {
        cx<double> ca, cb;
        ca.x = a.real();
        ca.y = a.imag();
        cb.x = b.real();
        cb.y = b.imag();
        hipError_t e = launch_axpby(xv, yv, ca, cb, N, st);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve_lanczos: axpby");
    }

    // out = M in = Lambda_q^{-1/2} A_r Lambda_q^{-1/2} in
    int mprod(const cx<double>* in, cx<double>* out) {
        hipError_t e = launch_scale_modes<double>(in, tmp, sqd, n, 1, st);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: scaling");
        int rc = p->apply(Plan::OP_AR, kappa, PCX_FP64, tmp, out, 1);
        if (rc) return rc;
        e = launch_scale_modes<double>(out, out, sqd, n, 1, st);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_solve_lanczos: scaling");
    }

    // x = M^{-1} c by CG from x = 0 (c in rhs)
    int cg() {
        hipError_t e = hipMemsetAsync(x, 0, sizeof(cx<double>) * N, st);
        if (e == hipSuccess) e = hipMemcpyAsync(r, rhs, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(pp, rhs, sizeof(cx<double>) * N, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: CG start");
        zc rr;
        int rc = dot(r, r, &rr);
        if (rc) return rc;
        const double cnorm = std::sqrt(std::max(rr.real(), 0.0));
        if (cnorm == 0.0) return PCX_OK;
        double rho = rr.real();
        for (int it = 0; it < o.max_cg; ++it) {
            if ((rc = mprod(pp, q))) return rc;
            ++stats.cg_iterations;
            ++stats.matvecs;
            zc pq;
            if ((rc = dot(pp, q, &pq))) return rc;
            if (!(pq.real() > 0.0)) return fail(PCX_E_NOCONV, "pcx_solve_lanczos: CG lost positive definiteness");
            const double alpha = rho / pq.real();
            if ((rc = axpby(pp, x, alpha, 1.0))) return rc;
            if ((rc = axpby(q, r, -alpha, 1.0))) return rc;
            zc rn;
            if ((rc = dot(r, r, &rn))) return rc;
            const double rho1 = rn.real();
            if (std::sqrt(std::max(rho1, 0.0)) <= o.tol_inner * cnorm) return PCX_OK;
            if ((rc = axpby(r, pp, 1.0, rho1 / rho))) return rc;      // p = r + (rho1 / rho) p
            rho = rho1;
        }
        return PCX_OK;      // the outer residual estimate judges the result
    }

    // w -= V[0..m) (V[0..m)^H w), the coefficients returned in h
    int project(int m, std::vector<zc>& h) {
        int rc = gram(colset(V, m), w, h);
        if (rc) return rc;
        std::vector<zc> C(m + 1);
        for (int i = 0; i < m; ++i) C[i] = -h[i];
        C[m] = 1.0;
        cx<double>* dc = small + (m + 1);
        hipError_t e = hipMemcpyAsync(dc, C.data(), sizeof(zc) * (m + 1), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = launch_combine<double>(colset(V, m, w, 1), dc, colset(w, 1), N, st);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: reorthogonalisation");
        return sync();      // the pageable coefficient copy must not be overwritten early
    }
};

}  // namespace

extern "C" void pcx_lanczos_opts_default(pcx_lanczos_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol_outer = 1e-12;
    o->tol_inner = 1e-13;
    o->max_steps = 200;
    o->max_cg = 2000;
    o->seed = 4242;
}

extern "C" int pcx_solve_lanczos(pcx_plan* pp, const double kappa[3], int nev, const pcx_lanczos_opts* opts,
                                 double* lambda, pcx_lanczos_stats* stats_out) {
    const auto t0 = std::chrono::steady_clock::now();
    Plan* p = (Plan*)pp;
    if (!p || !kappa || !lambda) return fail(PCX_E_ARG, "pcx_solve_lanczos: null pointer");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_solve_lanczos: permittivity not set");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "pcx_solve_lanczos: non-finite kappa");
    Lanczos L;
    if (opts) L.o = *opts;
    else pcx_lanczos_opts_default(&L.o);
    const long n = p->n, N = 2 * n;
    if (nev < 1 || nev > PCX_MAX_BLOCK) return fail(PCX_E_ARG, "pcx_solve_lanczos: nev outside [1, %d]", PCX_MAX_BLOCK);
    if (L.o.max_steps < nev + 1 || L.o.max_steps > N - 2 || L.o.max_cg < 1 || !(L.o.tol_outer > 0) ||
        !(L.o.tol_inner > 0))
        return fail(PCX_E_ARG, "pcx_solve_lanczos: bad options");
    int rc = p->check_fits(PCX_FP64);
    if (rc) return rc;
    L.p = p;
    L.kappa = kappa;
    L.n = n;
    L.N = N;
    L.st = p->stream;
    const int ms = L.o.max_steps;
    L.chunks = (int)std::min<long>(1024, std::max<long>(1, N / 512));
    const size_t vec = sizeof(cx<double>) * (size_t)N;
    // partial sums: the Gram product's (chunks + 32) (ms + 2), at least the inner product's 1024
    const size_t nparts = std::max<size_t>((size_t)(L.chunks + 32) * (ms + 2), 1024);
    const size_t bytes = vec * ((size_t)ms + 1 + 7) + 2 * sizeof(double) * (size_t)n +
                         sizeof(cx<double>) * (nparts + 2 * (size_t)(ms + 2)) + 1024;
    hipError_t e = hipMalloc(&L.mem, bytes);
    if (e != hipSuccess) {
        L.mem = nullptr;
        return fail(PCX_E_OOM, "pcx_solve_lanczos: %zu bytes of workspace", bytes);
    }
    char* q = (char*)L.mem;
    L.V = (cx<double>*)q;
    q += vec * ((size_t)ms + 1);
    cx<double>** vs[] = {&L.x, &L.r, &L.pp, &L.q, &L.tmp, &L.w, &L.rhs};
    for (auto v : vs) {
        *v = (cx<double>*)q;
        q += vec;
    }
    L.sqd = (double*)q;
    L.prec = L.sqd + n;
    q += 2 * sizeof(double) * (size_t)n;
    L.part = (cx<double>*)q;
    q += sizeof(cx<double>) * nparts;
    L.small = (cx<double>*)q;

    Grid g;
    if ((rc = p->grid_for(kappa, &g))) return rc;
    e = launch_precond_diag(g, p->tables, L.prec, L.st);
    if (e == hipSuccess) e = launch_sqrt(L.prec, L.sqd, n, L.st);
    // start vector: seeded, zero on the masked mode, unit norm
    if (e == hipSuccess) e = launch_random<double>(L.V, N, L.o.seed, 1.0, L.st);
    if (e == hipSuccess) e = launch_mask<double>(L.V, L.prec, n, 1, L.st);
    if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: start");
    zc nn;
    if ((rc = L.dot(L.V, L.V, &nn))) return rc;
    if (!(nn.real() > 0)) return fail(PCX_E_ARG, "pcx_solve_lanczos: empty search space");
    if ((rc = L.axpby(L.V, L.V, 0.0, 1.0 / std::sqrt(nn.real())))) return rc;

    std::vector<double> alpha, beta;
    std::vector<double> theta;
    std::vector<double> res(nev, 1.0);
    bool done = false;
    int m = 0;
    for (int j = 0; j < ms && !done; ++j) {
        cx<double>* vj = L.V + (size_t)j * N;
        e = launch_scale_modes<double>(vj, L.rhs, L.sqd, n, 1, L.st);          // Sigma_r^{-1} v
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: scaling");
        if ((rc = L.cg())) return rc;                                           // M^{-1} Sigma_r^{-1} v
        e = launch_scale_modes<double>(L.x, L.w, L.sqd, n, 1, L.st);           // w = A_r^{-1} v
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_lanczos: scaling");
        std::vector<zc> h;
        if ((rc = L.project(j + 1, h))) return rc;
        alpha.push_back(h[j].real());
        if ((rc = L.project(j + 1, h))) return rc;
        zc ww;
        if ((rc = L.dot(L.w, L.w, &ww))) return rc;
        const double b = std::sqrt(std::max(ww.real(), 0.0));
        beta.push_back(b);
        m = j + 1;
        L.stats.steps = m;
        if (m >= nev) {
            // Ritz pairs of the tridiagonal matrix: the nev largest theta (lowest of -T)
            std::vector<zc> T((size_t)m * m, zc(0, 0));
            for (int i = 0; i < m; ++i) {
                T[(size_t)i * m + i] = -alpha[i];
                if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = -beta[i];
            }
            std::vector<double> ev;
            std::vector<zc> S;
            if (!herm_eig(m, T, ev, S, nev)) return fail(PCX_E_NOCONV, "pcx_solve_lanczos: tridiagonal eigen-solve");
            theta.assign(nev, 0.0);
            bool all = true;
            for (int i = 0; i < nev; ++i) {
                theta[i] = -ev[i];
                res[i] = b * std::abs(S[(size_t)(m - 1) * nev + i]) / std::max(std::fabs(theta[i]), 1e-300);
                all = all && theta[i] > 0 && res[i] <= L.o.tol_outer;
            }
            done = all;
        }
        if (b == 0.0) break;                                                   // invariant subspace
        if (!done && j + 1 < ms) {
            if ((rc = L.axpby(L.w, L.V + (size_t)(j + 1) * N, 1.0 / b, 0.0))) return rc;
        }
    }
    int conv = 0;
    for (int i = 0; i < nev; ++i) {
        lambda[i] = i < (int)theta.size() && theta[i] > 0 ? 1.0 / theta[i] : 0.0;
        if (i < PCX_MAX_BLOCK) L.stats.residual[i] = res[i];
        if (i < (int)theta.size() && theta[i] > 0 && res[i] <= L.o.tol_outer) ++conv;
    }
    L.stats.converged = conv;
    L.stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats_out) *stats_out = L.stats;
    if (conv < nev) return fail(PCX_E_NOCONV, "pcx_solve_lanczos: %d of %d converged after %d steps", conv, nev, m);
    return PCX_OK;
}
