// Host side of the C ABI: lattice geometry (Section 2.2), plans and the apply entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "pcx_host.h"

namespace pcx {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? PCX_E_OOM : PCX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- Section 2.2
// floor when the fractional part is below 1/2, ceil otherwise; arguments within 1e-9 of an
// integer are taken as that integer.
static long round_half_up(double x) {
    const double r = std::round(x);
    if (std::fabs(x - r) < 1e-9) return (long)r;
    const double f = std::floor(x);
    return (x - f) < 0.5 ? (long)f : (long)std::ceil(x);
}

static bool smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

bool make_fft_plan(int n, FftPlan* fp) {
    if (!smooth235(n) || n > PCX_MAX_N) return false;
    fp->n = n;
    fp->npass = 0;
    int m = n;
    while (m % 8 == 0) { fp->rad[fp->npass++] = 8; m /= 8; }
    while (m % 4 == 0) { fp->rad[fp->npass++] = 4; m /= 4; }
    while (m % 2 == 0) { fp->rad[fp->npass++] = 2; m /= 2; }
    while (m % 3 == 0) { fp->rad[fp->npass++] = 3; m /= 3; }
    while (m % 5 == 0) { fp->rad[fp->npass++] = 5; m /= 5; }
    return fp->npass <= kMaxPasses;
}

static double col_norm(const double* a, int c) {
    return std::sqrt(a[0 * 3 + c] * a[0 * 3 + c] + a[1 * 3 + c] * a[1 * 3 + c] + a[2 * 3 + c] * a[2 * 3 + c]);
}
static double col_dot(const double* a, int c, int d) {
    return a[0 * 3 + c] * a[0 * 3 + d] + a[1 * 3 + c] * a[1 * 3 + d] + a[2 * 3 + c] * a[2 * 3 + d];
}

}  // namespace pcx

using namespace pcx;

extern "C" const char* pcx_last_error(void) { return g_err.c_str(); }

extern "C" int pcx_geometry(const double avec[9], int n1, int n2, int n3, pcx_geom* out) {
    if (!avec || !out) return fail(PCX_E_ARG, "pcx_geometry: null pointer");
    if (n1 < 1 || n2 < 1 || n3 < 1) return fail(PCX_E_ARG, "pcx_geometry: grid sizes must be positive");
    for (int n : {n1, n2, n3})
        if (!smooth235(n) || n > PCX_MAX_N)
            return fail(PCX_E_SIZE, "pcx_geometry: grid size %d is not a product of 2, 3, 5 up to %d", n, PCX_MAX_N);
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(avec[i])) return fail(PCX_E_ARG, "pcx_geometry: non-finite lattice vector");
    const double L1 = col_norm(avec, 0), L2 = col_norm(avec, 1), L3 = col_norm(avec, 2);
    if (!(L1 > 0 && L2 > 0 && L3 > 0)) return fail(PCX_E_LATTICE, "pcx_geometry: zero lattice vector");
    const double det = avec[0] * (avec[4] * avec[8] - avec[5] * avec[7]) -
                       avec[1] * (avec[3] * avec[8] - avec[5] * avec[6]) +
                       avec[2] * (avec[3] * avec[7] - avec[4] * avec[6]);
    if (std::fabs(det) < 1e-12 * L1 * L2 * L3)
        return fail(PCX_E_LATTICE, "pcx_geometry: lattice vectors are linearly dependent");
    const double cgp = col_dot(avec, 0, 1) / (L1 * L2);
    const double cbp = col_dot(avec, 0, 2) / (L1 * L3);
    const double cap = col_dot(avec, 1, 2) / (L2 * L3);
    const double dx = L1 / n1;
    long m1, m2, m3;
    int r1, r2, r3;
    double cg, cb, ca;
    if (cgp >= 0.0) {
        r1 = 0;
        m1 = round_half_up(L2 * cgp / dx);
        cg = m1 * dx / L2;
    } else {
        r1 = 1;
        m1 = round_half_up((L1 + L2 * cgp) / dx);
        cg = (m1 * dx - L1) / L2;
    }
    if (std::fabs(cg) >= 1.0) return fail(PCX_E_LATTICE, "pcx_geometry: a2 does not fit in the cell along x");
    const double sg = std::sqrt(1.0 - cg * cg);
    const double l2 = L2 * sg;
    const double dy = l2 / n2;
    if (cbp >= 0.0) {
        r2 = 0;
        m2 = round_half_up(L3 * cbp / dx);
        cb = m2 * dx / L3;
    } else {
        r2 = 1;
        m2 = round_half_up((L1 + L3 * cbp) / dx);
        cb = (m2 * dx - L1) / L3;
    }
    if (std::fabs(cb) > 1.0) return fail(PCX_E_LATTICE, "pcx_geometry: a3 does not fit in the cell along x");
    const double dp = cap - cg * cb;
    if (dp >= 0.0) {
        r3 = 0;
        m3 = round_half_up(L3 * dp / (dy * sg));
        ca = m3 * dy * sg / L3 + cg * cb;
    } else {
        r3 = 1;
        m3 = round_half_up((L2 * sg * sg + L3 * dp) / (dy * sg));
        ca = (m3 * dy * sg - L2 * sg * sg) / L3 + cg * cb;
    }
    if (!(0 <= m1 && m1 <= n1 && 0 <= m2 && m2 <= n1 && 0 <= m3 && m3 <= n2))
        return fail(PCX_E_LATTICE, "pcx_geometry: primitive-cell condition violated (m = %ld, %ld, %ld)", m1, m2, m3);
    const long s1 = m1 - (long)r1 * n1, s2 = m2 - (long)r2 * n1, s3 = m3 - (long)r3 * n2;
    if (std::labs(s3) >= n2) return fail(PCX_E_LATTICE, "pcx_geometry: a3 does not fit in the cell along y");
    const double disc = 1.0 - cg * cg - cb * cb - ca * ca + 2.0 * cg * cb * ca;
    if (!(disc > 0.0)) return fail(PCX_E_LATTICE, "pcx_geometry: corrected lattice is degenerate");
    const double l3 = L3 * std::sqrt(disc) / sg;
    pcx_geom g;
    std::memset(&g, 0, sizeof(g));
    g.n[0] = n1; g.n[1] = n2; g.n[2] = n3;
    g.m[0] = (int)m1; g.m[1] = (int)m2; g.m[2] = (int)m3;
    g.rho[0] = r1; g.rho[1] = r2; g.rho[2] = r3;
    g.shift[0] = (int)s1; g.shift[1] = (int)s2; g.shift[2] = (int)s3;
    g.delta[0] = dx; g.delta[1] = dy; g.delta[2] = l3 / n3;
    const double R[9] = {L1, L2 * cg, L3 * cb, 0.0, L2 * sg, L3 * (ca - cg * cb) / sg, 0.0, 0.0, l3};
    std::memcpy(g.avec_rot, R, sizeof(R));
    g.cos_angles[0] = cg; g.cos_angles[1] = cb; g.cos_angles[2] = ca;
    *out = g;
    return PCX_OK;
}

extern "C" int pcx_omega(const double avec[9], const pcx_geom* g, double omega[9]) {
    if (!avec || !g || !omega) return fail(PCX_E_ARG, "pcx_omega: null pointer");
    // [a]^{-T} = cof(A) / det(A) for A = g->avec_rot (row-major, columns the corrected vectors)
    const double* A = g->avec_rot;
    auto at = [&](int r, int c) { return A[3 * r + c]; };
    double cof[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            cof[3 * r + c] = at(r1, c1) * at(r2, c2) - at(r1, c2) * at(r2, c1);
        }
    const double det = at(0, 0) * cof[0] + at(0, 1) * cof[1] + at(0, 2) * cof[2];
    if (!(std::fabs(det) > 0) || !std::isfinite(det)) return fail(PCX_E_LATTICE, "pcx_omega: singular lattice");
    // Omega[r][c] = sum_m [a]^{-T}[r][m] [a~]^T[m][c] = sum_m cof[r][m] avec[c][m] / det
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += cof[3 * r + m] * avec[3 * c + m];
            omega[3 * r + c] = s / det;
        }
    return PCX_OK;
}

extern "C" int pcx_kappa_from_bloch(const double avec[9], const double kvec[3], double kappa[3]) {
    if (!avec || !kvec || !kappa) return fail(PCX_E_ARG, "pcx_kappa_from_bloch: null pointer");
    for (int l = 0; l < 3; ++l) {
        const double d = avec[0 * 3 + l] * kvec[0] + avec[1 * 3 + l] * kvec[1] + avec[2 * 3 + l] * kvec[2];
        kappa[l] = d / (2.0 * M_PI);
    }
    return PCX_OK;
}

// ---------------------------------------------------------------- plans

namespace pcx {

static void host_twiddles(int n, std::vector<cx<double>>& out) {
    out.resize(n);
    for (int m = 0; m < n; ++m) {
        // exp(2 pi i m / n) with the angle reduced to (-pi, pi]
        long mm = m;
        if (2 * mm > n) mm -= n;
        const double a = 2.0 * M_PI * (double)mm / (double)n;
        out[m].x = std::cos(a);
        out[m].y = std::sin(a);
    }
}

// kernel attributes (dynamic LDS limits) are set once per process, whichever thread creates the
// first plan (batch workers may create plans concurrently)
static std::once_flag g_config_once;
static hipError_t g_config_status = hipErrorNotReady;

static int ensure_configured() {
    std::call_once(g_config_once, [] {
        hipError_t e = configure_kernels();
        if (e == hipSuccess) e = configure_block_kernels();
        g_config_status = e;
    });
    if (g_config_status != hipSuccess) return hip_fail(g_config_status, "kernel configuration");
    return PCX_OK;
}

void Plan::set_eps_pointers() {
    inv_eps64 = eps_mem;
    inv_epsn64 = (double*)inv_eps64 + 3 * n;
    inv_eps32 = (double*)inv_epsn64 + 3 * n;
    inv_epsn32 = (float*)inv_eps32 + 3 * n;
    epsn64 = (float*)inv_epsn32 + 3 * n;
    epsn32 = (double*)epsn64 + 3 * n;
}

int Plan::grow(void** buf, size_t* have, size_t need) {
    if (*have >= need) return PCX_OK;
    if (*buf) (void)hipFree(*buf);
    *buf = nullptr;
    *have = 0;
    hipError_t e = hipMalloc(buf, need);
    if (e != hipSuccess) {
        *buf = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    *have = need;
    return PCX_OK;
}

Grid Plan::grid(const double kappa[3]) const {
    Grid g;
    g.n1 = geom.n[0];
    g.n2 = geom.n[1];
    g.n3 = geom.n[2];
    g.s1 = geom.shift[0];
    g.s2 = geom.shift[1];
    g.s3 = geom.shift[2];
    for (int l = 0; l < 3; ++l) {
        g.kap[l] = kappa[l];
        g.dlt[l] = geom.delta[l];
    }
    g.fx = fx;
    g.fy = fy;
    g.fz = fz;
    g.codes = (const unsigned char*)codes;
    for (int f = 0; f < 2; ++f) {
        g.generic[f] = (variant == PCX_VARIANT_GENERIC || tuned_nt[f] > 0) ? 1 : 0;
        g.plane_nt[f] = tuned_nt[f] > 0 ? tuned_nt[f] : 0;
        g.fixed_kind[f] = (tuned_nt[f] == -1 || variant == PCX_VARIANT_THREE_PLANE)
                              ? 3
                              : ((tuned_nt[f] == -2 || variant == PCX_VARIANT_TWO_PLANE)
                                     ? 2
                                     : ((tuned_nt[f] == -3 || variant == PCX_VARIANT_REGISTER) ? 4 : 0));
    }
    for (int f = 0; f < 2; ++f) g.split[f] = split_plane_needed(g.n2, g.n3, f) ? 1 : 0;
    g.nvk = 0;
    g.kaps = nullptr;
    g.wtab[0] = g.wtab[1] = nullptr;
    return g;
}

int Plan::grid_for(const double kappa[3], Grid* g) {
    int rc = grow(&codes, &codes_cap, (size_t)n);
    if (rc) return rc;
    if (!codes_valid || kappa[0] != codes_kappa[0] || kappa[1] != codes_kappa[1] || kappa[2] != codes_kappa[2]) {
        codes_valid = false;
        Grid g0 = grid(kappa);
        hipError_t e = launch_modecode(g0, (unsigned char*)codes, stream);
        if (e != hipSuccess) return hip_fail(e, "mode codes");
        for (int l = 0; l < 3; ++l) codes_kappa[l] = kappa[l];
        codes_valid = true;
        wtab_valid[0] = wtab_valid[1] = false;
    }
    *g = grid(kappa);
    // the FP32 W table where the fixed-size FP32 plane kernels run: the adjoint kernel then reads
    // W instead of forming it per vector
    const bool regs = (g->fixed_kind[0] == 0 || g->fixed_kind[0] == 4) && wave_plane_available(*g, 0);
    if (!g->generic[0] && !regs && fixed_plane_available(g->n2, g->n3, 0, g->fixed_kind[0])) {
        if (!wtab_valid[0]) {
            if ((rc = grow(&wtab_mem, &wtab_cap, 6 * (size_t)n * sizeof(cx<float>)))) return rc;
            bool done = false;
            hipError_t e = launch_wtable<float>(*g, tables, (cx<float>*)wtab_mem, stream, &done);
            if (e != hipSuccess) return hip_fail(e, "mixing table");
            wtab_valid[0] = done;
        }
        if (wtab_valid[0]) g->wtab[0] = wtab_mem;
    }
    return PCX_OK;
}

int Plan::grid_multi(const double* kappas, int nk, int nvk, Grid* g) {
    int rc = grow(&mcodes, &mcodes_cap, (size_t)nk * n);
    if (rc) return rc;
    if ((rc = grow(&kaps_dev, &kaps_cap, 3 * sizeof(double) * (size_t)nk))) return rc;
    const bool same = mcodes_valid && (int)mkaps.size() == 3 * nk &&
                      std::equal(mkaps.begin(), mkaps.end(), kappas);
    if (!same) {
        mcodes_valid = false;
        for (int k = 0; k < nk; ++k) {
            Grid gk = grid(kappas + 3 * k);
            hipError_t e = launch_modecode(gk, (unsigned char*)mcodes + (size_t)k * n, stream);
            if (e != hipSuccess) return hip_fail(e, "mode codes");
        }
        mkaps.assign(kappas, kappas + 3 * nk);
        hipError_t e = hipMemcpyAsync(kaps_dev, mkaps.data(), 3 * sizeof(double) * (size_t)nk, hipMemcpyHostToDevice,
                                      stream);
        if (e != hipSuccess) return hip_fail(e, "wave vector upload");
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "wave vector upload");
        mcodes_valid = true;
    }
    *g = grid(kappas);
    g->codes = (const unsigned char*)mcodes;
    g->nvk = nvk;
    g->kaps = (const double*)kaps_dev;
    return PCX_OK;
}

}  // namespace pcx

extern "C" int pcx_plan_create(const pcx_geom* g, int max_vectors, void* hip_stream, pcx_plan** out) {
    if (!g || !out) return fail(PCX_E_ARG, "pcx_plan_create: null pointer");
    *out = nullptr;
    if (max_vectors == 0) max_vectors = PCX_MAX_BLOCK;
    if (max_vectors < 1 || max_vectors > 4096) return fail(PCX_E_ARG, "pcx_plan_create: max_vectors out of range");
    FftPlan fx, fy, fz;
    if (!make_fft_plan(g->n[0], &fx) || !make_fft_plan(g->n[1], &fy) || !make_fft_plan(g->n[2], &fz))
        return fail(PCX_E_SIZE, "pcx_plan_create: grid sizes must be 2,3,5-smooth and <= %d", PCX_MAX_N);
    for (int l = 0; l < 3; ++l)
        if (!(g->delta[l] > 0) || !std::isfinite(g->delta[l])) return fail(PCX_E_ARG, "pcx_plan_create: bad delta");
    if (std::abs(g->shift[2]) >= g->n[1]) return fail(PCX_E_LATTICE, "pcx_plan_create: bad shift");
    // LDS budget of the plane kernels (FP64 must fit for the FP64 paths; checked per call)
    int rc = ensure_configured();
    if (rc) return rc;
    Plan* p = new Plan();
    p->geom = *g;
    p->fx = fx;
    p->fy = fy;
    p->fz = fz;
    p->n = (long)g->n[0] * g->n[1] * g->n[2];
    p->max_vectors = max_vectors;
    p->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    if ((rc = noalloc_setup(p->device))) {
        delete p;
        return rc;
    }
    // twiddle tables
    std::vector<cx<double>> h[3];
    for (int a = 0; a < 3; ++a) host_twiddles(g->n[a], h[a]);
    std::vector<cx<double>> half(g->n[2]);
    for (int k = 0; k < g->n[2]; ++k) {
        const double ang = M_PI * (double)k / (double)g->n[2];
        half[k].x = std::cos(ang);
        half[k].y = std::sin(ang);
    }
    // exp(-2 pi i m / M), M = n2 n3
    const long M = (long)g->n[1] * g->n[2];
    std::vector<cx<double>> rot(M);
    for (long m = 0; m < M; ++m) {
        long mm = m;
        if (2 * mm > M) mm -= M;
        const double ang = -2.0 * M_PI * (double)mm / (double)M;
        rot[m].x = std::cos(ang);
        rot[m].y = std::sin(ang);
    }
    size_t tot = 0;
    for (int a = 0; a < 3; ++a) tot += h[a].size();
    const size_t bytes = (tot + half.size() + rot.size()) * sizeof(cx<double>) + (tot + rot.size()) * sizeof(cx<float>);
    e = hipMalloc(&p->tables_mem, bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc tables");
    }
    cx<double>* d64 = (cx<double>*)p->tables_mem;
    cx<float>* d32 = (cx<float>*)(d64 + tot + half.size() + rot.size());
    auto put = [&](cx<double>* dst64, cx<float>* dst32, const std::vector<cx<double>>& src) -> hipError_t {
        hipError_t r = hipMemcpy(dst64, src.data(), src.size() * sizeof(cx<double>), hipMemcpyHostToDevice);
        if (r != hipSuccess || !dst32) return r;
        std::vector<cx<float>> f(src.size());
        for (size_t m = 0; m < src.size(); ++m) {
            f[m].x = (float)src[m].x;
            f[m].y = (float)src[m].y;
        }
        return hipMemcpy(dst32, f.data(), f.size() * sizeof(cx<float>), hipMemcpyHostToDevice);
    };
    hipError_t ec = hipSuccess;
    for (int a = 0; a < 3 && ec == hipSuccess; ++a) {
        p->tables.tw64[a] = d64;
        p->tables.tw32[a] = d32;
        ec = put(d64, d32, h[a]);
        d64 += h[a].size();
        d32 += h[a].size();
    }
    p->tables.halfz = d64;
    if (ec == hipSuccess) ec = put(d64, nullptr, half);
    d64 += half.size();
    p->tables.rot64 = d64;
    p->tables.rot32 = d32;
    if (ec == hipSuccess) ec = put(d64, d32, rot);
    if (ec != hipSuccess) {
        pcx_plan_destroy((pcx_plan*)p);
        return hip_fail(ec, "hipMemcpy tables");
    }
    *out = (pcx_plan*)p;
    return PCX_OK;
}

extern "C" void pcx_plan_destroy(pcx_plan* pp) {
    Plan* p = (Plan*)pp;
    if (!p) return;
    void* bufs[] = {p->tables_mem, p->eps_mem, p->work,   p->lob_mem,  p->prec,     p->gram_part,
                    p->small_mem,  p->codes,   p->mcodes, p->kaps_dev, p->wtab_mem, p->aux,
                    p->mix};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
}

extern "C" int pcx_plan_set_eps(pcx_plan* pp, const double* eps, int layout) {
    Plan* p = (Plan*)pp;
    if (!p || !eps) return fail(PCX_E_ARG, "pcx_plan_set_eps: null pointer");
    if (layout != PCX_EPS_YEE3 && layout != PCX_EPS_VOXEL) return fail(PCX_E_ARG, "pcx_plan_set_eps: bad layout");
    const long n = p->n;
    std::vector<double> inv(3 * n), invn(3 * n), en(3 * n);
    std::vector<float> inv32(3 * n), invn32(3 * n), en32(3 * n);
    double emin = 1e300, emax = -1e300;
    for (long q = 0; q < 3 * n; ++q) {
        const double e = layout == PCX_EPS_YEE3 ? eps[q] : eps[q % n];
        if (!std::isfinite(e) || !(e > 0.0))
            return fail(PCX_E_ARG, "pcx_plan_set_eps: permittivity must be finite and positive (index %ld)", q);
        emin = std::min(emin, e);
        emax = std::max(emax, e);
        inv[q] = 1.0 / e;
        invn[q] = 1.0 / (e * (double)n);
        inv32[q] = (float)inv[q];
        invn32[q] = (float)invn[q];
        en[q] = e / (double)n;
        en32[q] = (float)en[q];
    }
    const size_t bytes = Plan::eps_bytes(n);
    int rc = p->grow(&p->eps_mem, &p->eps_cap, bytes);
    if (rc) return rc;
    p->set_eps_pointers();
    hipError_t e;
    if ((e = hipMemcpy(p->inv_eps64, inv.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->inv_epsn64, invn.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->inv_eps32, inv32.data(), 3 * n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->inv_epsn32, invn32.data(), 3 * n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->epsn64, en.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->epsn32, en32.data(), 3 * n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "pcx_plan_set_eps: copy");
    p->eps_min = emin;
    p->eps_max = emax;
    p->eps_set = true;
    return PCX_OK;
}

namespace pcx {

int Plan::check_fits(int precision) const {
    const int fp64 = precision == PCX_FP64;
    const size_t limit = 160 * 1024;
    const bool plane_ok = plane_kernel_lds(geom.n[1], geom.n[2], fp64) <= limit ||
                          split_kernel_lds(geom.n[1], geom.n[2], fp64) <= limit;
    if (!plane_ok || xline_kernel_lds(geom.n[0], fp64) > limit)
        return fail(PCX_E_SIZE, "grid %dx%dx%d does not fit the kernels' LDS at %s", geom.n[0], geom.n[1], geom.n[2],
                    fp64 ? "FP64" : "FP32");
    return PCX_OK;
}

int Plan::ensure_work(int nvec) {
    // 3n per vector; twice that when FP64 planes take the two-pass path (FP32 fits in the same bytes)
    const size_t per = split_plane_needed(geom.n[1], geom.n[2], 1) ? 2 : 1;
    const size_t need = per * (size_t)nvec * 3 * n * sizeof(cx<double>);
    return grow(&work, &work_cap, need);
}

int Plan::precond_mixed(const double kappa[3], const void* y, void* z, const double* scale, int nvec, bool* done) {
    *done = false;
    if (!eps_set || nvec < 1 || nvec > max_vectors || check_fits(PCX_FP32) != PCX_OK) return PCX_OK;
    int rc = ensure_work(nvec);
    if (rc) return rc;
    Grid g;
    if ((rc = grid_for(kappa, &g))) return rc;
    const hipError_t e = launch_precond_mixed(g, tables, (const float*)epsn32, (const cx<double>*)y, (cx<double>*)z,
                                              (cx<float>*)work, scale, nvec, stream);
    if (e == hipErrorNotSupported) return PCX_OK;
    if (e != hipSuccess) return hip_fail(e, "preconditioner launch");
    *done = true;
    return PCX_OK;
}

int Plan::apply(int op, const double kappa[3], int precision, const void* in, void* out, int nvec) {
    if (!in || !out || !kappa) return fail(PCX_E_ARG, "apply: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "apply: bad precision");
    if (nvec < 1 || nvec > max_vectors) return fail(PCX_E_ARG, "apply: nvec %d outside [1, %d]", nvec, max_vectors);
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "apply: non-finite kappa");
    if ((op == OP_AR || op == OP_EIGVEC || op == OP_AR_EPS) && !eps_set)
        return fail(PCX_E_ARG, "apply: permittivity not set");
    int rc = check_fits(precision);
    if (rc) return rc;
    rc = ensure_work(nvec);
    if (rc) return rc;
    Grid g;
    if ((rc = grid_for(kappa, &g))) return rc;
    hipError_t e = hipSuccess;
    if (precision == PCX_FP64) {
        auto* w = (cx<double>*)work;
        switch (op) {
            case OP_AR: e = launch_apply_Ar<double>(g, tables, (const double*)inv_epsn64, (const cx<double>*)in,
                                                    (cx<double>*)out, w, nvec, stream); break;
            case OP_AR_EPS: e = launch_apply_Ar<double>(g, tables, (const double*)epsn64, (const cx<double>*)in,
                                                        (cx<double>*)out, w, nvec, stream); break;
            case OP_QS: e = launch_QS<double>(g, tables, nullptr, (const cx<double>*)in, (cx<double>*)out, w, nvec,
                                              stream); break;
            case OP_EIGVEC: e = launch_QS<double>(g, tables, (const double*)inv_eps64, (const cx<double>*)in,
                                                  (cx<double>*)out, w, nvec, stream); break;
            case OP_QSADJ: e = launch_QS_adjoint<double>(g, tables, (const cx<double>*)in, (cx<double>*)out, w, nvec,
                                                         stream); break;
        }
    } else {
        auto* w = (cx<float>*)work;
        switch (op) {
            case OP_AR: e = launch_apply_Ar<float>(g, tables, (const float*)inv_epsn32, (const cx<float>*)in,
                                                   (cx<float>*)out, w, nvec, stream); break;
            case OP_AR_EPS: e = launch_apply_Ar<float>(g, tables, (const float*)epsn32, (const cx<float>*)in,
                                                       (cx<float>*)out, w, nvec, stream); break;
            case OP_QS: e = launch_QS<float>(g, tables, nullptr, (const cx<float>*)in, (cx<float>*)out, w, nvec,
                                             stream); break;
            case OP_EIGVEC: e = launch_QS<float>(g, tables, (const float*)inv_eps32, (const cx<float>*)in,
                                                 (cx<float>*)out, w, nvec, stream); break;
            case OP_QSADJ: e = launch_QS_adjoint<float>(g, tables, (const cx<float>*)in, (cx<float>*)out, w, nvec,
                                                        stream); break;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "apply: kernel launch");
    return PCX_OK;
}

}  // namespace pcx

extern "C" int pcx_plan_set_variant(pcx_plan* p, int variant) {
    if (!p) return fail(PCX_E_ARG, "pcx_plan_set_variant: null plan");
    if (variant < PCX_VARIANT_AUTO || variant > PCX_VARIANT_REGISTER)
        return fail(PCX_E_ARG, "pcx_plan_set_variant: unknown variant %d", variant);
    Plan* pl = (Plan*)p;
    pl->variant = variant;
    pl->tuned_nt[0] = pl->tuned_nt[1] = 0;
    pl->tune_checked[0] = pl->tune_checked[1] = true;   // an explicit choice: no tuning by default
    return PCX_OK;
}

namespace {

int curl_args(Plan* p, const double kappa[3], int precision, const void* in, void* out, int nvec, const char* who) {
    if (!p || !kappa || !in || !out) return fail(PCX_E_ARG, "%s: null pointer", who);
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "%s: bad precision", who);
    if (nvec < 1 || nvec > p->max_vectors) return fail(PCX_E_ARG, "%s: nvec %d outside [1, %d]", who, nvec, p->max_vectors);
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "%s: non-finite kappa", who);
    return PCX_OK;
}

template <typename R>
int hfield_impl(Plan* p, const double kappa[3], const void* y, void* h, int nvec) {
    const long n = p->n;
    int rc = p->grow(&p->aux, &p->aux_cap, (size_t)nvec * 5 * n * sizeof(cx<R>));
    if (!rc) rc = p->grow(&p->prec, &p->prec_cap, n * sizeof(double));
    if (rc) return rc;
    Grid g;
    if ((rc = p->grid_for(kappa, &g))) return rc;
    cx<R>* tmp = (cx<R>*)p->aux;                       // Lambda_q^{-1} y
    cx<R>* u = tmp + (size_t)nvec * 2 * n;             // Q_r Sigma_r (Lambda_q^{-1} y)
    hipError_t e = launch_precond_diag(g, p->tables, (double*)p->prec, p->stream);
    if (e == hipSuccess) e = launch_scale_modes<R>((const cx<R>*)y, tmp, (const double*)p->prec, n, nvec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_hfield: scaling");
    if ((rc = p->apply(Plan::OP_QS, kappa, sizeof(R) == 8 ? PCX_FP64 : PCX_FP32, tmp, u, nvec))) return rc;
    e = launch_curl<R>(g, u, (cx<R>*)h, nvec, false, p->stream);
    return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_hfield: curl");
}

template <typename R>
int hoperator_impl(Plan* p, const double kappa[3], const void* h, void* z, int nvec) {
    const long n = p->n;
    int rc = p->grow(&p->aux, &p->aux_cap, (size_t)nvec * 5 * n * sizeof(cx<R>));
    if (rc) return rc;
    Grid g = p->grid(kappa);
    cx<R>* t = (cx<R>*)p->aux;
    const R* inv = sizeof(R) == 8 ? (const R*)p->inv_eps64 : (const R*)p->inv_eps32;
    hipError_t e = launch_curl<R>(g, (const cx<R>*)h, t, nvec, true, p->stream);
    if (e == hipSuccess) e = launch_scale3<R>(inv, t, 3 * n, nvec, p->stream);
    if (e == hipSuccess) e = launch_curl<R>(g, t, (cx<R>*)z, nvec, false, p->stream);
    return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_apply_hfield_operator");
}

}  // namespace

extern "C" int pcx_apply_curl(pcx_plan* pp, const double kappa[3], int precision, const void* u, void* v, int nvec,
                              int adjoint) {
    Plan* p = (Plan*)pp;
    int rc = curl_args(p, kappa, precision, u, v, nvec, "pcx_apply_curl");
    if (rc) return rc;
    Grid g = p->grid(kappa);
    hipError_t e = precision == PCX_FP64
                       ? launch_curl<double>(g, (const cx<double>*)u, (cx<double>*)v, nvec, adjoint != 0, p->stream)
                       : launch_curl<float>(g, (const cx<float>*)u, (cx<float>*)v, nvec, adjoint != 0, p->stream);
    return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_apply_curl");
}

extern "C" int pcx_hfield(pcx_plan* pp, const double kappa[3], int precision, const void* y, void* h, int nvec) {
    Plan* p = (Plan*)pp;
    int rc = curl_args(p, kappa, precision, y, h, nvec, "pcx_hfield");
    if (rc) return rc;
    if ((rc = p->check_fits(precision))) return rc;
    return precision == PCX_FP64 ? hfield_impl<double>(p, kappa, y, h, nvec) : hfield_impl<float>(p, kappa, y, h, nvec);
}

extern "C" int pcx_apply_hfield_operator(pcx_plan* pp, const double kappa[3], int precision, const void* h, void* z,
                                         int nvec) {
    Plan* p = (Plan*)pp;
    int rc = curl_args(p, kappa, precision, h, z, nvec, "pcx_apply_hfield_operator");
    if (rc) return rc;
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_apply_hfield_operator: permittivity not set");
    return precision == PCX_FP64 ? hoperator_impl<double>(p, kappa, h, z, nvec)
                                 : hoperator_impl<float>(p, kappa, h, z, nvec);
}

extern "C" int pcx_apply_Ar(pcx_plan* p, const double kappa[3], int precision, const void* y, void* z, int nvec) {
    if (!p) return fail(PCX_E_ARG, "pcx_apply_Ar: null plan");
    return ((Plan*)p)->apply(Plan::OP_AR, kappa, precision, y, z, nvec);
}
extern "C" int pcx_apply_precond(pcx_plan* pp, const double kappa[3], int precision, const void* y, void* z,
                                 int nvec) {
    Plan* p = (Plan*)pp;
    if (!p || !kappa || !y || !z) return fail(PCX_E_ARG, "pcx_apply_precond: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32 && precision != PCX_FP64_OP32)
        return fail(PCX_E_ARG, "pcx_apply_precond: bad precision");
    if (nvec < 1 || nvec > p->max_vectors)
        return fail(PCX_E_ARG, "pcx_apply_precond: nvec %d outside [1, %d]", nvec, p->max_vectors);
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_apply_precond: permittivity not set");
    for (int l = 0; l < 3; ++l)
        if (!std::isfinite(kappa[l])) return fail(PCX_E_ARG, "pcx_apply_precond: non-finite kappa");
    const bool mixed = precision == PCX_FP64_OP32;
    int rc = p->check_fits(mixed ? PCX_FP32 : precision);
    if (rc) return rc;
    if ((rc = p->grow(&p->prec, &p->prec_cap, p->n * sizeof(double)))) return rc;
    Grid g;
    if ((rc = p->grid_for(kappa, &g))) return rc;
    hipError_t e = launch_precond_diag(g, p->tables, (double*)p->prec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_apply_precond: Lambda_q^{-1}");
    const double* d = (const double*)p->prec;
    if (mixed) {
        // the FP64 solver's preconditioner: inner D in FP64, the operator in FP32, outer D in FP64
        e = launch_scale_modes<double>((const cx<double>*)y, (cx<double>*)z, d, p->n, nvec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_apply_precond: scaling");
        bool done = false;
        if ((rc = p->precond_mixed(kappa, z, z, d, nvec, &done))) return rc;
        if (done) return PCX_OK;
        const long len = 2 * p->n * (long)nvec;
        if ((rc = p->grow(&p->mix, &p->mix_cap, 2 * len * sizeof(cx<float>)))) return rc;
        cx<float>* tin = (cx<float>*)p->mix;
        cx<float>* tout = tin + len;
        e = launch_convert((const cx<double>*)z, tin, len, p->stream);
        if (e != hipSuccess) return hip_fail(e, "pcx_apply_precond: conversion");
        if ((rc = p->apply(Plan::OP_AR_EPS, kappa, PCX_FP32, tin, tout, nvec))) return rc;
        e = launch_scale_modes(tout, (cx<double>*)z, d, p->n, nvec, p->stream);
        return e == hipSuccess ? PCX_OK : hip_fail(e, "pcx_apply_precond: scaling");
    }
    if (precision == PCX_FP64)
        e = launch_scale_modes<double>((const cx<double>*)y, (cx<double>*)z, d, p->n, nvec, p->stream);
    else
        e = launch_scale_modes<float>((const cx<float>*)y, (cx<float>*)z, d, p->n, nvec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_apply_precond: scaling");
    if ((rc = p->apply(Plan::OP_AR_EPS, kappa, precision, z, z, nvec))) return rc;
    if (precision == PCX_FP64)
        e = launch_scale_modes<double>((const cx<double>*)z, (cx<double>*)z, d, p->n, nvec, p->stream);
    else
        e = launch_scale_modes<float>((const cx<float>*)z, (cx<float>*)z, d, p->n, nvec, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_apply_precond: scaling");
    return PCX_OK;
}

extern "C" int pcx_apply_Ar_multi(pcx_plan* pp, int nk, const double* kappas, int precision, const void* y,
                                  void* z, int nvec_per_k) {
    Plan* p = (Plan*)pp;
    if (!p || !kappas || !y || !z) return fail(PCX_E_ARG, "pcx_apply_Ar_multi: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_apply_Ar_multi: bad precision");
    if (nk < 1 || nvec_per_k < 1 || (long)nk * nvec_per_k > p->max_vectors)
        return fail(PCX_E_ARG, "pcx_apply_Ar_multi: nk * nvec_per_k must be in [1, %d]", p->max_vectors);
    for (int q = 0; q < 3 * nk; ++q)
        if (!std::isfinite(kappas[q])) return fail(PCX_E_ARG, "pcx_apply_Ar_multi: non-finite kappa");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_apply_Ar_multi: permittivity not set");
    int rc = p->check_fits(precision);
    if (rc) return rc;
    const int nv = nk * nvec_per_k;
    if ((rc = p->ensure_work(nv))) return rc;
    Grid g;
    if ((rc = p->grid_multi(kappas, nk, nvec_per_k, &g))) return rc;
    hipError_t e;
    if (precision == PCX_FP64)
        e = launch_apply_Ar<double>(g, p->tables, (const double*)p->inv_epsn64, (const cx<double>*)y, (cx<double>*)z,
                                    (cx<double>*)p->work, nv, p->stream);
    else
        e = launch_apply_Ar<float>(g, p->tables, (const float*)p->inv_epsn32, (const cx<float>*)y, (cx<float>*)z,
                                   (cx<float>*)p->work, nv, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_apply_Ar_multi: kernel launch");
    return PCX_OK;
}

extern "C" int pcx_apply_QS(pcx_plan* p, const double kappa[3], int precision, const void* y, void* u, int nvec) {
    if (!p) return fail(PCX_E_ARG, "pcx_apply_QS: null plan");
    return ((Plan*)p)->apply(Plan::OP_QS, kappa, precision, y, u, nvec);
}
extern "C" int pcx_apply_QS_adjoint(pcx_plan* p, const double kappa[3], int precision, const void* u, void* z,
                                    int nvec) {
    if (!p) return fail(PCX_E_ARG, "pcx_apply_QS_adjoint: null plan");
    return ((Plan*)p)->apply(Plan::OP_QSADJ, kappa, precision, u, z, nvec);
}
extern "C" int pcx_eigvec(pcx_plan* p, const double kappa[3], int precision, const void* y, void* x, int nvec) {
    if (!p) return fail(PCX_E_ARG, "pcx_eigvec: null plan");
    return ((Plan*)p)->apply(Plan::OP_EIGVEC, kappa, precision, y, x, nvec);
}

// the Rayleigh-Ritz products on their own (scratch allocated per call; the solver keeps its own)
extern "C" int pcx_block_gram(pcx_plan* pp, int precision, const void* a, int ka, const void* b, int kb, long len,
                              int herm, double* g) {
    Plan* p = (Plan*)pp;
    if (!p || !a || !g || (!b && !(herm && kb == ka))) return fail(PCX_E_ARG, "pcx_block_gram: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_block_gram: bad precision");
    if (ka < 1 || kb < 1 || ka > 3 * PCX_MAX_BLOCK || kb > 6 * PCX_MAX_BLOCK || len < 1)
        return fail(PCX_E_ARG, "pcx_block_gram: bad sizes");
    if (herm && kb != ka && kb != 2 * ka) return fail(PCX_E_ARG, "pcx_block_gram: herm needs kb = ka or 2 ka");
    const size_t es = precision == PCX_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
    void* A = const_cast<void*>(a);
    ColSet As = colset(A, ka);
    ColSet Bs = herm ? (kb == ka ? colset(A, ka) : colset(A, ka, const_cast<void*>(b), ka))
                     : colset(const_cast<void*>(b), kb);
    (void)es;
    const int chunks = gram_chunks_for(len);
    const size_t count = (size_t)ka * kb;
    void* part = nullptr;
    void* out = nullptr;
    hipError_t e = hipMalloc(&part, sizeof(cx<double>) * (size_t)(chunks + 33) * count);
    if (e == hipSuccess) e = hipMalloc(&out, sizeof(cx<double>) * count);
    if (e != hipSuccess) {
        (void)hipFree(part);
        (void)hipGetLastError();
        return fail(PCX_E_OOM, "pcx_block_gram: scratch");
    }
    e = precision == PCX_FP64
            ? launch_gram<double>(As, Bs, len, (cx<double>*)part, chunks, (cx<double>*)out, p->stream, herm != 0)
            : launch_gram<float>(As, Bs, len, (cx<double>*)part, chunks, (cx<double>*)out, p->stream, herm != 0);
    if (e == hipSuccess) e = hipMemcpyAsync(g, out, sizeof(cx<double>) * count, hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(part);
    (void)hipFree(out);
    if (e != hipSuccess) return hip_fail(e, "pcx_block_gram");
    if (herm) {
        // the lower triangle of each half from the upper one (each half Hermitian)
        cx<double>* G = (cx<double>*)g;
        for (int h = 0; h < kb / ka; ++h)
            for (int i = 0; i < ka; ++i) {
                G[(size_t)i * kb + h * ka + i].y = 0.0;
                for (int j = 0; j < i; ++j) {
                    const cx<double> u = G[(size_t)j * kb + h * ka + i];
                    G[(size_t)i * kb + h * ka + j].x = u.x;
                    G[(size_t)i * kb + h * ka + j].y = -u.y;
                }
            }
    }
    return PCX_OK;
}

extern "C" int pcx_block_combine(pcx_plan* pp, int precision, const void* s, int ks, const double* c, int m, void* y,
                                 long len) {
    Plan* p = (Plan*)pp;
    if (!p || !s || !c || !y) return fail(PCX_E_ARG, "pcx_block_combine: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_block_combine: bad precision");
    if (ks < 1 || m < 1 || ks > 3 * PCX_MAX_BLOCK || m > 3 * PCX_MAX_BLOCK || len < 1)
        return fail(PCX_E_ARG, "pcx_block_combine: bad sizes");
    void* dc = nullptr;
    hipError_t e = hipMalloc(&dc, sizeof(cx<double>) * (size_t)ks * m);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PCX_E_OOM, "pcx_block_combine: scratch");
    }
    e = hipMemcpyAsync(dc, c, sizeof(cx<double>) * (size_t)ks * m, hipMemcpyHostToDevice, p->stream);
    const ColSet S = colset(const_cast<void*>(s), ks), Y = colset(y, m);
    if (e == hipSuccess)
        e = precision == PCX_FP64 ? launch_combine<double>(S, (const cx<double>*)dc, Y, len, p->stream)
                                  : launch_combine<float>(S, (const cx<double>*)dc, Y, len, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    (void)hipFree(dc);
    if (e != hipSuccess) return hip_fail(e, "pcx_block_combine");
    return PCX_OK;
}

extern "C" int pcx_time_Ar_kernels(pcx_plan* pp, const double kappa[3], int precision, const void* y, void* z,
                                   int nvec, int reps, double ms_out[3]) {
    Plan* p = (Plan*)pp;
    if (!p || !kappa || !y || !z || !ms_out) return fail(PCX_E_ARG, "pcx_time_Ar_kernels: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_time_Ar_kernels: bad precision");
    if (nvec < 1 || nvec > p->max_vectors || reps < 1) return fail(PCX_E_ARG, "pcx_time_Ar_kernels: bad nvec/reps");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_time_Ar_kernels: permittivity not set");
    int rc = p->check_fits(precision);
    if (rc) return rc;
    if ((rc = p->ensure_work(nvec))) return rc;
    Grid g;
    if ((rc = p->grid_for(kappa, &g))) return rc;
    hipError_t e;
    if (precision == PCX_FP64)
        e = time_apply_Ar<double>(g, p->tables, (const double*)p->inv_epsn64, (const cx<double>*)y, (cx<double>*)z,
                                  (cx<double>*)p->work, nvec, reps, p->stream, ms_out);
    else
        e = time_apply_Ar<float>(g, p->tables, (const float*)p->inv_epsn32, (const cx<float>*)y, (cx<float>*)z,
                                 (cx<float>*)p->work, nvec, reps, p->stream, ms_out);
    if (e != hipSuccess) return hip_fail(e, "pcx_time_Ar_kernels");
    return PCX_OK;
}

extern "C" int pcx_grad_eps(pcx_plan* pp, int nvec, const void* x, const double* weight, void* grad, int layout) {
    Plan* p = (Plan*)pp;
    if (!p || !x || !weight || !grad) return fail(PCX_E_ARG, "pcx_grad_eps: null pointer");
    if (nvec < 1 || nvec > PCX_MAX_BLOCK) return fail(PCX_E_ARG, "pcx_grad_eps: nvec out of range");
    if (layout != PCX_EPS_YEE3 && layout != PCX_EPS_VOXEL) return fail(PCX_E_ARG, "pcx_grad_eps: bad layout");
    int rc = p->grow(&p->small_mem, &p->small_cap, 1 << 16);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(p->small_mem, weight, nvec * sizeof(double), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_grad_eps: copy");
    e = launch_grad((const cx<double>*)x, (const double*)p->small_mem, nvec, p->n, (double*)grad,
                    layout == PCX_EPS_VOXEL, p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_grad_eps: launch");
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "pcx_grad_eps: sync");
    return PCX_OK;
}
