// Batches of independent eigenproblems and the per-plan kernel autotuner.
//
// One GEP per wave vector (Section 5.2: the band structure is a sequence of independent
// problems, one per k), so a request of several lattices x wave vectors is a bag of independent
// LOBPCG solves.  pcx_solve_batch runs them concurrently: each worker thread owns one HIP stream
// and, per lattice it meets, a private clone of that lattice's plan (workspaces, mode codes and
// a device copy of 1/eps), and takes problems from a shared counter.  The GPU then overlaps the
// kernels of different problems, and one problem's host Rayleigh-Ritz step hides behind the
// others' device work.  All wave vectors of one lattice can also go through a single launch of
// each A_r kernel (pcx_apply_Ar_multi).
//
// pcx_plan_autotune times the A_r kernels of a plan in each available variant (fixed-size
// kernels for the grid, generic kernels at 256 / 512 / 1024 threads per plane) on the plan's
// stream and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pcx_host.h"

using namespace pcx;

namespace {

// a worker's private copy of `src`: same geometry, variant and permittivity, own stream and buffers
int clone_plan(const Plan* src, hipStream_t st, Plan** out) {
    *out = nullptr;
    pcx_plan* q = nullptr;
    int rc = pcx_plan_create(&src->geom, src->max_vectors, st, &q);
    if (rc) return rc;
    Plan* p = (Plan*)q;
    p->variant = src->variant;
    p->tuned_nt[0] = src->tuned_nt[0];
    p->tuned_nt[1] = src->tuned_nt[1];
    const size_t bytes = Plan::eps_bytes(src->n);
    if ((rc = p->grow(&p->eps_mem, &p->eps_cap, bytes))) {
        pcx_plan_destroy(q);
        return rc;
    }
    p->set_eps_pointers();
    hipError_t e = hipMemcpyAsync(p->eps_mem, src->eps_mem, bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        pcx_plan_destroy(q);
        return hip_fail(e, "pcx_solve_batch: permittivity copy");
    }
    p->eps_min = src->eps_min;
    p->eps_max = src->eps_max;
    p->eps_set = true;
    *out = p;
    return PCX_OK;
}

}  // namespace

extern "C" int pcx_solve_batch(pcx_plan* const* plans, int nplans, const int* nk, const double* kappas, int nev,
                               const pcx_opts* opts, int nworkers, double* lambda, void* const* y_out,
                               pcx_stats* stats) {
    if (!plans || !nk || !kappas || !lambda || nplans < 1) return fail(PCX_E_ARG, "pcx_solve_batch: null pointer");
    std::vector<int> owner;   // problem -> plan
    for (int p = 0; p < nplans; ++p) {
        const Plan* pl = (const Plan*)plans[p];
        if (!pl) return fail(PCX_E_ARG, "pcx_solve_batch: null plan %d", p);
        if (!pl->eps_set) return fail(PCX_E_ARG, "pcx_solve_batch: permittivity not set on plan %d", p);
        if (nk[p] < 0) return fail(PCX_E_ARG, "pcx_solve_batch: negative wave-vector count");
        for (int k = 0; k < nk[p]; ++k) owner.push_back(p);
    }
    const int total = (int)owner.size();
    if (total == 0) return PCX_OK;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(PCX_E_DEVICE, "pcx_solve_batch: no device");
    for (int p = 0; p < nplans; ++p)
        if (((const Plan*)plans[p])->device != device)
            return fail(PCX_E_ARG, "pcx_solve_batch: plan %d lives on another device", p);
    const int W = std::max(1, std::min(total, nworkers > 0 ? nworkers : 4));

    std::atomic<int> next(0);
    std::vector<int> rc(total, PCX_OK);
    std::vector<std::string> msg(total);
    std::vector<int> worker_rc(W, PCX_OK);
    std::vector<std::string> worker_msg(W);
    auto work = [&](int w) {
        if (hipSetDevice(device) != hipSuccess) {
            worker_rc[w] = PCX_E_DEVICE;
            worker_msg[w] = "hipSetDevice failed";
            return;
        }
        hipStream_t st = nullptr;
        if (hipStreamCreate(&st) != hipSuccess) {
            worker_rc[w] = PCX_E_DEVICE;
            worker_msg[w] = "hipStreamCreate failed";
            return;
        }
        std::vector<Plan*> mine(nplans, nullptr);
        for (int q = next++; q < total; q = next++) {
            const int p = owner[q];
            if (!mine[p]) {
                int r = clone_plan((const Plan*)plans[p], st, &mine[p]);
                if (r) {
                    rc[q] = r;
                    msg[q] = pcx_last_error();
                    continue;
                }
            }
            pcx_stats local;
            int r = pcx_solve((pcx_plan*)mine[p], kappas + 3 * q, nev, opts, lambda + (size_t)q * nev,
                              y_out ? y_out[q] : nullptr, nullptr, stats ? &stats[q] : &local);
            rc[q] = r;
            if (r) msg[q] = pcx_last_error();
        }
        for (Plan* c : mine)
            if (c) pcx_plan_destroy((pcx_plan*)c);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    };
    std::vector<std::thread> th;
    for (int w = 1; w < W; ++w) th.emplace_back(work, w);
    work(0);
    for (auto& t : th) t.join();
    for (int w = 0; w < W; ++w)
        if (worker_rc[w]) return fail(worker_rc[w], "pcx_solve_batch: worker %d: %s", w, worker_msg[w].c_str());
    // the first hard error, else the first non-convergence
    for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < total; ++q)
            if (rc[q] && (pass == 1 || rc[q] != PCX_E_NOCONV))
                return fail(rc[q], "pcx_solve_batch: problem %d: %s", q, msg[q].c_str());
    return PCX_OK;
}

extern "C" int pcx_plan_autotune(pcx_plan* pp, const double kappa[3], int precision, int nvec, int* choice_out,
                                 double* ms_out) {
    Plan* p = (Plan*)pp;
    if (!p || !kappa) return fail(PCX_E_ARG, "pcx_plan_autotune: null pointer");
    if (precision != PCX_FP64 && precision != PCX_FP32) return fail(PCX_E_ARG, "pcx_plan_autotune: bad precision");
    if (nvec < 1 || nvec > p->max_vectors) return fail(PCX_E_ARG, "pcx_plan_autotune: nvec outside [1, max_vectors]");
    if (!p->eps_set) return fail(PCX_E_ARG, "pcx_plan_autotune: permittivity not set");
    int rc = p->check_fits(precision);
    if (rc) return rc;
    const size_t c = precision == PCX_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
    const size_t bytes = (size_t)nvec * 2 * p->n * c;
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, 2 * bytes);
    if (e != hipSuccess) return hip_fail(e, "pcx_plan_autotune: buffers");
    // any input will do for timing: a constant block
    e = hipMemsetAsync(buf, 0, 2 * bytes, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        (void)hipFree(buf);
        return hip_fail(e, "pcx_plan_autotune: buffers");
    }
    const int f = precision == PCX_FP64 ? 1 : 0;
    std::vector<int> cands;       // tuned_nt values: -1 fixed-size kernels, else generic group size
    if (fixed_plane_available(p->geom.n[1], p->geom.n[2], f, 3)) cands.push_back(-1);
    if (fixed_plane_available(p->geom.n[1], p->geom.n[2], f, 2)) cands.push_back(-2);
    cands.push_back(256);
    cands.push_back(512);
    if (!f) cands.push_back(1024);
    const int keep_v = p->variant, keep_t = p->tuned_nt[f];
    double best = 1e300;
    int pick = keep_t;
    p->variant = PCX_VARIANT_AUTO;
    for (int cd : cands) {
        p->tuned_nt[f] = cd;
        double ms[3] = {0, 0, 0};
        rc = pcx_time_Ar_kernels(pp, kappa, precision, buf, (char*)buf + bytes, nvec, 2, ms);   // warm-up
        if (!rc) rc = pcx_time_Ar_kernels(pp, kappa, precision, buf, (char*)buf + bytes, nvec, 5, ms);
        if (rc) break;
        const double t = ms[0] + ms[1] + ms[2];
        if (t < best) {
            best = t;
            pick = cd;
        }
    }
    (void)hipFree(buf);
    p->variant = keep_v;
    if (rc) {
        p->tuned_nt[f] = keep_t;
        return rc;
    }
    p->tuned_nt[f] = pick;
    if (choice_out) *choice_out = pick;
    if (ms_out) *ms_out = best;
    return PCX_OK;
}
