// Batches of independent eigenproblems and the per-plan kernel autotuner.
//
// One GEP per wave vector (Section 5.2: the band structure is a sequence of independent
// problems, one per k), so a request of several lattices x wave vectors is a bag of independent
// LOBPCG solves.  pcx_solve_batch runs them concurrently: each worker thread owns one HIP stream,
// a private clone of every lattice's plan (mode codes and a device copy of 1/eps) and one set of
// matvec and eigensolver storage shared by its clones, all created before the workers start,
// and takes problems from a shared counter.  The GPU then overlaps the
// kernels of different problems, and one problem's host Rayleigh-Ritz step hides behind the
// others' device work.  All wave vectors of one lattice can also go through a single launch of
// each A_r kernel (pcx_apply_Ar_multi).
//
// pcx_plan_autotune times the A_r kernels of a plan in each available variant (the automatic
// choice, fixed-size kernels for the grid, generic kernels at 256 / 512 / 1024 threads per plane)
// on the plan's stream and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
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

// The matvec and eigensolver storage of a plan.  The plans of one worker never run at the same
// time, so they share one set: it is moved into a plan for the duration of a solve and back out.
struct Storage {
    void* work = nullptr; size_t work_cap = 0;
    void* lob_mem = nullptr; size_t lob_cap = 0;
    void* prec = nullptr; size_t prec_cap = 0;
    void* gram_part = nullptr; size_t gram_part_cap = 0;
    void* small_mem = nullptr; size_t small_cap = 0;
    void* pinned = nullptr; size_t pinned_cap = 0;
};

void swap_storage(Plan* p, Storage& s) {
    std::swap(p->work, s.work); std::swap(p->work_cap, s.work_cap);
    std::swap(p->lob_mem, s.lob_mem); std::swap(p->lob_cap, s.lob_cap);
    std::swap(p->prec, s.prec); std::swap(p->prec_cap, s.prec_cap);
    std::swap(p->gram_part, s.gram_part); std::swap(p->gram_part_cap, s.gram_part_cap);
    std::swap(p->small_mem, s.small_mem); std::swap(p->small_cap, s.small_cap);
    std::swap(p->pinned, s.pinned); std::swap(p->pinned_cap, s.pinned_cap);
}

// Per-worker resources, all created on the calling thread before any worker starts and released
// there after every worker has joined and every stream has drained: no allocation or free runs
// beside another worker's kernels.
struct Workers {
    std::vector<hipStream_t> streams;
    std::vector<std::vector<Plan*>> clones;   // [worker][plan]
    std::vector<Storage> storage;             // [worker]

    ~Workers() {
        for (hipStream_t st : streams)
            if (st) (void)hipStreamSynchronize(st);
        for (size_t w = 0; w < clones.size(); ++w) {
            // hand the shared storage to one clone so that its destroy frees it
            for (Plan* c : clones[w])
                if (c) {
                    swap_storage(c, storage[w]);
                    break;
                }
            for (Plan* c : clones[w])
                if (c) pcx_plan_destroy((pcx_plan*)c);
        }
        for (hipStream_t st : streams)
            if (st) (void)hipStreamDestroy(st);
    }
};

}  // namespace

extern "C" int pcx_solve_batch(pcx_plan* const* plans, int nplans, const int* nk, const double* kappas, int nev,
                               const pcx_opts* opts, int nworkers, double* lambda, void* const* y_out,
                               pcx_stats* stats) {
    if (!plans || !nk || !kappas || !lambda || nplans < 1) return fail(PCX_E_ARG, "pcx_solve_batch: null pointer");
    if (nev < 1) return fail(PCX_E_ARG, "pcx_solve_batch: nev must be >= 1");
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
    pcx_opts o;
    if (opts) o = *opts;
    else pcx_opts_default(&o);
    const bool use32 = o.mode != PCX_MODE_FP64, use64 = o.mode != PCX_MODE_FP32;

    // the default tuning of every plan (on this thread, before the clones copy the choice)
    {
        std::vector<bool> seen(nplans, false);
        for (size_t q = 0; q < owner.size(); ++q) {
            const int p = owner[q];
            if (seen[p]) continue;
            seen[p] = true;
            Plan* pl = (Plan*)plans[p];
            const int bt = std::min(solver_max_block(nev, &o), pl->max_vectors);
            const double* kq = kappas + 3 * q;
            int r = PCX_OK;
            if (use32 || o.precondition == PCX_PRECOND_INVERSE) r = autotune_default(pl, kq, PCX_FP32, bt);
            if (!r && use64) r = autotune_default(pl, kq, PCX_FP64, bt);
            if (r) return r;
        }
    }

    // streams, plan clones and storage for every worker, before any worker starts
    Workers wk;
    wk.streams.assign(W, nullptr);
    wk.clones.assign(W, std::vector<Plan*>(nplans, nullptr));
    wk.storage.assign(W, Storage());
    std::vector<bool> used(nplans, false);
    for (int p : owner) used[p] = true;
    for (int w = 0; w < W; ++w) {
        hipError_t e = hipStreamCreate(&wk.streams[w]);
        if (e != hipSuccess) return hip_fail(e, "pcx_solve_batch: stream");
        for (int p = 0; p < nplans; ++p) {
            if (!used[p]) continue;
            int r = clone_plan((const Plan*)plans[p], wk.streams[w], &wk.clones[w][p]);
            if (r) return r;
            // grow the worker's shared storage to what this plan's largest block needs
            Plan* c = wk.clones[w][p];
            const int bmax = std::min(solver_max_block(nev, &o), c->max_vectors);
            c->block_cap = bmax;
            swap_storage(c, wk.storage[w]);
            r = solver_reserve(c, bmax, use32, use64);
            if (!r) r = c->ensure_work(bmax);
            swap_storage(c, wk.storage[w]);
            if (r) return r;
        }
    }

    std::atomic<int> next(0);
    std::vector<int> rc(total, PCX_OK);
    std::vector<std::string> msg(total);
    std::vector<int> worker_rc(W, PCX_OK);
    auto work = [&](int w) {
        if (hipSetDevice(device) != hipSuccess) {
            worker_rc[w] = PCX_E_DEVICE;
            return;
        }
        for (int q = next++; q < total; q = next++) {
            Plan* c = wk.clones[w][owner[q]];
            pcx_stats local;
            swap_storage(c, wk.storage[w]);
            int r = pcx_solve((pcx_plan*)c, kappas + 3 * q, nev, &o, lambda + (size_t)q * nev,
                              y_out ? y_out[q] : nullptr, nullptr, stats ? &stats[q] : &local);
            swap_storage(c, wk.storage[w]);
            rc[q] = r;
            if (r) msg[q] = pcx_last_error();
        }
        (void)hipStreamSynchronize(wk.streams[w]);
    };
    std::vector<std::thread> th;
    for (int w = 1; w < W; ++w) th.emplace_back(work, w);
    work(0);
    for (auto& t : th) t.join();
    for (int w = 0; w < W; ++w)
        if (worker_rc[w]) return fail(worker_rc[w], "pcx_solve_batch: worker %d: hipSetDevice failed", w);
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
    // tuned_nt values: 0 the plan's automatic choice (where the planes are too large for the
    // one-pass kernels, the two-pass planes with the fixed-size x lines), -1 / -2 / -3 the fixed-size
    // three-plane / two-plane / register kernels, else the generic kernels' group size
    std::vector<int> cands{0};
    if (fixed_plane_available(p->geom.n[1], p->geom.n[2], f, 3)) cands.push_back(-1);
    if (fixed_plane_available(p->geom.n[1], p->geom.n[2], f, 2)) cands.push_back(-2);
    // the register kernels (FP32 64 x 64 planes, n1 a multiple of 8)
    if (!f && p->geom.n[1] == 64 && p->geom.n[2] == 64 && p->geom.n[0] % 8 == 0) cands.push_back(-3);
    cands.push_back(256);
    cands.push_back(512);
    if (!f) cands.push_back(1024);
    const int keep_v = p->variant, keep_t = p->tuned_nt[f];
    double best = 1e300;
    int pick = keep_t;
    p->variant = PCX_VARIANT_AUTO;
    // the GPU's clocks rise over some tens of milliseconds of load: a sustained warm-up first, then
    // the best of two rounds over the candidates, so that no candidate is timed on a cold device
    {
        double ms[3] = {0, 0, 0};
        for (int w = 0; w < 4 && !rc; ++w)
            rc = pcx_time_Ar_kernels(pp, kappa, precision, buf, (char*)buf + bytes, nvec, 5, ms);
    }
    std::vector<double> tbest(cands.size(), 1e300);
    for (int round = 0; round < 2 && !rc; ++round)
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            p->tuned_nt[f] = cands[ci];
            double ms[3] = {0, 0, 0};
            rc = pcx_time_Ar_kernels(pp, kappa, precision, buf, (char*)buf + bytes, nvec, 1, ms);   // warm-up
            if (!rc) rc = pcx_time_Ar_kernels(pp, kappa, precision, buf, (char*)buf + bytes, nvec, 4, ms);
            if (rc) break;
            tbest[ci] = std::min(tbest[ci], ms[0] + ms[1] + ms[2]);
        }
    for (size_t ci = 0; ci < cands.size() && !rc; ++ci)
        if (tbest[ci] < best) {
            best = tbest[ci];
            pick = cands[ci];
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

// ------------------------------------------------------------------ tuning by default
namespace pcx {

int autotune_default(Plan* p, const double kappa[3], int precision, int nvec) {
    const int f = precision == PCX_FP64 ? 1 : 0;
    if (p->variant != PCX_VARIANT_AUTO || p->tuned_nt[f] != 0 || p->tune_checked[f]) return PCX_OK;
    p->tune_checked[f] = true;
    // one choice per (grid, precision) for the whole process
    static std::mutex mu;
    static std::vector<std::array<int, 5>> cache;   // n1, n2, n3, precision, choice
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const auto& c : cache)
            if (c[0] == p->geom.n[0] && c[1] == p->geom.n[1] && c[2] == p->geom.n[2] && c[3] == f) {
                p->tuned_nt[f] = c[4];
                return PCX_OK;
            }
    }
    int choice = 0;
    double ms = 0;
    // tuning only chooses among correct variants: where it cannot run (no room for the precision's
    // kernels, no scratch) the default choice stays
    if (p->check_fits(precision) != PCX_OK) return PCX_OK;
    const int rc = pcx_plan_autotune((pcx_plan*)p, kappa, precision, std::max(1, std::min(nvec, p->max_vectors)),
                                     &choice, &ms);
    if (rc) return PCX_OK;
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({p->geom.n[0], p->geom.n[1], p->geom.n[2], f, choice});
    return PCX_OK;
}

}  // namespace pcx
