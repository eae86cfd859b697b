// Host-side plan object shared by the ABI entry points and the eigensolver.
#pragma once

#include <vector>

#include "pcx_internal.h"

namespace pcx {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
bool make_fft_plan(int n, FftPlan* fp);

struct Plan {
    // OP_AR_EPS: Sigma_r Q_r^* B Q_r Sigma_r, the operator with eps in place of 1/eps
    enum { OP_AR = 0, OP_QS = 1, OP_QSADJ = 2, OP_EIGVEC = 3, OP_AR_EPS = 4 };

    pcx_geom geom;
    FftPlan fx, fy, fz;
    long n = 0;
    int max_vectors = 0;
    int device = 0;
    hipStream_t stream = nullptr;

    void* tables_mem = nullptr;
    DeviceTables tables;

    // 1/eps (FP64), 1/(n eps) (FP64), 1/eps (FP32), 1/(n eps) (FP32), eps/n (FP64), eps/n (FP32):
    // 3n each, one allocation
    void* eps_mem = nullptr;
    size_t eps_cap = 0;
    static size_t eps_bytes(long n) { return 3 * (size_t)n * (3 * sizeof(double) + 3 * sizeof(float)); }
    void* inv_eps64 = nullptr;
    void* inv_epsn64 = nullptr;
    void* inv_eps32 = nullptr;
    void* inv_epsn32 = nullptr;
    void* epsn64 = nullptr;          // eps / n: the approximate-inverse preconditioner
    void* epsn32 = nullptr;
    bool eps_set = false;
    double eps_min = 0, eps_max = 0;

    // matvec workspace (3n complex per vector)
    void* work = nullptr;
    size_t work_cap = 0;
    // magnetic-field maps: 2n + 3n complex per vector
    void* aux = nullptr;
    size_t aux_cap = 0;

    // eigensolver storage
    void* lob_mem = nullptr;
    size_t lob_cap = 0;
    void* prec = nullptr;
    size_t prec_cap = 0;
    void* mix = nullptr;             // FP32 copies for pcx_apply_precond(PCX_FP64_OP32) off the register kernels
    size_t mix_cap = 0;
    void* gram_part = nullptr;
    size_t gram_part_cap = 0;
    void* small_mem = nullptr;
    size_t small_cap = 0;
    void* pinned = nullptr;          // pinned host staging: coefficient uploads, small results
    size_t pinned_cap = 0;

    // mixing-basis codes for the last kappa (n bytes), recomputed when kappa changes
    void* codes = nullptr;
    size_t codes_cap = 0;
    double codes_kappa[3] = {0, 0, 0};
    bool codes_valid = false;

    // FP32 W table for the kappa of the codes (6 n complex), built with them for grids that have
    // fixed-size FP32 plane kernels
    void* wtab_mem = nullptr;
    size_t wtab_cap = 0;
    bool wtab_valid[2] = {false, false};

    // largest automatic LOBPCG block pcx_solve may pick for this plan (0: max_vectors); a batch sets
    // it to the storage it reserved before its workers started
    int block_cap = 0;

    // kernel variant of the A_r path (PCX_VARIANT_*)
    int variant = PCX_VARIANT_AUTO;
    // autotuned choice per precision ([0] FP32, [1] FP64): 0 untuned, -1 / -2 the three- / two-
    // plane fixed-size kernels, 256 / 512 / 1024 generic kernels with that work-group size
    int tuned_nt[2] = {0, 0};
    // the default tuning was looked up (or run) for this precision
    bool tune_checked[2] = {false, false};

    // mode codes (n bytes each) and device kappas of the last multi-k launch
    void* mcodes = nullptr;
    size_t mcodes_cap = 0;
    void* kaps_dev = nullptr;
    size_t kaps_cap = 0;
    std::vector<double> mkaps;
    bool mcodes_valid = false;

    int grow(void** buf, size_t* have, size_t need);
    // inv_eps64 / inv_epsn64 / inv_eps32 / inv_epsn32 / epsn64 / epsn32 inside eps_mem (3n values each)
    void set_eps_pointers();
    // grid description for kappa (computes the mode codes on the plan stream when kappa is new)
    int grid_for(const double kappa[3], Grid* g);
    Grid grid(const double kappa[3]) const;
    // grid description for nk wave vectors in one launch, nvk vectors each ([k][v] order)
    int grid_multi(const double* kappas, int nk, int nvk, Grid* g);
    int check_fits(int precision) const;
    // z = diag(scale) A_r(eps) y, FP64 y and z, FP32 register kernels (in place allowed); false when
    // those kernels do not apply to this grid and choice (nothing launched)
    int precond_mixed(const double kappa[3], const void* y, void* z, const double* scale, int nvec, bool* done);
    int ensure_work(int nvec);
    int apply(int op, const double kappa[3], int precision, const void* in, void* out, int nvec);
};

// eigensolver storage of a plan for a block of b columns (pcx_solve grows it on demand; batches
// reserve it before their worker threads start)
int solver_reserve(Plan* p, int b, bool use32, bool use64);
// the largest block pcx_solve picks for nev bands under these options
int solver_max_block(int nev, const pcx_opts* o);
int gram_chunks_for(long N);
// Before the first solve on a plan whose variant is PCX_VARIANT_AUTO: the autotuner's choice for this
// grid and precision (tuned once per process and grid with nvec vectors, then reused by every plan
// of that grid).  A plan with an explicit variant or choice keeps it.  Not thread-safe per plan.
int autotune_default(Plan* p, const double kappa[3], int precision, int nvec);
// device address of the static scratch array of pcx_apply_Ar_noalloc on `device` (current),
// looked up once per device
int noalloc_setup(int device);

}  // namespace pcx
