/*
 * pcx.h -- C ABI of the MI355X nullspace-free Maxwell eigensolver.
 *
 * Problem (Huang et al., "Eigenvalue Problems of Discrete Curl Operators on
 * Various Lattices for Simulating Three Dimensional Photonic Crystals",
 * arXiv:1806.10284): the Yee-discretised double-curl generalized eigenproblem
 *     C* C x = lambda B x                                   (Section 3, eq. GEP)
 * on a Bravais lattice with quasi-periodic (Bloch) boundary conditions
 * (Section 1.2, eq. quasi_periodic), reduced to the nullspace-free standard
 * eigenproblem (Section 5.2, Theorem 5.2, eq. NFSEP)
 *     A_r y = Sigma_r Q_r* B^{-1} Q_r Sigma_r y = lambda y,  x = B^{-1} Q_r Sigma_r y,
 * where Q_r Sigma_r = (I_3 (x) T) W is applied with FFTs (Algorithms 5.1, 5.2).
 *
 * Conventions
 * -----------
 * - Every call returns PCX_OK (0) or a negative pcx_status; pcx_last_error()
 *   then returns a thread-local message.  No exception or abort crosses the ABI.
 * - Host pointers are plain C arrays owned by the caller.  "device" pointers
 *   are HIP device allocations owned by the caller (for example torch tensors);
 *   the library never frees them.  The plan owns its own workspaces.
 * - Complex numbers are interleaved (re, im): double2 for PCX_FP64 and float2
 *   for PCX_FP32 (torch.complex128 / torch.complex64).
 * - Real-space field layout ("e-layout", Section 3, vec()): component l of a
 *   3n vector occupies [l*n, (l+1)*n) with index a + n1*(b + n2*c), the x index
 *   a fastest.  Component 1 lives at the Yee point (a+1/2, b, c), 2 at
 *   (a, b+1/2, c), 3 at (a, b, c+1/2).
 * - Fourier layout of the 2n vectors y (Section 5.2, y = [y_1; y_2]): block q
 *   occupies [q*n, (q+1)*n) with the mode index (i*n2 + j)*n3 + k (the column
 *   order of T, eq. T).  Mode (i,j,k) is the plane wave exp(i g.p) with
 *   g = 2 pi M^{-1}(kappa + (i,j,k)), M the lattice rows in grid units
 *   (L1 = (n1,0,0), L2 = (s1,n2,0), L3 = (s2,s3,n3)).
 * - A block of nvec vectors is stored vector after vector (vector v at offset
 *   v * 2n for y-blocks, v * 3n for real-space blocks).
 * - kappa[l] = k . a_l is the Bloch phase per lattice vector (the Bloch wave
 *   vector is 2 pi k); pcx_kappa_from_bloch converts a Cartesian Bloch vector.
 * - All launches go to the HIP stream given at plan creation; calls that return
 *   host results synchronise that stream.  Calls on one plan must not overlap.
 */
#ifndef PCX_H
#define PCX_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pcx_status {
    PCX_OK = 0,
    PCX_E_ARG = -1,      /* bad argument (null pointer, size out of range, bad enum) */
    PCX_E_SIZE = -2,     /* a grid size is not a product of 2, 3, 5 or exceeds PCX_MAX_N */
    PCX_E_LATTICE = -3,  /* degenerate lattice or one violating the primitive-cell condition */
    PCX_E_NOCONV = -4,   /* eigensolver hit max_iter; lambda and residuals are still filled */
    PCX_E_OOM = -5,      /* device allocation failed */
    PCX_E_DEVICE = -6    /* a HIP runtime call failed */
} pcx_status;

enum { PCX_FP64 = 0, PCX_FP32 = 1 };                 /* arithmetic / storage precision */
/* pcx_apply_precond only: complex128 in and out, the scalings in FP64 and the operator between
 * them in FP32 (what the FP64 phase of PCX_MODE_FP32_REFINE applies) */
enum { PCX_FP64_OP32 = 2 };
enum { PCX_EPS_YEE3 = 0, PCX_EPS_VOXEL = 1 };        /* permittivity layouts */
enum { PCX_MODE_FP64 = 0, PCX_MODE_FP32_REFINE = 1, PCX_MODE_FP32 = 2 };
/* kernel variants of the A_r path */
enum { PCX_VARIANT_AUTO = 0, PCX_VARIANT_GENERIC = 1, PCX_VARIANT_THREE_PLANE = 2, PCX_VARIANT_TWO_PLANE = 3,
       PCX_VARIANT_REGISTER = 4 };

#define PCX_MAX_N 256      /* largest supported n1, n2, n3 */
#define PCX_MAX_BLOCK 64   /* largest LOBPCG block */

/* Section 2.2 (eq. transvec): the rotated and angle-corrected lattice. */
typedef struct pcx_geom {
    int n[3];            /* grid n1, n2, n3 */
    int m[3];            /* grid offsets m1, m2, m3 (round half up) */
    int rho[3];          /* 1 where the obtuse case (Case II) was used for m1, m2, m3 */
    int shift[3];        /* signed offsets s = m - rho*n: a2_x = s1 dx, a3_x = s2 dx, a3_y = s3 dy */
    double delta[3];     /* mesh sizes dx, dy, dz */
    double avec_rot[9];  /* row-major 3x3 whose columns are the corrected a1, a2, a3 */
    double cos_angles[3];/* corrected cos(gamma), cos(beta), cos(alpha) */
} pcx_geom;

/* Section 2.2.  avec: row-major 3x3 whose COLUMNS are the user's primitive
 * vectors a~1, a~2, a~3 (any Cartesian frame).  Pure host computation.
 * Errors: PCX_E_ARG (null/n<1), PCX_E_SIZE (n not 2,3,5-smooth or > PCX_MAX_N),
 * PCX_E_LATTICE (dependent vectors, or an offset outside 0 <= m <= n). */
int pcx_geometry(const double avec[9], int n1, int n2, int n3, pcx_geom *out);

/* kappa_l = kvec . a~_l / (2 pi), kvec = the Bloch vector 2 pi k (Section 1.2). Host. */
int pcx_kappa_from_bloch(const double avec[9], const double kvec[3], double kappa[3]);

/* Section 2.3: Omega = [a1 a2 a3]^{-T} [a~1 a~2 a~3]^T, the map from the user's reciprocal
 * frame to that of the rotated, angle-corrected vectors of g (as computed by pcx_geometry from
 * the same avec): a Bloch vector 2 pi k of the user's frame (for example a Brillouin-zone corner
 * point) becomes Omega (2 pi k), and (Omega k) . a_l = k . a~_l, so the phases kappa_l are the
 * same in both frames.  Omega is a rotation when no angle needed correcting.  omega: row-major
 * 3x3.  Pure host computation.  Errors: PCX_E_ARG (null pointer), PCX_E_LATTICE (singular). */
int pcx_omega(const double avec[9], const pcx_geom *g, double omega[9]);

typedef struct pcx_plan pcx_plan;

/* Creates a plan for one grid/lattice.  max_vectors bounds nvec in the apply
 * calls (workspace sizing; 0 selects PCX_MAX_BLOCK).  hip_stream: a hipStream_t
 * (NULL = default stream).  Selects device = the current HIP device.
 * Errors: PCX_E_ARG, PCX_E_OOM, PCX_E_DEVICE. */
int pcx_plan_create(const pcx_geom *g, int max_vectors, void *hip_stream, pcx_plan **out);
void pcx_plan_destroy(pcx_plan *p);

/* B = diag(eps) of Section 3.  eps: HOST array of doubles, 3n values in the
 * e-layout (PCX_EPS_YEE3) or n voxel values broadcast to the three Yee edges
 * owned by each grid point (PCX_EPS_VOXEL).  Every value must be finite and > 0
 * (else PCX_E_ARG).  Copied to the device (1/eps in FP64 and FP32). */
int pcx_plan_set_eps(pcx_plan *p, const double *eps, int layout);

/* Kernel variant used by the apply calls and the eigensolver of this plan (both
 * precisions; replaces an autotuned choice).  PCX_VARIANT_AUTO (default): the
 * fixed-size kernels compiled for common plane shapes (all transform lengths
 * known at compile time; the three field components of a plane staged together
 * in LDS, or two of them with the third held in registers when three planes do
 * not fit) where the grid and precision have them, else the generic kernels.
 * For FP32 64 x 64 planes (n1 a multiple of 8, one wave vector per launch) AUTO takes the register
 * kernels: each 64-point line held by 8 lanes with 8 values each, both radix-8 passes on registers
 * with a wavefront-local LDS exchange between them, one plane component in LDS at a time for the
 * row/column exchange, W formed per mode from FP64 per-plane tables, work-groups plane-major per XCD.
 * PCX_VARIANT_REGISTER: those kernels where they apply, else as AUTO.
 * PCX_VARIANT_GENERIC: runtime-sized kernels for every grid.
 * PCX_VARIANT_THREE_PLANE / _TWO_PLANE: that fixed-size kind where compiled,
 * else the generic kernels.  All compute the same A_r (Section 5.1, Algorithms
 * 5.1 and 5.2) up to rounding order.  Errors: PCX_E_ARG (null plan, unknown
 * variant). */
int pcx_plan_set_variant(pcx_plan *p, int variant);

/* z = A_r y (eq. NFSEP) for nvec vectors.  y, z: device, 2n complex each, in
 * `precision`; y and z may not overlap.  Errors: PCX_E_ARG (nvec out of
 * [1, max_vectors], eps not set), PCX_E_DEVICE. */
int pcx_apply_Ar(pcx_plan *p, const double kappa[3], int precision, const void *y, void *z, int nvec);

/* z = A_r(k) y for nk wave vectors in ONE launch of each matvec kernel: the blocks
 * of all wave vectors of a band-structure path go through the same three kernels, each
 * work-group picking its wave vector's phases and mode codes.  kappas: host, 3*nk
 * doubles; y, z: device, nk*nvec_per_k vectors of 2n complex, ordered [k][v].
 * Requires nk*nvec_per_k <= max_vectors.  Same errors as pcx_apply_Ar. */
int pcx_apply_Ar_multi(pcx_plan *p, int nk, const double *kappas, int precision, const void *y, void *z,
                       int nvec_per_k);

/* u = Q_r Sigma_r y = (I_3 (x) T)(W y) (Section 5.1): 2n -> 3n real space. Device. */
int pcx_apply_QS(pcx_plan *p, const double kappa[3], int precision, const void *y, void *u, int nvec);

/* z = Sigma_r Q_r* u = W^H (I_3 (x) T*) u: 3n real space -> 2n. Device. */
int pcx_apply_QS_adjoint(pcx_plan *p, const double kappa[3], int precision, const void *u, void *z, int nvec);

/* x = B^{-1} Q_r Sigma_r y (Theorem 5.2): the GEP eigenvector for an NFSEP one. Device. */
int pcx_eigvec(pcx_plan *p, const double kappa[3], int precision, const void *y, void *x, int nvec);

/* The dense products of the block eigensolver's Rayleigh-Ritz step (Section 5.2), as the solver
 * runs them (FP64 accumulation; FP64 matrix cores for Hermitian bases of up to 96 columns and for
 * combinations of up to 96 inputs, VALU kernels beyond).  Column blocks on the device: column c of
 * a block of k columns of length len starts at base + c * len, complex in `precision`.
 * pcx_block_gram: g = A^H B into the HOST array g (ka x kb complex128, row-major), synchronous.
 *   herm = 1: B = [A | A2] (b = A2, kb = 2 ka) or B = A (b = NULL, kb = ka), with A^H A2 Hermitian;
 *   only the upper triangle of each ka x ka half is formed and the lower one mirrored from it.
 *   herm = 0: B = b (kb columns), the general product.
 * pcx_block_combine: y = s c, s (ks columns) and y (m columns) on the device, c a HOST array (ks x m
 *   complex128, row-major); synchronous.  y may not overlap s.
 * len <= 2n of the plan is not required: any len >= 1.  Errors: PCX_E_ARG (null pointers, sizes
 * outside [1, 3 PCX_MAX_BLOCK], herm with kb != ka, 2 ka), PCX_E_OOM, PCX_E_DEVICE. */
int pcx_block_gram(pcx_plan *p, int precision, const void *a, int ka, const void *b, int kb, long len, int herm,
                   double *g);
int pcx_block_combine(pcx_plan *p, int precision, const void *s, int ks, const double *c, int m, void *y, long len);

/* LOBPCG preconditioners for A_r = Sigma_r Q_r^* B^{-1} Q_r Sigma_r (Section 5.2, eq. NFSEP).
 *   PCX_PRECOND_NONE:    none.
 *   PCX_PRECOND_DIAG:    D = Sigma_r^{-2} = Lambda_q^{-1} per mode (zero on a masked mode); the
 *                        preconditioned operator is similar to Q_r^* B^{-1} Q_r, whose condition
 *                        number is at most eps_max / eps_min (the bound of Section 5.2).
 *   PCX_PRECOND_INVERSE: D Sigma_r Q_r^* B Q_r Sigma_r D = Sigma_r^{-1} (Q_r^* B Q_r) Sigma_r^{-1},
 *                        the same FFT operator with eps in place of 1/eps: an approximate inverse
 *                        of A_r (exact for constant eps).  The preconditioned operator is similar
 *                        to (Q_r^* B Q_r)(Q_r^* B^{-1} Q_r), whose eigenvalues lie in
 *                        [1, (eps_max + eps_min)^2 / (4 eps_max eps_min)] (Kantorovich), e.g.
 *                        [1, 3.77] for contrast 13 instead of [1, 13]; one extra A_r-type
 *                        application per block column and iteration.  Not in the paper, whose
 *                        inner CG solves run without a preconditioner. */
enum { PCX_PRECOND_NONE = 0, PCX_PRECOND_DIAG = 1, PCX_PRECOND_INVERSE = 2 };

/* z = T y with T the PCX_PRECOND_INVERSE preconditioner D Sigma_r Q_r^* B Q_r Sigma_r D,
 * D = Lambda_q^{-1} per mode (0 on a masked mode): the three A_r kernels with eps in place of
 * 1/eps between two mode scalings.  y, z: device, nvec vectors of 2n complex (complex128 for
 * PCX_FP64 and PCX_FP64_OP32, complex64 for PCX_FP32); z may equal y.  PCX_FP64_OP32 rounds D y
 * to FP32, applies the kernels in FP32 and the outer D in FP64 (on the 64 x 64-plane register
 * kernels: inside them, with no conversion pass; elsewhere through an FP32 copy of 2 x 2n
 * complex64 per vector that the plan keeps).  Same errors as pcx_apply_Ar. */
int pcx_apply_precond(pcx_plan *p, const double kappa[3], int precision, const void *y, void *z, int nvec);

typedef struct pcx_opts {
    int mode;            /* PCX_MODE_FP64 | PCX_MODE_FP32_REFINE | PCX_MODE_FP32 */
    int block;           /* LOBPCG block size >= nev (0: nev + max(2, (nev+4)/5)) */
    int max_iter;        /* total iterations over both phases */
    double tol;          /* converged when ||A_r y - lambda y|| <= tol * lambda (||y|| = 1) */
    double tol_fp32;     /* FP32_REFINE: leave the FP32 phase at this residual */
    unsigned long long seed;  /* start block */
    int precondition;    /* PCX_PRECOND_NONE | PCX_PRECOND_DIAG | PCX_PRECOND_INVERSE (default) */
    int verbose;         /* 1: print one line per iteration to stderr */
    const void *y0;      /* warm start: device, n_y0 vectors of 2n complex128 (e.g. the y of a
                            nearby solve), copied into the first n_y0 columns of the start
                            block; NULL: plane-wave start only */
    int n_y0;            /* 0 <= n_y0 <= block */
    int orthonormalize_w; /* 1: every LOBPCG iteration orthonormalises the new directions W against
                             X on the host before their A_r product (two host synchronisations per
                             iteration); 0 (default): W enters the Rayleigh-Ritz basis as it is, one
                             synchronisation per iteration, and a phase switches to the former only
                             if that basis fails to factor (pcx_stats.orth_fallbacks) */
} pcx_opts;

void pcx_opts_default(pcx_opts *o);

typedef struct pcx_stats {
    int iterations, iterations_fp32;
    long long matvecs, matvecs_fp32;   /* single-vector A_r applications */
    double seconds;                    /* wall time of pcx_solve */
    double seconds_matvec;             /* of which in A_r applications (stream-synchronised) */
    double residual[PCX_MAX_BLOCK];    /* final relative residual per returned band */
    int converged;                     /* bands with residual <= tol */
    long long precond_applies;         /* single-vector applications of Sigma_r Q_r^* B Q_r Sigma_r
                                          (PCX_PRECOND_INVERSE; the A_r kernels with eps for 1/eps) */
    long long precond_applies_fp32;    /* of which in FP32 */
    int restarts;                      /* 1 if the FP64 phase (after the FP32 phase of
                                          PCX_MODE_FP32_REFINE, or started from y0) stagnated with
                                          bands open and the solve was repeated in FP64 alone from
                                          the plain start block (without y0), else 0 */
    unsigned long long floor_mask;     /* bit j set: band j counted as converged with a relative
                                          residual above tol, because its absolute residual reached
                                          the working-precision floor (1024 eps_64 ||A_r|| in FP64)
                                          while tol * lambda_j lies four orders below that floor:
                                          bands that go to zero next to Gamma.  Every other
                                          converged band has residual[j] <= tol. */
    int orth_fallbacks;                /* LOBPCG phases that went on with two host synchronisations
                                          per iteration (W orthonormalised against X first) because
                                          the pencil of the plain basis [X W P] did not factor */
} pcx_stats;

/* Smallest nev positive eigenvalues of C*C x = lambda B x at Bloch phases kappa
 * (Section 5.2: block LOBPCG on A_r, Rayleigh-Ritz in FP64 on the host).
 * lambda: host, nev doubles, ascending.  y_out: device, nev * 2n complex128
 * (orthonormal NFSEP vectors) or NULL.  x_out: device, nev * 3n complex128
 * GEP eigenvectors x = B^{-1} Q_r Sigma_r y (so x* B x = lambda), or NULL.
 * opts may be NULL (defaults), stats may be NULL.
 * Errors: PCX_E_ARG (nev < 1, block > PCX_MAX_BLOCK or > 2n - 2, eps not set),
 * PCX_E_NOCONV (lambda and stats filled), PCX_E_OOM, PCX_E_DEVICE. */
int pcx_solve(pcx_plan *p, const double kappa[3], int nev, const pcx_opts *opts,
              double *lambda, void *y_out, void *x_out, pcx_stats *stats);

/* Independent problems (plans x wave vectors) solved concurrently: one GEP per wave
 * vector (Section 5.2), so the problems of a band structure or of several lattices share
 * nothing but the device.  Problem q (plan-major: the nk[0] wave vectors of plans[0], then
 * those of plans[1], ...) has kappa = kappas[3q..3q+2] and returns lambda[q*nev ..] (host),
 * y_out[q] (device, nev * 2n complex128, or NULL; y_out itself may be NULL) and stats[q]
 * (or stats == NULL).  nworkers host threads (0: min(#problems, 4)), each with its own HIP
 * stream and private copies of the plans' workspaces and 1/eps, take problems in turn, so
 * the device overlaps the kernels of different problems.  opts as for pcx_solve (shared).
 * Every plan must have its permittivity set and live on the current device.  Returns the
 * first error of any problem (PCX_E_NOCONV only if nothing worse happened); all problems are
 * attempted. */
int pcx_solve_batch(pcx_plan *const *plans, int nplans, const int *nk, const double *kappas, int nev,
                    const pcx_opts *opts, int nworkers, double *lambda, void *const *y_out, pcx_stats *stats);

/* Autotuner: times one A_r application of nvec vectors at kappa in `precision` for every
 * kernel variant the plan's grid has (the plan's automatic choice; the three-plane and two-plane
 * fixed-size kernels where compiled for this plane shape and precision; the register kernels for
 * FP32 64 x 64 planes; the generic plane kernels with 256, 512 and, in FP32, 1024 threads) with
 * HIP events on the plan's stream, and keeps the fastest for the plan in that precision.
 * choice_out (may be NULL): 0 the automatic choice, -1 three-plane, -2 two-plane fixed-size
 * kernels, -3 register kernels, else the generic work-group size; ms_out (may be NULL): its time
 * per application
 * in ms.  The candidates are timed after a sustained warm-up, best of two rounds.
 * pcx_solve and pcx_solve_batch run it by default, once per process for each grid and precision they
 * use (nvec = the LOBPCG block), on plans whose variant is PCX_VARIANT_AUTO and that carry no choice
 * yet, and reuse the choice for every later plan of the same grid; pcx_plan_set_variant (any
 * variant, PCX_VARIANT_AUTO included: then the built-in choice) or a choice already made here turns
 * that off for the plan.
 * Allocates and frees two scratch blocks.  Errors: PCX_E_ARG, PCX_E_SIZE, PCX_E_DEVICE. */
int pcx_plan_autotune(pcx_plan *p, const double kappa[3], int precision, int nvec, int *choice_out,
                      double *ms_out);

/* Eigenvalue gradient (not in the paper: first-order perturbation of the
 * Hermitian-definite pencil): for x = B^{-1} Q_r Sigma_r y with ||y|| = 1,
 * d lambda / d B_pp = -|x_p|^2.  grad = sum_t weight[t] * d lambda_t / d B.
 * x: device, nvec * 3n complex128 (as returned by pcx_solve), weight: host nvec
 * doubles, grad: device doubles, 3n (PCX_EPS_YEE3) or n summed over the three
 * components (PCX_EPS_VOXEL).  Overwrites grad. */
int pcx_grad_eps(pcx_plan *p, int nvec, const void *x, const double *weight, void *grad, int layout);

/* The paper's own eigen-driver (Section 5.2): Lanczos on A_r^{-1} = Sigma_r^{-1} M^{-1}
 * Sigma_r^{-1}, M = Q_r^* B^{-1} Q_r, every application of M^{-1} an unpreconditioned CG solve
 * (kappa(M) <= eps_max / eps_min, the bound of Section 5.2), every M product the A_r kernels
 * between two Lambda_q^{-1/2} scalings; full reorthogonalisation of the Lanczos basis (twice
 * classical Gram-Schmidt); the largest Ritz values theta of A_r^{-1} give lambda = 1 / theta.
 * FP64 throughout, single start vector (an exactly repeated eigenvalue appears once per copy
 * that rounding brings in, as in the paper's method). */
typedef struct pcx_lanczos_opts {
    double tol_outer;        /* Ritz pair accepted when beta_j |s_j| <= tol_outer * theta (1e-12) */
    double tol_inner;        /* CG stops at ||r|| <= tol_inner ||rhs|| (1e-13) */
    int max_steps;           /* Lanczos steps, the basis kept for reorthogonalisation (200) */
    int max_cg;              /* CG iterations per inner solve (2000) */
    unsigned long long seed; /* start vector */
} pcx_lanczos_opts;

typedef struct pcx_lanczos_stats {
    int steps;                         /* Lanczos steps taken */
    long long cg_iterations;           /* over all inner solves */
    long long matvecs;                 /* single-vector A_r kernel applications (= cg_iterations) */
    double seconds;
    double residual[PCX_MAX_BLOCK];    /* beta_j |s_j| / theta per returned band */
    int converged;
} pcx_lanczos_stats;

void pcx_lanczos_opts_default(pcx_lanczos_opts *o);

/* lambda: host, nev doubles ascending (nev <= PCX_MAX_BLOCK).  Device workspace of about
 * (max_steps + 6) * 2n complex128, allocated for the call.  Errors: PCX_E_ARG (bad arguments,
 * eps not set), PCX_E_NOCONV (lambda and stats filled with the current Ritz values), PCX_E_OOM,
 * PCX_E_DEVICE. */
int pcx_solve_lanczos(pcx_plan *p, const double kappa[3], int nev, const pcx_lanczos_opts *opts, double *lambda,
                      pcx_lanczos_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): z = A_r y exactly as pcx_apply_Ar computes it (up to
 * rounding order: the fixed-size FP32 adjoint kernels form the mixing W per mode instead of
 * reading the plan's table), with every temporary -- the mode codes of kappa (n bytes) and the
 * matvec workspace (3n complex per vector in `precision`, twice that where the planes take the
 * two-pass path) -- in a static device array of PCX_NOALLOC_SCRATCH_BYTES per device, held from
 * library load to process end.  The call allocates nothing; the plan (created earlier, eps set)
 * supplies the twiddle tables and 1/eps.  nvec is not bounded by max_vectors but by the scratch:
 * a block that does not fit returns PCX_E_SIZE with the largest nvec that does (64^3: 20 vectors
 * in FP32, 10 in FP64).  Calls on one device share the array: calls that overlap on one device
 * (two streams, two threads) race.  The plan's device must be current.  y, z: device, nvec
 * vectors of 2n complex, may not overlap.  Errors: PCX_E_ARG, PCX_E_SIZE, PCX_E_DEVICE. */
#define PCX_NOALLOC_SCRATCH_BYTES (128u << 20)
int pcx_apply_Ar_noalloc(pcx_plan *p, const double kappa[3], int precision, const void *y, void *z, int nvec);

/* The magnetic-field side of the SVD C = P_r Sigma_r Q_r^* (Section 5.1, eq. SVD, Theorem 5.1):
 *
 * pcx_apply_curl: v = C u (adjoint = 0) or v = C^* u (adjoint != 0), the discrete curl of Section 3
 *   as real-space forward (backward) differences with the quasi-periodic wraps of Section 1.2
 *   (C = [[0, -C3, C2], [C3, 0, -C1], [-C2, C1, 0]]).  u, v: device, nvec vectors of 3n complex in
 *   the e-layout; they may not overlap.
 * pcx_hfield: h = P_r y = C Q_r Sigma_r^{-1} y (2n -> 3n): for an NFSEP eigenvector y the
 *   magnetic-field eigenvector of C B^{-1} C^* h = lambda h (same lambda; ||h|| = ||y||), since
 *   P_r^* (C B^{-1} C^*) P_r = A_r.  At kappa in Z^3 the one mode with Lambda_q = 0 has no range
 *   (the Gamma-point SVD: n + 2 zero singular values) and contributes nothing.  y, h: device.
 * pcx_apply_hfield_operator: z = C B^{-1} C^* h (3n -> 3n), the magnetic-field operator.
 *
 * All three use a plan workspace of 5n complex per vector (allocated on growth).  Errors:
 * PCX_E_ARG (null pointer, nvec outside [1, max_vectors], eps not set for the operator),
 * PCX_E_DEVICE. */
int pcx_apply_curl(pcx_plan *p, const double kappa[3], int precision, const void *u, void *v, int nvec,
                   int adjoint);
int pcx_hfield(pcx_plan *p, const double kappa[3], int precision, const void *y, void *h, int nvec);
int pcx_apply_hfield_operator(pcx_plan *p, const double kappa[3], int precision, const void *h, void *z, int nvec);

/* Measurement hook: runs the three kernels of pcx_apply_Ar (plane forward, x-line, plane
 * adjoint) `reps` times, queued back to back on the plan's stream in that order, each kernel
 * recording HIP events at its own start and end (hipExtLaunchKernel), and returns their mean
 * durations in milliseconds in ms_out[0..2].  Same arguments and effect on z as pcx_apply_Ar.
 * Synchronises the stream once, at the end. */
int pcx_time_Ar_kernels(pcx_plan *p, const double kappa[3], int precision, const void *y, void *z,
                        int nvec, int reps, double ms_out[3]);

const char *pcx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PCX_H */
