/*
 * msp.h -- mirror-symmetric Poisson solver for AMD Instinct MI355X (gfx950).
 *
 * C interface of the library that solves A x = b for a symmetric positive
 * definite matrix A whose unknowns carry s mirror symmetries, following
 * arXiv 2407.05930 ("A multigrid reduction framework for domains with
 * symmetries"):
 *
 *   setup (Sec. 2, eqs. (2.4)-(2.6) and the text after them): the caller
 *     passes the full matrix and the symmetry map; the library extracts the
 *     base-mesh blocks H_j, checks the block structure "block (a,b) of A =
 *     H_{a xor b}" bit for bit, keeps only the shared inner block
 *     A_inn = H_0 plus the per-subsystem outer part (eq. (2.14)), and builds
 *     one preconditioner shared by all 2^s subsystems: the multigrid
 *     reduction hierarchy of Sec. 3.2 (Alg. 2, eqs. (3.13)-(3.15)) on A_inn,
 *     or the FSAI of A_inn (eq. (2.17)), optionally with per-subsystem
 *     low-rank corrections (LRCAMG(k), eq. (2.32); LRCFSAI(k), eq. (2.24)).
 *   solve (Alg. 1): bhat = Q_s b, decoupled PCG on every subsystem and
 *     right-hand side with the shared preconditioner applied to all
 *     2^s * m columns at once (SpMM, eqs. (2.7)-(2.8)), x = Q_s xhat.
 *
 * Conventions
 *   - Matrices are CSR with 64-bit row pointers and 32-bit column indices,
 *     FP64 values, 0-based.  Rows need not be sorted; duplicates are an error.
 *   - The symmetry map is img[i * 2^s + a] = row of image a of base cell i,
 *     for 0 <= i < n_b = n / 2^s and 0 <= a < 2^s.  Bit t of a means
 *     "reflected about mirror plane t"; images compose by XOR; a = 0 is the
 *     base mesh.  It must be a permutation of 0..n-1.
 *   - Right-hand sides and solutions are n x m column-major arrays
 *     (element (row g, rhs j) at [j * n + g]).  2^s * m must not exceed 64.
 *   - Every function returns an msp_status; no C++ exception crosses the
 *     interface.  msp_last_error() returns a thread-local message for the
 *     last failing call on that thread.
 *   - The caller owns every array it passes; setup copies what it needs.
 *     A context is not thread-safe; distinct contexts are independent.
 */
#ifndef MSP_H
#define MSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSP_OK = 0,
    MSP_NOT_CONVERGED = 1,       /* maxit reached; x holds the last iterate */
    MSP_ERR_ARG = -1,            /* bad argument (null, size, layout) */
    MSP_ERR_NOT_SYMMETRIC = -2,  /* A != A^T, or A inconsistent with the map */
    MSP_ERR_BAD_MAP = -3,        /* map is not a permutation */
    MSP_ERR_BREAKDOWN = -4,      /* PCG: p^T A p <= 0 or a non-finite value */
    MSP_ERR_HIP = -5,            /* HIP runtime error */
    MSP_ERR_OOM = -6,            /* host or device allocation failed */
    MSP_ERR_NOT_SPD = -7,        /* a dense Cholesky factorisation failed */
    MSP_ERR_UNSUPPORTED = -8     /* input outside what the library handles */
} msp_status;

/* MSP_MIXED_FP32: FP32 V-cycle (smoother M = omega G^T G formed explicitly),
   FP64 outer PCG and dots.  The dense coarsest inverse is computed in FP64;
   the shared cycle applies it in FP64, the per-subsystem cycle reads its
   inverses rounded to FP32 (sums in FP64).  MSP_MIXED_FP32_BF16G: as
   MSP_MIXED_FP32 but the FSAI factors G, G^T are stored in bfloat16 and the
   smoother is applied factored, G^T (G r), which keeps it SPD.
   MSP_MIXED_BF16: as MSP_MIXED_FP32 but the V-cycle multivectors are stored
   in bfloat16 (FP32 matrices, FP32 arithmetic and accumulation); the outer
   PCG stays FP64. */
enum { MSP_FP64 = 0, MSP_MIXED_FP32 = 1, MSP_MIXED_FP32_BF16G = 2, MSP_MIXED_BF16 = 3 };
/* Preconditioners of the decoupled subsystems A_a = A_inn + diag(sigma_a)
   (Sec. 2, eqs. (2.13)-(2.14)):
   MSP_PC_AMGR: the AMGR hierarchy of A_inn (Sec. 3.2, Alg. 2 and 3) shared by
     every subsystem, applied to all columns at once; low-rank corrections per
     subsystem on top (LRCAMG(k), eq. (2.32)).
   MSP_PC_FSAI: FSAI of A_inn with LRCFSAI(k) corrections (eq. (2.24)).
   MSP_PC_NONE: plain CG.
   MSP_PC_AMGR_SUB: AMGR of every subsystem A_a (Sec. 3.2 applied to each
     decoupled system).  The reduction level is shared: its C/F split forces
     the interface coarse, so P_0 = [W; I] serves every a and the level-0
     residual uses A_a itself.  Below it each subsystem has its own reduced
     operator A_1,a = P_0^T A_a P_0 and levels built from it with the shared
     C/F splits and sparsity patterns (values per subsystem, so one SpMM pass
     still serves all columns); each has its own dense coarsest inverse.
     Optional LRCAMG(k) on top. */
/* MSP_PC_AMGS: the Schur-complement AMG of Sec. 3.1 on every decoupled
     subsystem (eq. (3.12)), base cells ordered inner first (eq. (3.1)):
     t = AMG_K r_I, q = r_G - B^T t, z_G = S_a^{-1} q, z_I = t - K^{-1} B z_G,
     with K, B, C_1 the inner, inner-interface and interface blocks of A_inn,
     AMG_K this library's hierarchy built on K (empty interface), K^{-1} in
     the last step AMG_K again (symmetric; standard PCG) or, with
     amgs_light = 1, G_K^T G_K (the FSAI of K; flexible CG, as the form is
     not symmetric).  S_a^{-1} ~ G_S1^T G_S1 (the FSAI of
     S_G1 = C_1 - B^T G_K^T G_K B, eqs. (3.4), (3.9)) plus, when lrc_k > 0,
     lrc_k low-rank corrections per subsystem toward
     S_AMG,a = C_1 + Sigma_a - B^T AMG_K B (eqs. (3.8), (3.11)).  FSAI
     patterns: the lower triangle of the pattern of K_f^2 and of S_f^3,
     M_f = M without the off-diagonal entries
     |m_ij| < schur_tau sqrt(|m_ii m_jj|).  FP64
     only (other precisions: MSP_ERR_UNSUPPORTED).  The hierarchy that
     msp_num_levels / msp_export_level report is the one of K. */
enum { MSP_PC_AMGR = 0, MSP_PC_FSAI = 1, MSP_PC_NONE = 2, MSP_PC_AMGR_SUB = 3, MSP_PC_AMGS = 4 };

typedef struct msp_ctx msp_ctx;

/* Full matrix A (host memory). */
typedef struct {
    int64_t n;
    const int64_t* rowptr;   /* n + 1 */
    const int32_t* col;      /* rowptr[n] */
    const double* val;       /* rowptr[n] */
} msp_csr;

/* Symmetry map (host memory). */
typedef struct {
    int32_t s;               /* number of mirror symmetries, 0..6 */
    int64_t n_b;             /* base-mesh unknowns, n = n_b << s */
    const int64_t* img;      /* n_b * 2^s */
} msp_symmap;

/* A domain made of copies of one subdomain (host memory): translated or
   reflected copies, any number of them, whose boundary conditions may differ
   from copy to copy.  sub[i * copies + a] is the row of unknown i of the base
   copy in copy a (a permutation of 0..n-1, n = n_b * copies). */
typedef struct {
    int32_t copies;          /* number of copies, >= 1 */
    int64_t n_b;             /* unknowns of one copy */
    const int64_t* sub;      /* n_b * copies */
} msp_copies;

typedef struct {
    int32_t precision;   /* MSP_FP64 | MSP_MIXED_FP32 | MSP_MIXED_FP32_BF16G | MSP_MIXED_BF16 */
    int32_t pc;          /* MSP_PC_AMGR | MSP_PC_FSAI | MSP_PC_NONE | MSP_PC_AMGR_SUB */
    int32_t lrc_k;       /* low-rank correction rank per subsystem, >= 0 */
    int32_t dist;        /* interpolation distance d of Alg. 2 (>= 1) */
    double theta;        /* strength threshold */
    int32_t jacobi0;     /* interpolation smoothing steps at the reduction level */
    int32_t jacobi;      /* interpolation smoothing steps below it */
    int32_t coarse_max;  /* a level with at most this many rows is solved densely */
    int32_t max_levels;
    double max_ratio;    /* stop coarsening when n_{l+1} > max_ratio * n_l */
    double tol;          /* per right-hand side, ||b - A x|| <= tol ||b|| */
    int32_t maxit;
    int32_t device;      /* HIP device ordinal; -1 = host-only setup (no solve) */
    uint64_t seed;       /* seed of the hash priorities and start vectors */
    double trunc0;       /* reduction-level interpolation: each F row drops the weights below
                            trunc0 * (its largest weight magnitude) before the row-sum rescaling;
                            0 keeps every weight of the symbolic pattern; 0 <= trunc0 < 1 */
    int32_t coarse64;    /* mixed modes with MSP_PC_AMGR_SUB: 1 = the per-subsystem coarsest
                            inverses are read in FP64 (the V-cycle's vectors are converted at that
                            level), 0 = rounded to FP32 (default) */
    int32_t nu1, nu2;    /* smoothing sweeps before and after the coarse correction on every level
                            (Alg. 3): s = M y then nu1 - 1 sweeps s += M (y - A s); after the
                            correction nu2 such sweeps.  1..8 and nu1 == nu2 (PCG needs a symmetric
                            cycle; otherwise MSP_ERR_UNSUPPORTED).  Default 1, 1 */
    int32_t amgs_light;      /* MSP_PC_AMGS: 1 = G_K^T G_K in the last step (flexible CG), 0 = AMG_K */
    double schur_tau;        /* MSP_PC_AMGS: pre-filter of the FSAI patterns (default 0.01), >= 0 */
    int32_t true_residual;   /* 1: after the solve the library forms b - A x from x and b and reports
                                ||b - A x|| / ||b|| per right-hand side in msp_stats.relres_true
                                (two transforms, one operator product and one dot more); 0 (default):
                                relres_true is -1 */
    int32_t afsai_nnz;       /* > 0: adaptive FSAI smoothers. Each row's lower pattern grows from the
                                diagonal, one entry per step, to at most afsai_nnz entries. A step adds the
                                candidate j < i (same F/C block at the reduction level) with the largest
                                (A g)_j^2 / a_jj, g the row's current minimiser of g^T A g with g_i = 1.
                                Scores within 1e-10 of the best tie to the smaller column. The static FSAI
                                on that pattern follows. Sec. 5 uses an adaptive FSAI with five entries per
                                row. 0 (default): static FSAI on the strong lower pattern. At most 64 */
    int32_t emin_steps;      /* > 0: every interpolation is refined by this many Jacobi-preconditioned
                                conjugate-gradient steps on tr(P^T A P), its pattern and row sums fixed
                                (energy minimisation, which Sec. 5 applies). 0 (default): none. At most
                                100. The device re-setup (msp_refresh) repeats it */
} msp_opts;

typedef struct {
    int32_t iters;               /* PCG iterations of the slowest column */
    int32_t status;
    double relres_rec[64];       /* per RHS (m <= 64): the relative residual the stopping test
                                    saw, sqrt(sum_a ||rhat_a||^2) / ||b_j|| from the recursively
                                    updated residuals; the true residual ||b - A x|| / ||b|| agrees
                                    with it to rounding (the library does not form A x) */
    int32_t nlev;
    int64_t rows[32];
    int64_t nnz[32];
    double op_complexity;        /* sum_l nnz(A_l) / nnz(A_0) */
    double c_rat;                /* n_1 / n_0 */
    double avg_nnzr;             /* nnz(A_1) / n_1 */
    double t_setup_s;
    double t_solve_s;
    double relres_true[64];      /* per RHS with opts.true_residual = 1: ||b - A x|| / ||b|| formed
                                    after the solve from the returned x; -1 otherwise */
    double t_vcycle_s;           /* GPU time of the V-cycle's kernels in the last solve, summed from the
                                    per-kernel event timers (msp_set_timing); -1 when none of the
                                    V-cycle timers is on */
    int64_t split_drift;         /* after msp_refresh: the points of the reduction level whose C/F decision
                                    a fresh setup of the new matrix would take differently (Alg. 2 redone on
                                    the device: strength, distance-d independent set under the same
                                    priorities); 0 when the kept structure is the fresh one. -1 before any
                                    re-setup, for domains of copies and for d > 3 */
    int64_t split_drift1;        /* after msp_refresh: the same count for level 1 (the standard split of
                                    the new shared A_1: strength, distance-1 independent set with the
                                    strong-dependant count, then the hash, as priority), against the kept
                                    level-1 split; -1 before any re-setup and for hierarchies of fewer than
                                    three levels */
} msp_stats;

/* Fill *o with the defaults: FP64, AMGR, k = 0, d = 2, theta = 0.25,
   jacobi0 = 3, jacobi = 1, coarse_max = 2560, max_levels = 20,
   max_ratio = 0.8, tol = 1e-10, maxit = 1000, device = 0, seed = 240705930,
   trunc0 = 0.05, coarse64 = 0, nu1 = nu2 = 1, amgs_light = 0, schur_tau = 0.01,
   true_residual = 0, afsai_nnz = 0, emin_steps = 0. */
int msp_default_opts(msp_opts* o);

/* Build a context from A and its symmetry map.  Validates the map
   (MSP_ERR_BAD_MAP) and the exact block structure and symmetry
   (MSP_ERR_NOT_SYMMETRIC); outer blocks H_j, j != 0, must be diagonal
   (two-point stencils; otherwise MSP_ERR_UNSUPPORTED).  With device >= 0 the
   hierarchy is uploaded to that GPU and low-rank corrections are computed
   there.  On success *out owns all library memory until msp_free. */
int msp_setup(const msp_csr* A, const msp_symmap* map, const msp_opts* o, msp_ctx** out);

/* AMGR in the original basis for a domain made of copies (Sec. 3 with the
   inner-interface ordering of eq. (3.1); Sec. 3.2: Alg. 2, eqs. (3.13)-(3.15),
   Alg. 3), for the domains the change of basis Q_s cannot take.  The
   interface is every base unknown that, in some copy, is coupled to another
   copy or has a row inside its copy (read in base numbering) that differs
   from the base copy's in pattern or value; every copy then has the same inner
   block.  Alg. 2 runs once, on the base copy's block with that interface, and
   its split is replicated to every copy (the populated interface); level 0 of
   the hierarchy on the whole matrix uses it (P = [W; I], block FSAI over the
   F/C blocks, A_c = P^T A P), the levels below are standard AMG.  The
   context solves the whole system in the caller's ordering through the same
   entry points as msp_setup's (one subsystem: msp_export_outer reports the
   interface over all n unknowns and a zero outer diagonal).  pc must be
   MSP_PC_AMGR, MSP_PC_FSAI or MSP_PC_NONE (MSP_PC_AMGR_SUB needs the Q_s
   subsystems: MSP_ERR_ARG).  Errors as msp_setup's; a copy map that is not a
   permutation is MSP_ERR_BAD_MAP.  On success *out owns all library memory
   until msp_free. */
int msp_setup_copies(const msp_csr* A, const msp_copies* map, const msp_opts* o, msp_ctx** out);

/* Numeric re-setup on the device for a new matrix with the sparsity of the
   setup matrix: d_val (device, rowptr[n] doubles) holds its values in the
   caller's CSR order of the arrays msp_setup was given; positions that held
   zeros then are ignored.  The structure of the setup is kept (the
   interface, every level's C/F split, the smoother patterns, the reduction
   level's truncated interpolation pattern); every value is recomputed on the
   GPU with the setup's formulas: A_inn and the outer diagonal (Sec. 2), the
   interpolation's Jacobi steps and row rescaling (eq. (3.13)), the FSAI
   factors and their damping (eq. (3.14)), the Galerkin products (eq. (3.15))
   as masked sparse products, the per-subsystem levels and the dense
   coarsest inverses (Gauss-Jordan), then the low-rank corrections (Lanczos
   on the device).  For the setup matrix itself, or a positive multiple of
   it, the result is the fresh setup's.  Device work on hip_stream; returns
   when done.  The first call builds the device-side structure (host work
   proportional to the hierarchy's size, once).  The caller keeps symmetry
   and the block structure of the map (not checked).  MSP_ERR_UNSUPPORTED for
   MSP_PC_AMGS and MSP_MIXED_FP32_BF16G; MSP_ERR_NOT_SPD when an FSAI block of
   the new matrix is not positive definite.  After any error part way the
   context's values are invalid: solves return MSP_ERR_ARG until a re-setup
   succeeds.  Sec. 6 names a device-side setup
   as future work; this is its numeric part. */
int msp_refresh(msp_ctx* c, const double* d_val, void* hip_stream);

/* A new context whose reduction level (level 0 of the AMGR hierarchy, Sec. 3.2:
   the Alg. 2 split, the interpolation P = [W; I] of eq. (3.13), the smoother of
   eq. (3.14)) is c's as it stands, values included -- after msp_refresh the
   re-set-up ones, fetched from the device -- and whose levels below it are built
   afresh on the host from c's level-1 operator (eq. (3.15)), as msp_setup builds
   them: standard splits, smoother and interpolation patterns, Galerkin products,
   coarsest inverses. For re-set-up contexts whose coarser splits have moved
   (msp_stats.split_drift1) and cost iterations.
   d_val NULL: the per-subsystem values are computed on the host too, then the
   context is uploaded with new low-rank corrections (c's device; none for a
   host-only c). d_val non-NULL: the device values of the matrix c was last set
   up or re-set up for (msp_refresh's d_val, CSR order of the setup matrix, FP64);
   the new context is uploaded and re-set up from them on the device
   (msp_refresh: every value, the per-subsystem ones and the corrections
   included), work enqueued on hip_stream, the call returning when it is done;
   the host then skips the per-subsystem values, the costly part of the rebuild.
   c stays valid and unchanged (its values are only fetched); *out owns its own
   memory until msp_free. AMGR and per-subsystem AMGR contexts of two or more
   levels, domains of copies included; MSP_ERR_UNSUPPORTED for other
   preconditioners and for d_val with the BF16-G variant, MSP_ERR_ARG after a
   failed re-setup of c, for d_val with a host-only c or a null argument. */
int msp_rebuild_below(msp_ctx* c, const double* d_val, void* hip_stream, msp_ctx** out);

/* Solve for m right-hand sides held in device memory (d_b, d_x: n x m
   column-major FP64, on the context's device), enqueued on hip_stream (NULL
   = the default stream).  Returns when the solve has finished.
   st may be NULL.  The first solve with a given column count times the
   candidate kernel shapes of every V-cycle matrix (lane-group splits; rows
   per wavefront of the per-subsystem coarsest solves) and keeps the fastest;
   with the environment variable MSP_AUTOTUNE_LOG set (not "0") the timings
   are printed to stderr. */
int msp_solve_device(msp_ctx* c, int32_t m, const double* d_b, double* d_x, void* hip_stream,
                     msp_stats* st);

/* Same with host arrays (copies in and out). */
int msp_solve(msp_ctx* c, int32_t m, const double* b, double* x, msp_stats* st);

/* For callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc): msp_solve_device without
   any allocation.  Same arguments, results and errors.  The whole workspace
   (PCG and V-cycle multivectors, partial sums, scalars) is carved from a
   128 MiB device array that every GPU running the library holds until the
   process ends; a system whose workspace for this column count exceeds it
   returns MSP_ERR_UNSUPPORTED (the message gives both sizes).  No kernel
   shapes are timed: the call uses the lane-group splits that an earlier
   msp_solve_device of this context and column count tuned, else the
   defaults.  Per-kernel timers must be off (MSP_ERR_ARG otherwise).  Every
   call on one GPU uses the same array, so calls that overlap on one GPU
   (on different streams, contexts or threads) race; the array keeps the
   last call's contents and each call clears what it needs cleared. */
int msp_solve_device_noalloc(msp_ctx* c, int32_t m, const double* d_b, double* d_x, void* hip_stream,
                             msp_stats* st);

/* Hierarchy introspection (works for host-only contexts). */
int msp_get_stats(const msp_ctx* c, msp_stats* st);
int msp_num_levels(const msp_ctx* c, int32_t* nlev);
/* Sizes of level lev: rows, nnz(A_lev), nnz(P_lev), nnz(G_lev) (0 on the
   coarsest level, which has no P and G). */
int msp_level_sizes(const msp_ctx* c, int32_t lev, int64_t* n, int64_t* nnz_A, int64_t* nnz_P,
                    int64_t* nnz_G);
/* Copy level lev into caller arrays sized from msp_level_sizes.  Any
   pointer may be NULL to skip that part.  cf[i] = 1 for coarse rows;
   P is n x n_{lev+1}; G is the lower-triangular smoother factor;
   omega its damping.  Rows are sorted by column. */
int msp_export_level(const msp_ctx* c, int32_t lev, int8_t* cf, int64_t* A_rp, int32_t* A_ci,
                     double* A_v, int64_t* P_rp, int32_t* P_ci, double* P_v, int64_t* G_rp,
                     int32_t* G_ci, double* G_v, double* omega);
/* MSP_PC_AMGR_SUB only: values of subsystem a (0 <= a < 2^s) on level
   lev >= 1, on the patterns msp_export_level gives for that level (A_v:
   nnz_A values, P_v: nnz_P, G_v: nnz_G; P and G absent on the coarsest
   level) and its damping.  Any pointer may be NULL.  MSP_ERR_ARG for
   another preconditioner, lev = 0 or an index out of range. */
int msp_export_sub_level(const msp_ctx* c, int32_t lev, int32_t a, double* A_v, double* P_v, double* G_v,
                         double* omega);
/* Outer part: sigma[i * 2^s + a] (diagonal of A_out,a) and the interface
   mask (1 for base cells coupled to another image).  With MSP_PC_AMGS both
   are in the library's inner-first order of the base cells. */
int msp_export_outer(const msp_ctx* c, double* sigma, int8_t* interface_mask);
/* pc = MSP_PC_AMGS parity hook: which = 0 B (n_I x n_G), 1 C_1, 2 G_K
   (n_I x n_I), 3 S_G1, 4 G_S1 (n_G x n_G), in the library's inner-first
   order of the base cells (inner, then interface, each by increasing base
   index).  Sizes are written to nrows, ncols, nnz; rp (nrows + 1), ci and v
   (nnz) are filled when not NULL.  MSP_ERR_ARG for another pc or which. */
int msp_export_amgs(const msp_ctx* c, int32_t which, int64_t* nrows, int64_t* ncols, int64_t* nnz, int64_t* rp,
                    int32_t* ci, double* v);
/* Low-rank corrections: number kept per subsystem (kept[a]) and the Ritz
   values found (ritz[a * k + t], k = lrc_k, ascending). */
int msp_export_lrc(const msp_ctx* c, int32_t* kept, double* ritz);

/* Optional per-kernel timers.  Launch classes ("kinds"):
     0 operator (A_inn + outer diagonal) SpMM, 1 per-column dots,
     2 r update with its dots, 3 x and p update, 4 Q_s butterflies, 5 precision casts,
     6 dense coarsest solve, 7 FSAI preconditioner products,
     8 low-rank corrections,
     16 + 8*l + {0: A_l, 1: M_l = omega_l G_l^T G_l (or G_l in the BF16
     variant, where the smoother stays factored), 2: G_l^T (BF16 variant),
     3: R_l = P_l^T, 4: P_l} (V-cycle level l).
   While a kind is on, each of its launches is bracketed by HIP events on
   the solve's stream; totals are folded in when the solve returns.
   msp_set_timing(c, -1, on) switches every kind.  total_bytes sums the
   algorithmic bytes of the timed launches (each operand read or written
   once). */
int msp_set_timing(msp_ctx* c, int32_t kind, int32_t on);
int msp_reset_timing(msp_ctx* c);
int msp_get_timing(const msp_ctx* c, int32_t kind, int64_t* count, double* total_ms, double* total_bytes);
/* Name of the kernel function (template instance, as a profiler lists it;
   "a+b" for a class that launches two kernels) of the last timed launch of
   a kind, NUL-terminated and truncated to len - 1 characters ("" if none). */
int msp_get_timing_kernel(const msp_ctx* c, int32_t kind, char* name, int32_t len);

/* ---------------------------------------------------------------------------
 * Batched solves: many independent systems (different sizes, symmetries and
 * right-hand-side counts) solved together.  Setup builds one context per
 * system (host parts in parallel threads).  A solve starts every system on
 * its own stream, then launches one captured HIP graph that holds a fixed
 * number of PCG iterations of every system on parallel branches.  The
 * iterations are gated on the device: each kernel of a system whose columns
 * have all converged (or that broke down) returns at once, so every system
 * does only the iterations it needs and the host reads the convergence flags
 * once, after the graph.  The graph holds the iterations the previous solve
 * needed (16 before the first solve, or msp_batch_set_chunk's value; at most
 * maxit); a system still active after it continues with one-iteration graph
 * launches up to maxit.  A gated kernel still dispatches its grid, so the
 * graph is captured again when a solve needs more iterations than it holds
 * or leaves two or more unused, and when the vector of m changes.  SpMM
 * kernel shapes are autotuned per matrix and column count.
 * --------------------------------------------------------------------------- */
typedef struct msp_batch msp_batch;   /* opaque; owned by the library until msp_batch_free */

/* nsys systems: A[i], maps[i] (host), common options (device >= 0). */
int msp_batch_setup(int32_t nsys, const msp_csr* A, const msp_symmap* maps, const msp_opts* o, msp_batch** out);
/* m[i] right-hand sides of system i; d_b[i], d_x[i]: device n_i x m[i]
   column-major; work ordered after hip_stream and before it continues;
   st: nsys statistics records or NULL.  Returns the worst status. */
int msp_batch_solve(msp_batch* bt, const int32_t* m, const double* const* d_b, double* const* d_x, void* hip_stream,
                    msp_stats* st);
int msp_batch_size(const msp_batch* bt, int32_t* nsys);
/* Iterations the next solve's graph holds (1..1000; clamped to maxit). */
int msp_batch_set_chunk(msp_batch* bt, int32_t iterations);
/* Graph launches of the last msp_batch_solve (1 when its graph held every
   iteration the systems needed). */
int msp_batch_last_launches(const msp_batch* bt, int32_t* launches);
void msp_batch_free(msp_batch* bt);

/* ---------------------------------------------------------------------------
 * Finite-volume operator and adjoint gradient (differentiable solves).
 *
 * The two-point-flux Poisson matrix -div(kappa grad p) is described by the
 * faces of the base mesh (one kappa per base cell, mirrored to every image):
 *   interior face (base cells a, b):  T = |S| / (d_a/kappa_a + d_b/kappa_b)
 *   Dirichlet wall face of cell a:    T = |S| kappa_a / d_a
 *   mirror-plane face of cell a:      T = |S| kappa_a / (2 d_a), coupling
 *                                     image c with image c xor 2^axis
 *   A_ii = sum of the cell's T, A_ij = -T.
 * For L(p) with p = A^{-1} f and lambda = A^{-T} dL/dp = A^{-1} dL/dp,
 *   dL/df = lambda,  dL/dkappa_i = - lambda^T (dA/dkappa_i) p
 *                               = sum_faces g_f dT_f/dkappa_i,
 *   g_f = -(lambda_u - lambda_v)(p_u - p_v)  (interior and mirror faces),
 *   g_f = -lambda_u p_u                      (wall faces),
 * summed over the images of base cell i and over right-hand sides.
 * --------------------------------------------------------------------------- */
typedef struct {
    int64_t nf;              /* number of faces touching base cells */
    const int64_t* cell_a;   /* base cell of the face */
    const int64_t* cell_b;   /* other base cell (interior faces), else -1 */
    const int8_t* kind;      /* 0 interior, 1 Dirichlet wall, 2 mirror plane */
    const int8_t* axis;      /* mirror faces: the symmetry bit it couples */
    const double* area;      /* |S_f| */
    const double* dist_a;    /* distance cell_a centroid -> face centroid */
    const double* dist_b;    /* same for cell_b (interior faces) */
} msp_faces;

typedef struct msp_fv msp_fv;   /* opaque; owned by the library until msp_fv_free */

/* Copy the face description and the symmetry map; with device >= 0 also
   upload them for msp_fv_kappa_grad. */
int msp_fv_create(const msp_faces* F, const msp_symmap* map, int32_t device, msp_fv** out);
/* Number of nonzeros of the assembled full matrix. */
int msp_fv_nnz(const msp_fv* f, int64_t* nnz);
/* Assemble the full n x n matrix for kappa_base (host, n_b) in the ordering of
   the map: rowptr (n + 1), col and val (nnz) are caller arrays; columns sorted. */
int msp_fv_assemble(const msp_fv* f, const double* kappa_base, int64_t* rowptr, int32_t* col, double* val);
/* The values of msp_fv_assemble's matrix computed on the device: d_kappa_base
   (device, n_b doubles, positive: not checked) gives d_val (device,
   msp_fv_nnz doubles) in msp_fv_assemble's positions, with its arithmetic
   (equal values).  With msp_refresh this rebuilds a solver for a new kappa
   without leaving the device.  Needs an operator created with device >= 0
   (else MSP_ERR_ARG); the first call builds the position map on the host and
   keeps it on the device (4 bytes per nonzero, plus one double per face and
   per base cell) until msp_fv_free; MSP_ERR_UNSUPPORTED for 2^31 or more faces
   or base cells.  Asynchronous on hip_stream. */
int msp_fv_assemble_device(msp_fv* f, const double* d_kappa_base, double* d_val, void* hip_stream);
/* d_grad[i] = dL/dkappa_i for base cell i (device arrays: kappa n_b; lambda and
   p n x m column-major; grad n_b), one thread per base cell gathering over its
   own faces (no atomics), enqueued on hip_stream. */
int msp_fv_kappa_grad(msp_fv* f, const double* d_kappa_base, int32_t m, const double* d_lambda, const double* d_p,
                      double* d_grad, void* hip_stream);
void msp_fv_free(msp_fv* f);

void msp_free(msp_ctx* c);
const char* msp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
