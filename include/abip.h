/*
 * abip.h -- C ABI of the MI355X (gfx950) ABIP solver library (libabip.so).
 *
 * ABIP is the ADMM-based interior-point method of Lin, Ma, Ye and Zhang
 * ("An ADMM-Based Interior-Point Method for Large-Scale Linear Programming",
 * arXiv:1805.12344).  It solves the standard-form pair
 *
 *     (P)  min c^T x  s.t.  A x = b, x >= 0
 *     (D)  max b^T y  s.t.  A^T y + s = c, s >= 0          (Section 2)
 *
 * through the homogeneous self-dual embedding Q u = v of Section 3.1, running
 * the simplified ADMM of Algorithm 2 (with the over-relaxation of Section 4.2)
 * inside a path-following loop on the barrier parameter mu, and stopping on the
 * optimality / infeasibility tests of Section 4.1.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers (hipMalloc'd or torch-allocated
 *     memory on the current HIP device) unless the comment says "host".
 *     Matrices are FP64; dense A is row-major m x n; CSR uses int32 indices.
 *   - abip_setup* copies A, b, c into the library's own device memory; the
 *     caller may free its buffers as soon as the call returns.  The returned
 *     work handle owns every device buffer (data copies, the cached factor of
 *     G = I + A A^T, the border of the Schur reduction, the iterate) until
 *     abip_free.
 *   - Output vectors belong to the caller and must hold the stated length.
 *   - Work is enqueued on the stream given at setup (a hipStream_t, passed as
 *     void*; NULL means the null stream).  Entry points that return results in
 *     host structs (abip_info) synchronise that stream before returning.
 *   - Errors are negative return codes; abip_last_error() returns a
 *     thread-local message for the last failing call on that thread.  No
 *     exception or exit() crosses the ABI.  Non-convergence is not an error:
 *     it is reported as status ABIP_MAX_ITERS in abip_info.
 *   - Calls on one work handle must not overlap (they share its buffers).
 */
#ifndef ABIP_H
#define ABIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes (return values) ---------------------------------------- */
#define ABIP_OK            0
#define ABIP_E_INVALID    -1   /* bad argument: null pointer, bad enum value */
#define ABIP_E_DIM        -2   /* bad or unsupported dimensions */
#define ABIP_E_NONFINITE  -3   /* NaN or Inf in A, b or c */
#define ABIP_E_HIP        -4   /* a HIP runtime call failed */
#define ABIP_E_OOM        -5   /* device allocation failed */
#define ABIP_E_STATE      -6   /* call out of order (e.g. backward before solve) */

/* ---- solve status (abip_info.status), Theorems 2.2-2.3 and Section 4.1 --- */
#define ABIP_UNSOLVED            0
#define ABIP_SOLVED              1  /* (x/tau, y/tau, s/tau) meets the three tests */
#define ABIP_PRIMAL_INFEASIBLE   2  /* y / (b^T y) is a certificate (Section 4.1) */
#define ABIP_DUAL_INFEASIBLE     3  /* -x / (c^T x) is a certificate (Section 4.1) */
#define ABIP_MAX_ITERS           4  /* max_admm_iters reached; last iterate returned */

/* ---- enums --------------------------------------------------------------- */
#define ABIP_DENSE_ROWMAJOR  0
#define ABIP_CSR             1

#define ABIP_PREC_FP64       0  /* every step in FP64 */
#define ABIP_PREC_FP32_POLISH 1 /* A and G^{-1} streamed in FP32 (FP64 accumulation,
                                   FP64 iterate), FP64 factor and checks, then FP64
                                   iterations until the FP64 tests pass */

#define ABIP_RESTART_HEURISTIC 0 /* Section 5: scale the smaller of (x_j,s_j), (tau,kappa) */
#define ABIP_RESTART_SQRT      1 /* eq. (update-next-iterate): everything times sqrt(gamma) */

#define ABIP_LIN_AUTO    0  /* dense -> direct, CSR -> CG */
#define ABIP_LIN_DIRECT  1  /* cached FP64 factorization of G = I + A A^T */
#define ABIP_LIN_CG      2  /* Jacobi-preconditioned CG on G, matrix-free (CSR) */
#define ABIP_LIN_TRSV    3  /* dense, one-workgroup engine: the cached Cholesky factor L of G
                               (G = L L^T) kept, and every update solves L z = t, L^T a = z by
                               blocked substitution (64-row blocks through the inverses of L's
                               diagonal blocks) instead of the product with G^{-1}; every LP is
                               streamed from device memory.  ABIP_E_INVALID for the grid engine,
                               CSR input and settings.bb. */

#define ABIP_ENGINE_AUTO   0 /* pick by size */
#define ABIP_ENGINE_WG     1 /* one workgroup owns one LP for the whole solve (persistent) */
#define ABIP_ENGINE_GRID   2 /* one LP spread over the whole GPU, a few kernels per iteration */

/* Run parameters.  eps is used for all five tolerances of Section 4.1
 * (eps_pres = eps_dres = eps_gap = eps_pinf = eps_dinf, as in Section 5). */
typedef struct {
    double  eps;               /* default 1e-6 */
    double  alpha;             /* over-relaxation in [0,2], Section 4.2; default 1.8 */
    double  beta;              /* penalty parameter, mu^0 = beta (Algorithm 2); default 1 */
    double  gamma;             /* mu reduction factor in (0,1); default 0.5 */
    int64_t max_admm_iters;    /* default 1e6 (Section 5) */
    int32_t restart_rule;      /* ABIP_RESTART_*; default heuristic */
    int32_t precision;         /* ABIP_PREC_*; default FP64 */
    int32_t lin_solver;        /* ABIP_LIN_*; default auto */
    int32_t engine;            /* ABIP_ENGINE_*; default auto */
    int64_t fp32_max_iters;    /* FP32 phase length cap before the FP64 polish
                                  starts regardless; default 1e6 */
    double  cg_tol;            /* CG stops when ||r|| <= cg_tol ||rhs|| (sparse engine); default 1e-7 */
    int32_t cg_max_iters;      /* per linear solve; default 500 */
    int32_t block_threads;     /* threads per workgroup for ENGINE_WG (256 or 512, honoured when
                                  the largest m <= 256; larger LPs always use 256); 0 = auto */
    double  adjoint_tol;       /* relative residual that stops the adjoint BiCGSTAB; default 1e-12 */
    int64_t adjoint_max_iters; /* default 2e5; 0 contracts one transposed step of dL/dz (testing) */
    int32_t cg_rule;           /* sparse engine: 0 (default) stops CG at ||r|| <= max(cg_tol ||rhs||,
                                  0.1 ||Q u - v|| / (1 + k)), k the ADMM count; 1: cg_tol alone */
    int32_t use_graph;         /* 1 (default): the dense engines replay hipGraphs (the batched
                                  solve's launches; chunks of 16 iterations of the grid engine),
                                  captured at the first solve of a handle and kept with it;
                                  0: plain stream launches.  Results are bitwise the same. */
    int32_t lds_resident;      /* 1 (default): in the batched engine (256 threads, m <= 256,
                                  n <= 512), an LP whose A and G^{-1} fit in one workgroup's LDS in
                                  the precision of the current phase is solved from LDS with no
                                  global memory traffic per iteration; one whose A fits but not
                                  together with G^{-1} holds A alone in LDS and reads G^{-1} from
                                  device memory once per pass (abip_info.lds_mode says which);
                                  0: every LP streams A and G^{-1} from HBM.  In the sparse engine, 1 lets each workgroup keep its
                                  rows of CSR(A) and CSR(A^T) in LDS for the CG passes when they
                                  fit; 0: the CG passes read them from global memory.  Same
                                  iteration and tests; the sums are formed in a different order,
                                  so results agree to rounding, not bitwise. */
    int32_t bb;                /* 1: Section 4.3's adaptive beta (every engine; in the grid engine
                                  each step of the choice runs while the grid waits, in the
                                  sparse engine inside its launch on each workgroup's rows and
                                  columns): every
                                  outer iteration that starts with ||Q u - v||^2 > mu takes two
                                  probe iterations from its initial point, estimates beta from the
                                  curvature of the three iterates (steepest-descent / minimum-
                                  gradient hybrid, correlation safeguard bb_eps_cor), keeps it,
                                  averages it or redoes the probes from the same point with the
                                  estimate (bb_eps_penalty, at most bb_max_redo redos); the probes
                                  are discarded and count in admm_iters.  0 (default): beta fixed */
    int32_t bb_max_redo;       /* default 10 */
    double  bb_eps_cor;        /* default 0.2 (Section 5) */
    double  bb_eps_penalty;    /* default 0.1 (Section 5) */
    int32_t scale_iters;       /* dense A: rounds of Ruiz equilibration at setup (the scaling of
                                  Section 4.5's remark, which defers to SCS): each round multiplies
                                  D_i by 1/sqrt(max_j |(D_i a_ij) E_j|) and E_j by
                                  1/sqrt(max_i |(D_i a_ij) E_j|); the solver then runs on
                                  (D A E, D b, E c) -- the Section 4.1 tests on that LP -- and
                                  returns x = E x', y = D y', s = s' / E; err_vs_fp64 measures the LP
                                  as given.  abip_backward refuses scaled handles; abip_set_state,
                                  abip_get_state, abip_iterate and abip_apply_iq work in the scaled
                                  variables.  0 (default): no scaling; at most 100.  CSR input:
                                  ABIP_E_INVALID. */
    int32_t sparse_gram;       /* sparse engine: 1 forms G~ = A A^T explicitly at setup (one
                                  workgroup per row gathers the products a_ik a_jk, sorts them by
                                  (j, k), sums each j in k order) when every row has at most 2048
                                  products; each CG iteration is then one product with G~ and one
                                  grid barrier instead of a product with A^T, one with A and two
                                  barriers, but it gathers a 32-byte CG record per entry of G~, so
                                  it pays only when G~ is about as sparse as A.  0 (default): the
                                  two products.  abip_info.gram_nnz says which ran. */
    int32_t grid_mirror;       /* one large dense LP (grid engine): 1 (default) tests at setup (and at
                                  each abip_update_data) whether n is even and the last n/2 columns of
                                  A are exactly the negated first n/2 (A = [A0, -A0], the split of a
                                  free variable into x+ - x-, as in basis pursuit); if so, each column
                                  pass reads A0 alone and treats column j and column j + n/2 together
                                  (their A^T products differ only in sign; their contributions to
                                  A (x+s) and A x are formed as A0 (f_j - f_{j+n/2})), so A is read
                                  half as often.  Same iteration and tests; the row sums are formed
                                  in a different order, so results agree to rounding, not bitwise.
                                  0: every column is read.  abip_info.grid_mirror says which ran. */
} abip_settings;

/* Per-LP result summary (host struct). */
typedef struct {
    int32_t status;            /* ABIP_SOLVED ... ABIP_MAX_ITERS */
    int64_t admm_iters;        /* ADMM updates, all phases */
    int64_t admm_iters_fp64;   /* of which FP64 (polish or plain) */
    int64_t ipm_iters;         /* outer (mu) iterations */
    int64_t cg_iters;          /* total CG iterations (CG solver only) */
    double  pres, dres, gap;   /* relative residuals of Section 4.1 at the last check */
    double  pobj, dobj;        /* c^T x / tau, b^T y / tau at the last check */
    double  tau, kappa, theta, mu;
    double  setup_ms, solve_ms;/* wall time of setup and of the solve (host clock) */
    int64_t colpass_fp32;      /* passes over A streamed in FP32 (updates, restarts, refreshes) */
    int64_t colpass_fp64;      /* passes over A streamed in FP64 */
    double  kernel_ms;         /* duration of the persistent solve launch, HIP events on the
                                  work stream (the same value for every LP of a batch) */
    int64_t ticks_colpass;     /* device wall-clock ticks (100 MHz) the LP's workgroup spent in */
    int64_t ticks_ginv;        /* passes over A, in passes over G^{-1}, and in the whole solve */
    int64_t ticks_total;       /* (one-workgroup engine only; 0 otherwise) */
    int64_t ticks_check;       /* ... in the check sums and tests after each pass over A */
    int64_t ticks_update;      /* ... in the border solve and the y update after each pass over G^{-1} */
                               /* sparse engine (workgroup 0): colpass_fp64 counts updates;
                                  ticks_colpass = column passes (A^T gathers), ticks_ginv = row
                                  passes (A gathers), ticks_check = grid barriers, ticks_update =
                                  reductions of the per-workgroup sums */
    int64_t colpass_lds_fp32;  /* of colpass_fp32 / colpass_fp64: passes that read A from LDS */
    int64_t colpass_lds_fp64;  /* (the rest streamed A from device memory) */
    int64_t ginv_hbm_fp32;     /* passes over G^{-1} read from device memory (streamed LPs, and */
    int64_t ginv_hbm_fp64;     /* LDS-resident LPs that hold A alone in LDS), per precision */
    int32_t lds_mode;          /* LDS-resident phases of the LP: bit 0 FP32 with A and G^{-1} in LDS,
                                  bit 1 FP64 likewise, bit 2 FP32 with A alone, bit 3 FP64 with A alone */
    double  fp32_exit_kkt;     /* ABIP_PREC_FP32_POLISH: relative KKT (largest of the three ratios of
                                  Section 4.1) of the FP32 phase's last iterate, measured with the FP64
                                  data at the handover to the FP64 polish; NaN if no FP32 phase ran */
    double  err_vs_fp64;       /* FP64 recheck of the returned point, computed after the solve by a
                                  separate pass over the FP64 copies of A, b, c (independent of the
                                  iteration's own sums and of the FP32 data): SOLVED / MAX_ITERS: the
                                  largest of pres, dres, gap of (x, y, s) as returned; PRIMAL_INFEASIBLE:
                                  ||A^T y + s|| ||b|| of the returned certificate (b^T y = 1);
                                  DUAL_INFEASIBLE: ||A x|| ||c|| of the returned ray (c^T x = -1).
                                  Each passes the Section 4.1 test when <= eps. */
    double  beta;              /* the last outer iteration's beta (settings.beta unless settings.bb) */
    int64_t bb_probe_iters;    /* of admm_iters: the probe iterations of the beta estimates */
    int32_t bb_estimates;      /* beta estimates taken (redos included) */
    int64_t gram_nnz;          /* sparse engine: entries of the explicit G~ = A A^T, 0 when the CG
                                  multiplies by A^T and A */
    int32_t grid_mirror;       /* 1: the grid engine's column passes read A0 of A = [A0, -A0] alone
                                  (settings.grid_mirror and the pairing test passed); 0 otherwise */
} abip_info;

/* A matrix description.  All pointers are device pointers; abip_setup copies
 * what they point to, so the caller may free them afterwards.
 * CSR (abip_setup only): rowptr nondecreasing with rowptr[0] = 0 and
 * rowptr[m] = nnz, colidx in [0, n) (any order inside a row; repeats add up),
 * finite values; violations return ABIP_E_INVALID / ABIP_E_NONFINITE.  A CSR
 * handle runs the sparse engine: FP64 throughout (settings.precision is not
 * used), the linear step by Jacobi-preconditioned CG on G = I + A A^T
 * (Section 4.4, indirect variant) with settings.cg_tol / cg_max_iters, in one
 * cooperative launch.  abip_apply_iq takes dense handles only (ABIP_E_STATE
 * otherwise). */
typedef struct {
    int32_t m, n;
    int32_t format;            /* ABIP_DENSE_ROWMAJOR or ABIP_CSR */
    const double*  val;        /* dense: m*n entries; CSR: nnz values */
    const int32_t* rowptr;     /* CSR: m+1 offsets (unused for dense) */
    const int32_t* colidx;     /* CSR: nnz column indices (unused for dense) */
    int64_t nnz;               /* CSR only */
} abip_matrix;

typedef struct abip_work abip_work;

/* Fill *s with the defaults listed above.  Returns ABIP_E_INVALID on NULL. */
int abip_default_settings(abip_settings* s);

/* Set up one LP: validate (dimensions, finiteness), copy A, b, c to the
 * library, form the HSD constants bbar = b - A e, cbar = c - e,
 * zbar = c^T e + 1 (eq. bar-b-c-z-re), factor G = I + A A^T once in FP64
 * (Section 4.4; dense) or prepare CG (CSR), and cache the border Z = M^{-1} H
 * and K^{-1} of the Schur reduction of I + Q (Section 4.4, with the theta
 * column kept).  b has length m, c length n.  settings may be NULL (defaults;
 * host pointer).  stream: hipStream_t or NULL.  On success *out owns all of it. */
int abip_setup(abip_work** out, const abip_matrix* A, const double* b, const double* c,
               const abip_settings* settings, void* stream);

/* Set up B independent LPs of any sizes in one work handle (all host arrays of
 * B entries; each A[k], b[k], c[k] as in abip_setup).  Dense only. */
int abip_setup_batch(abip_work** out, int32_t B, const abip_matrix* A,
                     const double* const* b, const double* const* c,
                     const abip_settings* settings, void* stream);

/* Load new data into a dense handle: A[k], b[k], c[k] (host arrays of B
 * entries, each as in abip_setup_batch; B and every LP's m and n must equal
 * those given at setup, else ABIP_E_DIM) replace the handle's LPs, and the whole
 * setup (copies, HSD constants, the factorization of G = I + A A^T and G^{-1},
 * the border) runs again in the buffers the handle already owns: no device
 * allocation, and the batched launch's captured graph is replayed by the next
 * solve.  For serving loops that solve new LPs of fixed shapes.  CSR handles:
 * ABIP_E_STATE.  On an error the handle must be loaded again or freed. */
int abip_update_data(abip_work* w, const abip_matrix* A, const double* const* b, const double* const* c);

/* Run Algorithm 2 from its start point (mu^0 = beta, (y,x,tau,theta) = (0,e,1,1),
 * (s,kappa) = (e,1)) until a test of Section 4.1 passes or max_admm_iters.
 * Outputs (device, caller-owned): x (n), y (m), s (n):
 *   SOLVED / MAX_ITERS: x/tau, y/tau, s/tau;
 *   PRIMAL_INFEASIBLE: y/(b^T y), s/(b^T y), x filled with NaN;
 *   DUAL_INFEASIBLE:   -x/(c^T x), y and s filled with NaN.
 * Any output pointer may be NULL to skip it.  info (host) may be NULL.
 * Requires a work handle made by abip_setup (B = 1). */
int abip_solve(abip_work* w, double* x, double* y, double* s, abip_info* info);

/* Solve every LP of a batch handle in one persistent launch (one workgroup per
 * LP, taken from a device work queue, largest first).  x, y, s, info are host
 * arrays of B entries (device vectors / host structs); entries may be NULL. */
int abip_solve_batch(abip_work* w, double* const* x, double* const* y, double* const* s,
                     abip_info* info);

/* Adjoint of the converged HSD fixed point (project extension, not in the paper).
 * For the loss L(x*) with gradient dL_dx (device, n) at the returned x* = x/tau,
 * solve the adjoint of the linearised ADMM fixed-point map at the final iterate,
 * (I - J^T) lam = dL/dz, by BiCGSTAB; each product with J^T is one transposed
 * ADMM step that reuses the cached factor ((I+Q)^T = I - Q has the same
 * G = I + A A^T).  Then contract with d(Q u)/d(c, b, A).  At the final iterate
 * this equals the adjoint of the central-path system (HSD-log-kkt) there.
 * Outputs (device, caller-owned): dL_dc (n), dL_db (m), dL_dA (may be NULL):
 * m*n row-major for a dense LP; for a CSR LP the nnz values of dL/dA on the
 * stored entries, in the order of the CSR input.  Requires a prior successful
 * abip_solve with status SOLVED (or a state loaded by abip_set_state), else
 * ABIP_E_STATE; ABIP_E_STATE also for a scaled handle (settings.scale_iters).
 * Batch handles: one workgroup per LP, the Krylov vectors in device memory.
 * One large dense LP and CSR LPs: the same recurrence driven from the host,
 * each product over the whole GPU (dense: A and G^{-1} from the cached pools;
 * CSR: products with A and A^T and G^{-1} by CG to max(1e-13, 0.1 adjoint_tol),
 * the border of I - Q computed by CG at the first call).  The CSR engine's CG
 * warm start is kept across the call. */
int abip_backward(abip_work* w, const double* dL_dx, double* dL_dc, double* dL_db,
                  double* dL_dA);

/* Batched form of abip_backward over a batch handle after abip_solve_batch;
 * host arrays of B device pointers (dL_dA entries may be NULL).  LPs whose solve
 * did not end SOLVED get NaN gradients. */
int abip_backward_batch(abip_work* w, const double* const* dL_dx, double* const* dL_dc,
                        double* const* dL_db, double* const* dL_dA);

/* After abip_backward*: BiCGSTAB iterations (host *iters) and final relative
 * residual (host *rel_resid) of LP k's adjoint solve. */
int abip_backward_stats(abip_work* w, int32_t k, int64_t* iters, double* rel_resid);

/* ---- step-level entry points (parity testing and tracing) ----------------
 * These expose the pieces of one inner iteration so that each can be compared
 * with an FP64 reference on identical inputs. */

/* (I+Q)^{-1} w for LP k of the handle (eq. Simple-Update:Affine) using the cached
 * factor: w and out are device vectors of length m+n+2 ordered (y, x, tau, theta).
 * flags bit 0: use the FP32 copies of A and G^{-1} (FP64 arithmetic);
 * flags bit 1: apply (I+Q)^{-T} = (I-Q)^{-1} instead (the adjoint's solve). */
int abip_apply_iq(abip_work* w, int32_t k, const double* win, double* out, int32_t flags);

/* Load an iterate into LP k: y (m), x (n), s (n) device vectors and host scalars
 * tau, kappa, theta, mu.  Marks the LP as mid-solve at that mu; abip_backward
 * may then differentiate this iterate directly. */
int abip_set_state(abip_work* w, int32_t k, const double* y, const double* x, const double* s,
                   double tau, double kappa, double theta, double mu);

/* Read back LP k's current iterate (device outputs y, x, s; host scalars[4] =
 * tau, kappa, theta, mu). */
int abip_get_state(abip_work* w, int32_t k, double* y, double* x, double* s, double* scalars);

/* Run exactly `iters` relaxed ADMM iterations of Algorithm 2 at the current mu
 * on LP k, without tests or restarts (FP64 data unless use_fp32 != 0). */
int abip_iterate(abip_work* w, int32_t k, int64_t iters, int32_t use_fp32);

/* Launch-configuration autotuner (project extension).  Runs `iters` ADMM
 * updates from Algorithm 2's start point with each candidate configuration of
 * the handle's engine, timed with HIP events on the work stream, and keeps the
 * fastest for later solves.  Candidates, in this order:
 *   one-workgroup engine (dense batch), 256 threads unless noted:
 *     0  LDS residency as the settings allow (A and G^{-1} in LDS where they
 *        fit, else A alone where it fits),
 *     1  only LPs whose A and G^{-1} both fit run LDS-resident,
 *     2  every LP streamed from device memory,
 *     -  512 threads, streamed (only when every LP has m <= 256),
 *     -  per-LP mix: policy 0, except that the LPs whose own clock ran faster
 *        in candidate 2 than in candidate 0 are streamed
 *     (settings.lds_resident == 0 leaves candidate 0, and the 512-thread one);
 *   grid engine: about 0.5 / 1 / 2 / 4 workgroups per CU;
 *   sparse engine: the setup's workgroup count (one per 256 rows or columns,
 *     at most one per CU) then 32 / 64 / 128 / 256 workgroups (up to what can
 *     be co-resident; its updates use the solve's CG stopping rule).
 * ms (host, may be NULL) receives each candidate's score, the quantity the
 * choice minimises (up to max_cand): for the grid and sparse engines the time
 * of the launch, for the one-workgroup engine the sum over LPs of each LP's own
 * device-clock time, in ms (a fixed-iteration launch lasts as long as its
 * largest LP alone, while a batch's throughput depends on every LP);
 * *ncand their number, *chosen the kept one: its index in the list above for
 * the one-workgroup engine, its workgroup count for the grid and sparse
 * engines; both may be NULL.  The per-LP LDS modes that a solve then uses are
 * reported in abip_info.lds_mode.  The iterate is reset to the start point.  A
 * configuration change can change the last bits of later results (sums are
 * reduced in a different fixed order), not their correctness. */
int abip_autotune(abip_work* w, int64_t iters, double* ms, int32_t max_cand, int32_t* ncand,
                  int32_t* chosen);

/* The row and column factors D (m) and E (n) of LP k's scaling
 * (settings.scale_iters; all 1 otherwise), copied to device buffers. */
int abip_get_scaling(abip_work* w, int32_t k, double* D, double* E);

/* ---- presolve / postsolve (Section 4.5), host ------------------------------
 * For LPs given in the bounded form  min c^T x  s.t.  A x = b,  l <= x <= w
 * (l_j may be -INFINITY, w_j +INFINITY).  abip_presolve applies the paper's
 * reductions on the host, repeated until none applies, each scan in ascending
 * index order: P3 (l_j > w_j: infeasible), P4 (l_j = w_j: fixed and substituted
 * out), P1 (an empty row: dropped when |b_i| <= 1e-9 (1 + max|b|), else
 * infeasible), P2 (an empty column: at the bound its cost favours; unbounded
 * when that bound is infinite), P6 (a singleton row fixes its variable;
 * infeasible outside the bounds by more than 1e-9 (1 + |bound|)).  The rest is
 * rewritten in the standard form of Section 2 as the paper describes: free
 * variables split (P5), variables bounded only above reflected, lower bounds
 * shifted to 0, each finite upper bound a row with a slack column.  Dependent
 * rows are kept (the linear step uses I + A A^T).  Host arrays: A dense
 * row-major m x n; l, w may be NULL (0 and +INFINITY).  *out receives a record
 * (free it with abip_presolve_free) whenever the return is ABIP_OK; *status is
 * ABIP_PRESOLVE_REDUCED (the standard form has *m_std rows and *n_std columns)
 * or a verdict.  Errors: ABIP_E_DIM, ABIP_E_INVALID (null arrays, NaN bounds),
 * ABIP_E_NONFINITE (non-finite A, b, c). */
#define ABIP_PRESOLVE_REDUCED    0
#define ABIP_PRESOLVE_INFEASIBLE 1
#define ABIP_PRESOLVE_UNBOUNDED  2
typedef struct abip_presolve_t abip_presolve_t;
int abip_presolve(int32_t m, int32_t n, const double* A, const double* b, const double* c, const double* l,
                  const double* w, abip_presolve_t** out, int32_t* status, int32_t* m_std, int32_t* n_std);

/* The standard form (host: A_std m_std x n_std row-major, b_std, c_std; any may
 * be NULL) and the objective constant of the removed part (c^T x = c_std^T x_std
 * + obj_offset).  ABIP_E_STATE after a verdict. */
int abip_presolve_get(const abip_presolve_t* p, double* A_std, double* b_std, double* c_std, double* obj_offset);

/* What the presolve did (host arrays, any may be NULL): *where = the row or
 * column that decided a verdict (-1 otherwise); rows_kept / cols_kept (as many
 * as remain, ascending); row_kind[m]: -1 kept, 0 removed empty, 1 removed
 * singleton; fixed_cols / fixed_vals in fixing order, *nfixed their number. */
int abip_presolve_info(const abip_presolve_t* p, int32_t* where, int32_t* rows_kept, int32_t* cols_kept,
                       int32_t* row_kind, int32_t* fixed_cols, double* fixed_vals, int32_t* nfixed);

/* Postsolve (host): from a solution (x_std, y_std) of the standard form, the
 * original x[n], the multipliers y[m] of the original rows (0 for removed empty
 * rows; for removed singleton rows, in reverse order of removal, the value that
 * makes the reduced cost of the variable it fixed zero) and the reduced costs
 * r[n] = c - A^T y (r_j > 0 at a lower bound, < 0 at an upper bound at an
 * optimum).  ABIP_E_STATE after a verdict. */
int abip_postsolve(const abip_presolve_t* p, const double* x_std, const double* y_std, double* x, double* y,
                   double* r);

int abip_presolve_free(abip_presolve_t* p);

/* ---- allocation-free solve -------------------------------------------------
 * For callers that cannot allocate device memory: tight serving loops that
 * must not call hipMalloc, harnesses that forbid it.  (The call synchronises
 * its stream, so it cannot itself be recorded into a graph capture.)
 * Sets up and solves ONE dense LP (row-major A, m <= ABIP_NOALLOC_MAX_M,
 * n <= ABIP_NOALLOC_MAX_N) exactly as abip_setup followed by abip_solve would
 * (same kernels, same results), but every device buffer it needs is carved out
 * of a fixed 5 MiB region of device memory built into the library (one per GPU,
 * held until the process ends); it calls no hipMalloc / hipFree and creates no
 * stream, event or graph (abip_info.kernel_ms is NaN).  Arguments as for
 * abip_setup (device pointers A->val, b, c; settings and info host, may be
 * NULL; stream as a hipStream_t or NULL) and abip_solve (device outputs x (n),
 * y (m), s (n), each may be NULL).  The call synchronises the stream before it
 * returns.  Errors: ABIP_E_DIM for sizes beyond the limits, ABIP_E_INVALID for
 * CSR input or settings.engine = ABIP_ENGINE_GRID.  All calls on one GPU share
 * the region: calls that overlap in time on the same GPU (other host threads,
 * or other streams of the same process) race and must be serialised by the
 * caller; sequential calls are independent (each clears what it uses). */
#define ABIP_NOALLOC_MAX_M 256
#define ABIP_NOALLOC_MAX_N 1024
int abip_solve_noalloc(const abip_matrix* A, const double* b, const double* c, double* x, double* y, double* s,
                       abip_info* info, const abip_settings* settings, void* stream);

/* Release everything owned by the handle.  NULL is accepted. */
int abip_free(abip_work* w);

/* Thread-local description of the last error on this thread ("" if none). */
const char* abip_last_error(void);

/* Library version string, e.g. "abip-mi355x 0.1 gfx950". */
const char* abip_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ABIP_H */
