/*
 * scylla_pdhg.h - C ABI of the MI355X (gfx950) PDHG library.
 *
 * The library solves LP relaxations
 *     min c^T x   subject to   A x (>=, <= or =) b,   l <= x <= u
 * with the Primal-Dual Hybrid Gradient method used as the inner loop of the
 * Scylla heuristic (Mexi et al., arXiv 2307.03466, Algorithm 1 and
 * Section 2.1), stopped by a relative KKT test (Section 2.2), and re-solves
 * such LPs warm-started from the previous primal-dual pair with only the
 * objective changed (Section 2.1, warm start; Algorithm 1, objective update).
 *
 * Conventions for every entry point:
 *   - All pointers in the problem description are HOST pointers and are
 *     only read during the call; the library keeps no pointer after it
 *     returns.  Handles own their device copies.
 *   - Return value: 0 on success (the solve status is reported separately in
 *     scylla_result.status), a negative errno-style code on failure:
 *       -EINVAL (-22) invalid argument (nothing is written to outputs),
 *       -ENOMEM (-12) host or device allocation failed,
 *       -EIO    (-5)  a HIP runtime call failed,
 *       -ENODEV (-19) no usable gfx950 device.
 *     scylla_last_error() returns a thread-local message for the last error.
 *   - No C++ exception crosses this boundary.
 *   - A handle (scylla_batch) must be used by one host thread at a time; its
 *     work is ordered on the HIP stream given at creation.
 *   - Limits: total rows, columns and nonzeros of a handle each < 2^31 - 1.
 *   - Environment: SCYLLA_TUNE_CACHE=<file> makes the autotuner read its
 *     choices (keyed by device architecture, precision, storage format and a
 *     hash of the batch's shape) from that file and append new ones; without
 *     it choices are cached for the life of the process only.
 */
#ifndef SCYLLA_PDHG_H
#define SCYLLA_PDHG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Constraint matrix in CSR form.  row_ptr[0] = 0, row_ptr[m] = nnz,
 * nondecreasing; col_idx strictly increasing within each row and in [0, n);
 * val finite (explicit zeros allowed). */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    const int64_t *row_ptr; /* [m + 1] */
    const int32_t *col_idx; /* [nnz]   */
    const double *val;      /* [nnz]   */
} scylla_csr;

/* One LP: A plus objective c[n], right-hand side b[m], senses[m] in
 * {'G' (>=), 'L' (<=), 'E' (=)}, bounds l[n], u[n] (-inf / +inf allowed;
 * l <= u, l != +inf, u != -inf).  c and b must be finite. */
typedef struct {
    scylla_csr A;
    const double *c;
    const double *b;
    const char *senses;
    const double *l;
    const double *u;
} scylla_lp;

enum { SCYLLA_SENSE_GE = 'G', SCYLLA_SENSE_LE = 'L', SCYLLA_SENSE_EQ = 'E' };

/* Arithmetic / storage precision of the device path.
 * SCYLLA_FP64: values, iterates and accumulation in FP64.
 * SCYLLA_FP32: iterates and accumulation in FP32; the matrix is stored
 *   exactly (small integers packed into the index word, else BF16 when every
 *   value is BF16-exact, else FP32); residual and gap norms, the
 *   termination test and the restart decision stay in FP64. */
enum { SCYLLA_FP64 = 0, SCYLLA_FP32 = 1 };

/* Solve parameters; scylla_params_default() fills the defaults noted. */
typedef struct {
    double tol;           /* relative KKT tolerance, > 0 (1e-4)            */
    int64_t iter_limit;   /* >= 0 iterations per call (100000); 0 = only
                             evaluate the (projected) start point          */
    int32_t precision;    /* SCYLLA_FP64 | SCYLLA_FP32 (SCYLLA_FP32)       */
    int32_t check_period; /* R: iterations between KKT checks, 1..1024 (64) */
    int32_t restarts;     /* 1 = restart scheme on (default), 0 = off      */
    int32_t autotune;     /* 1 = time the tile-size candidates once per
                             handle and keep the fastest (default 1)       */
    double eta;           /* step-size factor in (0, 1) (0.99); the first
                             step's with adaptive steps                   */
    double time_limit_s;  /* <= 0: none (0)                                */
    int32_t fused_window; /* 1 = when every instance fits in LDS, run each
                             check window (check, decision, R iterations)
                             as one kernel, one workgroup per instance
                             (default 1); 0 = always per-pass kernels     */
    int32_t adaptive;     /* 1 = adaptive step size: after the
                             k-th iteration of the call, eta <- min((1 -
                             (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta)
                             with eta_bar = (omega |D_c^-1 dx|^2 +
                             |D_r^-1 dy|^2 / omega) / (2 |dy^T A dx|) of
                             that iteration's move (PDLP's rule; a step is
                             never retried); eta starts at `eta`.  0 =
                             constant eta (default).  The device forms
                             A dx directly (the primal pass hands the dual
                             pass dx = x+ - x, and A x_bar = A x + 2 A dx
                             with an FP64 running A x reset at every
                             check).  The rule lets eta pass the global
                             step bound, so the iteration is not
                             nonexpansive: rounding differences grow about
                             10x per 10 iterations, and FP32 iterates
                             follow the FP64 ones to 1e-4 for about 10
                             iterations, not for 100                      */
    double infeas_tol;    /* > 0 (1e-8): at every check after the first,
                             the moves d = x - x_prev, v = y - y_prev since
                             the previous check end the solve with
                             SCYLLA_PRIMAL_INFEASIBLE when v is a dual ray:
                             rho = b^T v + sum (l lam+ + u lam-) > 0 for
                             lam = proj(-A^T v) onto the bounds' multiplier
                             cones and sqrt(|A^T v + lam|^2 + |v - proj_Y
                             v|^2) <= infeas_tol * rho; with
                             SCYLLA_DUAL_INFEASIBLE when d is a primal ray:
                             c^T d < 0 and the violation of A d against the
                             row cones and of d against the bounds'
                             recession cone (and |Q d|) <= infeas_tol
                             |c^T d| (PDLP's certificates).  0 = off.  The
                             optimality test comes first.                 */
    double stall_tol;     /* > 0: "bounds stalling" ends the solve (Algorithm
                             1's inner loop) with SCYLLA_STALLED when, at
                             stall_checks consecutive checks, neither the
                             primal objective P nor the dual objective D
                             moved by more than stall_tol (1 + |value|)
                             since the previous check; tested after the
                             optimality and infeasibility tests and before
                             the iteration limit.  0 = off (default)       */
    int32_t stall_checks; /* >= 1 checks in a row (3)                     */
    int32_t restart_avg;  /* 1 = restart to the average (PDLP's restart
                             candidates): the running mean of the iterates
                             produced since the last restart (equal
                             weights) is a candidate at every check; when
                             its relative KKT error is below the current
                             iterate's, that error drives the termination
                             test, the restart rule and E_prev, a restart
                             restarts to the mean, and an OPTIMAL or
                             iteration-limit stop returns it (infeasibility
                             and stalling look at the current iterate).
                             Costs a read and a write of the mean per
                             entry per pass and a second check; runs the
                             per-pass path (no fused window).  0 = off
                             (default)                                    */
    int32_t compact;      /* 1 (default): in a batch, once at most half of
                             the tiles the iteration launches run belong to
                             instances still running, the launches are
                             rebuilt over those tiles only (finished
                             instances then cost nothing per iteration;
                             results are unchanged bit for bit; the
                             environment variable SCYLLA_CUT_TRACE=1
                             prints each cut on stderr).  0 = off          */
} scylla_params;

enum {
    SCYLLA_RUNNING = 0,
    SCYLLA_OPTIMAL = 1,          /* relative KKT <= tol                     */
    SCYLLA_ITERATION_LIMIT = 2,  /* iter_limit reached                      */
    SCYLLA_TIME_LIMIT = 3,       /* time_limit_s reached                    */
    SCYLLA_NUMERICAL_ERROR = 4,  /* a residual or gap norm is not finite    */
    SCYLLA_PRIMAL_INFEASIBLE = 5,/* dual ray found (see infeas_tol)         */
    SCYLLA_DUAL_INFEASIBLE = 6,  /* primal ray found: unbounded if feasible */
    SCYLLA_STALLED = 7           /* objective bounds stalled (stall_tol)    */
};

/* Result of one LP solve.  rel_kkt = max(rho_primal, rho_dual, rho_gap):
 *   rho_primal = ||primal residual||_2 / (1 + ||b||_2)
 *   rho_dual   = ||c - A^T y - lambda||_2 / (1 + ||c||_2)
 *   rho_gap    = |P - D| / (1 + |P| + |D|)
 * evaluated in FP64 on the original (unscaled) problem at the returned
 * iterate.  primal_obj = c^T x, dual_obj = b^T y + bound terms. */
typedef struct {
    int32_t status;
    int32_t restarts;
    int64_t iterations;
    double rel_kkt, rho_primal, rho_dual, rho_gap;
    double primal_obj, dual_obj;
    double omega;          /* final primal weight                           */
    double solve_seconds;  /* wall time of the iteration loop               */
    double setup_seconds;  /* handle creation (upload + preconditioning)    */
    double tune_seconds;   /* pass-layout autotuning done by this call (the
                              first solve of a handle; 0 afterwards)         */
} scylla_result;

/* Fills *p with the defaults listed in scylla_params.  Returns 0, or
 * -EINVAL if p is NULL. */
int scylla_params_default(scylla_params *p);

/* Thread-local message describing the last failed call ("" if none).  The
 * string stays valid until the next library call on the same thread. */
const char *scylla_last_error(void);

/* Checks an LP description without touching the GPU (Algorithm 1 input form
 * with senses G/L/E).  Returns 0 or -EINVAL (message in scylla_last_error). */
int scylla_validate_lp(const scylla_lp *lp);

/* One-shot solve (Algorithm 1 inner loop): creates a device copy of the LP,
 * runs PDHG from the projection of (x0, y0) onto the bounds and the dual
 * sign cone (x0 / y0 may be NULL: 0 is used), and writes the last iterate to
 * x_out[n], y_out[m] (host) for every status.  On a negative return nothing
 * is written.  res may not be NULL. */
int scylla_pdhg_solve(const scylla_csr *A, const double *c, const double *b, const char *senses,
                      const double *l, const double *u, const scylla_params *p,
                      const double *x0, const double *y0, double *x_out, double *y_out,
                      scylla_result *res);

/* ------------------------------------------------------------ handles
 * A batch holds `count` independent LPs resident on the device (the problem
 * data, preconditioner and warm state (x, y, omega) per instance).  All
 * instances are iterated together in one sequence of launches; finished
 * instances stop updating while the others continue.  count = 1 is the
 * single-LP handle used for objective-only re-solves. */
typedef struct scylla_batch scylla_batch;

/* Uploads and preconditions `count` LPs (precision fixed for the handle).
 * hip_stream: a hipStream_t cast to void* on which all work of the handle is
 * ordered, or NULL to let the library create one. */
int scylla_batch_create(const scylla_lp *lps, int32_t count, int32_t precision, void *hip_stream,
                        scylla_batch **out);
void scylla_batch_destroy(scylla_batch *h);

/* Replaces the objective of instance `inst` by c_hat[n_inst] (host, finite).
 * The original objective passed at creation is kept for blending. */
int scylla_batch_set_objective(scylla_batch *h, int32_t inst, const double *c_hat);

/* Pump objective update on the device (Algorithm 1, objective update):
 *   c_hat_j = a * kappa * c_j + (1 - a) * g_j
 * with c the objective given at creation, g_j = +1 if bit j of xhat_bits is 0
 * (rounded value at its lower bound), -1 if it is 1 (at its upper bound), and
 * g_j = 0 where bit j of int_bits is 0 (continuous variable).  Bits are
 * little-endian within each byte; each array holds ceil(n_inst / 8) bytes
 * (host).  int_bits may be NULL (all integer).  Typically a = 0.9^K and
 * kappa = sqrt(|I|) / ||c||_2. */
/* Diagonal Hessian of instance `inst`'s objective: the handle then solves
 * min c_hat^T x + x^T diag(q) x / 2 (the diagonal-Hessian QPs Section 5
 * proposes for PDHG): the primal step solves each coordinate's proximal
 * problem exactly, x+ = proj_[l,u]((x + t D_c^2 (A^T y - c_hat)) /
 * (1 + t D_c^2 q)), and the KKT test uses the reduced cost c_hat + Q x - A^T y,
 * the primal objective + x^T Q x / 2 and the dual objective - x^T Q x / 2.
 * q: [n_inst] host, finite and >= 0, or NULL (zero).  Returns 0 or
 * -EINVAL. */
int scylla_batch_set_quadratic(scylla_batch *h, int32_t inst, const double *q);

int scylla_batch_set_blend(scylla_batch *h, int32_t inst, const uint8_t *xhat_bits,
                           const uint8_t *int_bits, double a, double kappa);

/* Sets the start point of instance `inst` from host x0[n_inst] / y0[m_inst]
 * (either may be NULL: keep the current one); it is projected on entry.
 * omega0 > 0 also sets the primal weight. */
int scylla_batch_set_start(scylla_batch *h, int32_t inst, const double *x0, const double *y0,
                           double omega0);

/* Sets the start point of every instance from DEVICE memory (the warm start
 * from a primal-dual pair of Section 2.1, handed over without a host copy):
 * x0_dev [n_total] and y0_dev [m_total] are FP64 device buffers holding the
 * concatenated vectors in instance order (either may be NULL: keep the
 * current one), read on the handle's stream (so the caller orders their
 * production before it, e.g. by creating the handle on the producing
 * stream); they are converted to the path precision and projected on
 * entry.  omega0: [count] host values, > 0 sets that instance's primal
 * weight, or NULL.  The buffers are checked on the device first: a NaN in
 * x0 or a non-finite value in y0 returns -EINVAL with nothing written.  The
 * call has finished reading them when it returns.  Returns 0, -EINVAL or
 * -EIO / -ENOMEM. */
int scylla_batch_set_start_device(scylla_batch *h, const double *x0_dev, const double *y0_dev,
                                  const double *omega0);

/* Runs PDHG on every instance of the batch.  warm = 0: every instance starts
 * from 0 (projected) with the primal weight from its data; warm = 1: every
 * instance continues from its current (x, y, omega) (the last solve's, or
 * what scylla_batch_set_start installed).  results[count] receives one
 * record per instance. */
int scylla_batch_solve(scylla_batch *h, const scylla_params *p, int32_t warm,
                       scylla_result *results);

/* Copies instance `inst`'s current iterate to host x[n_inst] / y[m_inst] as
 * FP64 (either may be NULL). */
int scylla_batch_get_solution(scylla_batch *h, int32_t inst, double *x, double *y);

/* Restart to the average (scylla_params.restart_avg): copies instance
 * `inst`'s running mean of the iterates since its last restart, as it stood
 * when the last solve stopped, to host x[n_inst] / y[m_inst] as FP64 (either
 * may be NULL; meaningful once an iterate was produced since the last
 * restart).  -EINVAL if no solve with restart_avg has run on the handle. */
int scylla_batch_get_average(scylla_batch *h, int32_t inst, double *x, double *y);

/* Copies the concatenated primal iterate of all instances (sum of n_inst
 * values, instance order) to host memory as FP64 in one transfer. */
int scylla_batch_get_x_all(scylla_batch *h, double *x_all);

/* Device buffers of the current iterates (for zero-copy consumers).  *x and
 * *y receive device pointers to the concatenated primal / dual iterates,
 * *elem_bytes 4 (FP32 handle) or 8 (FP64 handle).  The pointers stay valid
 * until the handle is destroyed. */
int scylla_batch_device_iterates(scylla_batch *h, void **x, void **y, int32_t *elem_bytes);

/* Shape of the handle: total rows, columns, nonzeros, instance count and the
 * matrix storage format chosen (0 packed integers, 1 BF16, 2 FP32, 3 FP64). */
typedef struct {
    int32_t count, precision, format;
    int32_t fused_eligible; /* 1 if every instance fits the fused window  */
    int64_t m_total, n_total, nnz_total;
    int32_t row_chunk, col_chunk; /* tile sizes in use (nonzeros per tile) */
    int32_t long_rows, long_cols; /* rows / columns split over several tiles */
    int32_t row_blocks, col_blocks; /* layout of each pass: 0 normal, 2, 4 or
                                       8 gather blocks, -1 LDS-staged, -6
                                       direct staged                         */
    int32_t row_staged_nnz, col_staged_nnz; /* staged tile size (nonzeros)  */
    int32_t row_staged_variant, col_staged_variant; /* staged kernel variant
                                       bits: 1 operand prefetch, 2 sub-tiles
                                       of 8192 nonzeros (else 4096)         */
    int32_t row_sliced, col_sliced; /* instances of an LDS-staged pass whose
                                       gathered vector is processed in LDS
                                       slices (partial sums + row combine)   */
    int32_t row_slices, col_slices; /* most slices of such an instance (each
                                       has ceil(vector / LDS room) slices)  */
    int32_t row_half_lds, col_half_lds; /* staged workgroups limited to half
                                       the LDS (two per CU)                  */
    int32_t row_tile_threads, col_tile_threads; /* threads per workgroup of
                                       the normal / gather-blocked tiles
                                       (256, or 1024 for ept -8 / -16)       */
    int32_t row_direct, col_direct; /* instances of a direct staged pass
                                       (blocks -6): whole gathered vector in
                                       LDS, rows reduced in registers        */
    int32_t row_cached, col_cached; /* 1: the pass reads the matrix with
                                       plain (cacheable) loads, 0: with
                                       non-temporal loads                    */
} scylla_batch_info;
int scylla_batch_get_info(scylla_batch *h, scylla_batch_info *info);

/* Matrix load policy of the iteration passes (FP32 path; the autotuner
 * chooses it by timing both passes together, a pinned layout starts with
 * 0): 1 = plain loads, which the device's last-level (Infinity) cache
 * keeps across iterations when an iteration's data fits in it, 0 =
 * non-temporal loads that stream past the caches.  Results do not depend
 * on it.  Call after scylla_batch_set_layout (which resets it).  Returns 0,
 * or -EINVAL (NULL handle, flags not 0 or 1). */
int scylla_batch_set_cached_loads(scylla_batch *h, int32_t row_cached, int32_t col_cached);

/* ------------------------------------------------------ pump loop
 * Fix-and-propagate rounding on the host (Section 2.3): integer variables
 * are fixed one at a time (increasing distance to the nearest integer, ties
 * by index) to the reference value rounded half down and clamped to the
 * current domain, each fixing followed by activity-based propagation of the
 * rows containing the variable (first-in first-out); a row whose activity
 * bounds exclude b, or whose derived bounds would empty a domain, is
 * ignored for the rest of the call.  Continuous variables take the
 * reference value projected onto their domain.  x_ref, x_hat: [n] host;
 * is_int: [n] 0/1 or NULL (all integer); info[0] = 1 if every row holds at
 * x_hat within 1e-6 (1 + |b_i|), info[1] = number of ignored rows.  Host
 * only (no GPU needed).  Returns 0 or -EINVAL. */
int scylla_fix_propagate(const scylla_lp *lp, const uint8_t *is_int, const double *x_ref, double *x_hat,
                         int32_t *info);

/* One record per (round, instance) of scylla_batch_pump and
 * scylla_batch_pump_ex (round = 0: the instance took no part in that round). */
typedef struct {
    int32_t round;          /* K, 1-based                                     */
    int32_t status;         /* status of this round's PDHG solve              */
    int64_t iterations;     /* PDHG iterations of this round                  */
    double rel_kkt;         /* relative KKT at the returned iterate           */
    int32_t lp_feasible;    /* the PDHG iterate itself is MIP-feasible (1e-6) */
    int32_t xhat_feasible;  /* the rounded point satisfies every row (1e-6)   */
    int32_t ignored_rows;   /* rows ignored by fix-and-propagate              */
    int32_t perturbed;      /* the rounding repeated an earlier one and was
                               perturbed (scylla_batch_pump_ex only)          */
    double xhat_obj;        /* c^T x_hat with the original objective          */
    double solve_seconds;   /* device solve of the round (the instance's
                               group of the batch), copy-out and checks      */
    double round_seconds;   /* the group's round: solve, copy-out, rounding,
                               objective update                             */
    double tune_seconds;    /* pass-layout autotuning inside the round's
                               solve (the handle's first solve only)         */
    double rounding_seconds; /* host rounding of the round (the instance's
                                group, thread pool): fix-and-propagate,
                                checks, history, next objective              */
    int32_t group;          /* device solve group of the instance (0 or 1,
                               see scylla_pump_params.pipeline); its round
                               timings are the group's                      */
    int32_t pad;
} scylla_pump_record;

/* MIP-feasibility of every instance's current primal iterate x (Algorithm 1
 * returns the PDHG point itself when it is already feasible for the MIP,
 * Section 2.1), evaluated on the device: every row holds within
 * tol (1 + |b_i|) with an FP64 activity sum_j a_ij x_j, every x_j lies within
 * tol of [l_j, u_j] and every integer x_j within tol of an integer;
 * a non-finite value fails.  The pump loops make this test every round with
 * tol = 1e-6.  is_int: [n_total] 0/1 (instance order) or NULL (all
 * integer); feasible: [count] receives 1 or 0.  Returns 0, -EINVAL (NULL
 * handle or feasible, tol not finite and > 0) or -EIO (HIP error). */
int scylla_batch_mip_feasible(scylla_batch *h, const uint8_t *is_int, double tol, int32_t *feasible);

/* scylla_batch_mip_feasible for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same test and outputs, with its device flags (integer
 * flags, row and column violations, per-instance results) in a static
 * device array of 16 MiB that each GPU holds from the first call on it
 * until the process ends, so it calls no hipMalloc, hipFree or other
 * allocating routine (host or device).  The batch must need at most that
 * much: 2 n_total + m_total + count bytes, each region rounded up to 256
 * bytes; larger batches fail with -EINVAL and nothing is written.  is_int
 * is copied to the device as given (nonzero = integer).  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU (other host
 * threads, other streams) race; each call overwrites every flag it reads.
 * Returns 0, -EINVAL (NULL handle or feasible, tol not finite and > 0, batch
 * too large) or -EIO (HIP error). */
int scylla_batch_mip_feasible_static(scylla_batch *h, const uint8_t *is_int, double tol, int32_t *feasible);

/* Batched fix-and-propagate on the device (one workgroup per instance): a
 * parallel form of the rounding of Section 2.3.  Per instance, the integer
 * variables are taken in the same order as scylla_fix_propagate (ascending
 * distance of x_bar_j to the nearest integer, ties by lower index), K unfixed
 * ones at a time: they are fixed together to x_bar_j rounded half down and
 * clamped to their domains, then propagation runs in synchronous rounds
 * (at most max_rounds per batch): every row of a variable that changed is
 * evaluated against the domains at the start of the round (activity bounds;
 * derived bounds, integer ones rounded inward with 1e-9 slack; a row whose
 * activity bounds exclude b by more than 1e-9 (1 + |b_i|) or whose bound
 * empties a domain is ignored for the rest of the call); per variable the
 * derived bounds that change it (integer: any tightening; continuous: by
 * more than 1e-9 (1 + |bound|), or from infinite to finite) combine by max
 * (lower) and min (upper); if the combined domain is empty by more than
 * 1e-9 (1 + |upper|), every row that would change that variable is ignored
 * and the combination is taken again without them; a crossing within that
 * tolerance sets both bounds to max(upper, old lower).  Variables left
 * unfixed take x_bar_j projected onto their domain.  The result does not
 * depend on the order of the rows and is exact (FP64, sums in row order); K
 * = 1 gives the sequential procedure's result wherever no row is ignored on
 * pure-integer problems.
 *   is_int:     [n_total] 0/1 or NULL (all integer).
 *   xbar:       [n_total] finite host values, or NULL for every instance's
 *               current primal iterate x (path precision, widened to FP64).
 *   K >= 1, max_rounds >= 1.
 *   xhat:       [n_total] receives the roundings.
 *   info:       [2 * count] receives per instance (every row holds at x_hat
 *               within 1e-6 (1 + |b_i|): 1 / 0, number of ignored rows).
 *   ignored:    [m_total] or NULL, receives 1 for every ignored row.
 * Returns 0, -EINVAL (NULL handle / xhat / info, K or max_rounds < 1, a
 * non-finite xbar) or -ENOMEM / -EIO.  A non-finite iterate (xbar NULL)
 * is not rejected: its non-finite integer entries come last in the fixing
 * order (before any continuous variable) and take the lower end of their
 * domain, and a row whose activity at the rounding is not finite counts as
 * violated.  Every round is
 * a few dependent device-memory round trips, so max_rounds also bounds the
 * run time of a call.  The problem's FP64 rows and column incidence are
 * copied to the device on the first call and kept. */
int scylla_batch_fix_propagate(scylla_batch *h, const uint8_t *is_int, const double *xbar, int32_t K,
                               int32_t max_rounds, double *xhat, int32_t *info, uint8_t *ignored);

/* Feasibility-pump-like loop of Algorithm 1 on every instance of the batch,
 * with all `rounds` rounds run: round 1 solves with the original objective
 * from the projected origin; after round K every instance is rounded on
 * the host by fix-and-propagate (thread pool of `threads` workers, 0 = one
 * per hardware thread) and its objective is replaced on the device by
 * alpha^K sqrt(|I|)/||c|| c + (1 - alpha^K) * (L1-distance gradient to the
 * rounding); round K + 1 is warm-started from (x, y, omega) of round K.
 * Cycle perturbation and early exit are not performed.  is_int: [n_total]
 * 0/1 (instance order) or NULL (all integer; general integers strictly
 * inside their bounds are rejected with -EINVAL when met).  records:
 * [rounds * count] (round-major).  xhat_out: [n_total] or NULL, receives per
 * instance the rounding of the first round whose rounding is feasible, else
 * the last round's.  An instance whose solve ends with
 * SCYLLA_NUMERICAL_ERROR is not rounded and is not solved again (its record
 * of that round carries the status; later records stay zero). */
int scylla_batch_pump(scylla_batch *h, const scylla_params *p, const uint8_t *is_int, int32_t rounds,
                      double alpha, int32_t threads, scylla_pump_record *records, double *xhat_out);

/* Options of the complete Algorithm 1 loop (scylla_batch_pump_ex). */
typedef struct {
    int32_t rounds;           /* most rounds K per instance, >= 1             */
    int32_t eps_schedule;     /* 1: round K solves to eps(K), eps(1) = eps1,
                                 eps(K+1) = max(beta eps(K), eps_floor)
                                 (Section 2.2); 0: params->tol every round     */
    double eps1, beta, eps_floor;
    double alpha;             /* objective-update factor, in [0, 1)           */
    int64_t total_iter_limit; /* cumulative PDHG iterations per instance over
                                 all rounds (0: none); a round may run at most
                                 min(params->iter_limit, what is left), and an
                                 instance with nothing left stops             */
    int32_t early_exit;       /* 1: an instance stops at the first round whose
                                 PDHG iterate or rounding is MIP-feasible      */
    int32_t perturb;          /* 1: a rounding equal to an earlier rounding of
                                 the instance is perturbed                    */
    uint64_t seed;            /* seed of the perturbation counts              */
    int32_t threads;          /* host rounding workers, 0 = one per hardware
                                 thread                                       */
    int32_t distance;         /* 1: L1 distance (Algorithm 1; linear
                                 objective; default); 2: L2 distance
                                 (Section 5: QP objective alpha^K kappa c^T x
                                 + (1 - alpha^K) |x_I - x_hat_I|^2, solved as
                                 c_hat = alpha^K kappa c - 2 (1 - alpha^K)
                                 x_hat, Hessian 2 (1 - alpha^K) on I; general
                                 integers need no auxiliary variables)        */
    int32_t pipeline;         /* 1: two groups of instances (split at half
                                 the nonzeros) alternate on the device, so
                                 one group's host rounding runs during the
                                 other group's solve; results equal those of
                                 0 (default: one group, rounds in lockstep).
                                 Pays off only when half the batch keeps the
                                 GPU as busy as the whole: a batch whose
                                 passes are one wave of workgroups takes
                                 about as long per iteration for half of it */
    int32_t fp_batch;         /* 0: rounding by scylla_fix_propagate's
                                 sequential procedure on the host (default);
                                 K >= 1: by the batched procedure of
                                 scylla_batch_fix_propagate on the device, K
                                 variables per batch (needs pipeline = 0)     */
    int32_t fp_max_rounds;    /* propagation rounds per batch of the device
                                 rounding, >= 1 (default 1000)                */
} scylla_pump_params;

/* Per-instance outcome of scylla_batch_pump_ex. */
typedef struct {
    int32_t found_kind;     /* 0 none, 1 the PDHG iterate, 2 the rounding     */
    int32_t found_round;    /* round of the first find, 0 if none             */
    int32_t rounds_run;     /* rounds in which the instance was solved        */
    int32_t perturbations;  /* roundings that were perturbed                  */
    int64_t iterations;     /* PDHG iterations over all its rounds            */
    double obj;             /* c^T of the returned point                      */
} scylla_pump_outcome;

/* Defaults of the paper's configuration: 20 rounds, eps schedule on
 * (0.01, 0.98, 1e-8), alpha 0.9, no cumulative limit, early exit and
 * perturbation on, seed 0, threads 0, L1 distance, one group. */
int scylla_pump_params_default(scylla_pump_params *o);

/* The complete outer loop of Algorithm 1 on every instance of the batch:
 * each round solves all unfinished instances together on the device
 * (warm-started from the previous round, round 1 from the projected origin),
 * copies the iterates to the host, and per instance (thread pool): returns
 * the PDHG iterate if it is MIP-feasible (rows within 1e-6 (1 + |b_i|),
 * bounds and integrality within 1e-6); else rounds it by fix-and-propagate
 * and returns the rounding if every row holds; else, when the rounding
 * equals one of the instance's earlier roundings (after their
 * perturbation), flips the T binary variables with the largest
 * |x_bar_j - x_hat_j| (ties by lower index) to their other bound, where
 * T = 10 + (SplitMix64(seed, instance * 2^20 + K) mod 21) and SplitMix64
 * (Steele, Lea and Flood 2014) is the output for the state
 * seed + (counter + 1) * 0x9E3779B97F4A7C15 (cycle perturbation, Algorithm 1
 * and Section 2.3); then replaces the instance's objective on the device by
 * alpha^K sqrt(|I|)/||c|| c + (1 - alpha^K) * (L1-distance gradient to the
 * rounding).  With early_exit = 0 every instance runs all rounds and the
 * first find is still reported.  The perturbation needs binary integer
 * variables (-EINVAL otherwise, when it is needed); general integers
 * strictly inside their bounds are rejected as in scylla_batch_pump.
 * is_int: [n_total] 0/1 or NULL (all integer).  records: [rounds * count]
 * round-major, or NULL.  outcome: [count] or NULL.  x_out: [n_total] or NULL,
 * receives per instance the point of its first find, else its last
 * rounding before perturbation (zeros if it ran no round).  An instance
 * whose solve ends with SCYLLA_NUMERICAL_ERROR leaves the loop unrounded
 * (found_kind 0).  params supplies
 * precision, check period, restarts, eta, per-round iteration and time
 * limits and, without the schedule, the tolerance.  Returns 0, -EINVAL or
 * -EIO (device error). */
int scylla_batch_pump_ex(scylla_batch *h, const scylla_params *params, const uint8_t *is_int,
                         const scylla_pump_params *opt, scylla_pump_record *records,
                         scylla_pump_outcome *outcome, double *x_out);

/* Pins the tile plan of both passes instead of autotuning it.  The
 * floating-point summation order (so the last bits of the iterates) is a
 * function of the plan; a pinned plan makes results reproducible across
 * runs and devices.  *_blocks: 0 = normal layout, 2, 4 or 8 = gather-blocked
 * layout with that many blocks (one per four XCDs, per XCD pair or per XCD), -1 = LDS-staged
 * layout (instances whose gathered vector fits in LDS are processed with
 * that vector copied to LDS, in tiles of about 32768 nonzeros), -2 = the
 * LDS-staged layout plus LDS slices (instances whose gathered vector is up
 * to four times too long are processed one equal slice of it at a time,
 * their per-slice row sums added in slice order), -3 = as -2 with at most
 * half the LDS per workgroup, -6 = direct staged
 * (instances whose whole gathered vector fits in the LDS alone: the vector
 * is copied to LDS and every row is reduced from its nonzeros in registers,
 * a lane group per row, fused epilogue; the other instances get normal
 * tiles), -7 / -8 = as -6 with at least 4 / 8 lanes per row; *_ept: 2, 4,
 * 8 or 16 nonzeros per thread (tiles of 256 * ept nonzeros), or -8 / -16 (the
 * tiles of ept 8 / 16 run by 1024-thread workgroups, 2 / 4 nonzeros per
 * thread).  -EINVAL otherwise. */
int scylla_batch_set_layout(scylla_batch *h, int32_t row_blocks, int32_t row_ept, int32_t col_blocks,
                            int32_t col_ept);

/* Profiling aid: launches the column pass (primal step) and the row pass
 * (dual step) of the handle `reps` times each on the handle's stream, with
 * the solve's tiles, launch shape and inputs but scratch outputs (the
 * iterates are not changed), and returns the average duration of one launch
 * of each in milliseconds, measured with HIP events.  reps >= 1. */
int scylla_batch_time_passes(scylla_batch *h, int32_t reps, double *ms_row, double *ms_col);


#ifdef __cplusplus
}
#endif
#endif /* SCYLLA_PDHG_H */
