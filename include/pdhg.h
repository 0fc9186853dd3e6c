/*
 * pdhg.h - C ABI of the MI355X (gfx950) restarted-PDHG LP library.
 *
 * Problem (the paper's LP, Section 1 and eq. LP-primal, widened to boxes
 * and >= rows):
 *
 *     minimize   c'x
 *     subject to (A x)_i  = b_i   for rows of kind 0,
 *                (A x)_i >= b_i   for rows of kind 1,
 *                l <= x <= u      (entries of l may be -inf, of u +inf).
 *
 * Method: restarted PDHG on the saddle problem
 * L(x,y) = c'x - y'Ax + b'y over X = {l <= x <= u},
 * Y = {y : y_i >= 0 on rows of kind 1} (eq. LP-Lagrangian).  One iteration
 * is the PDHG update (eq. PDHG-update) with primal step tau = eta/omega and
 * dual step sigma = eta*omega:
 *     x+ = proj_X(x - tau (c - A'y)),
 *     y+ = proj_Y(y + sigma (b - A(2x+ - x))),
 * followed by the running average of Algorithm 1.  Every `check_period`
 * iterations (Section 7 uses 30) the library evaluates the KKT error at the
 * current point and at the average, and the restart test of
 * eq. adaptive-restart-scheme, which needs the normalized duality gap
 * rho_r(z) of eq. rhorz; rho comes from the linear trust region of
 * Section 6.3.1 solved by bisection on the multiplier.
 *
 * Conventions for every entry point:
 *  - Device pointers point to memory on the current HIP device.  Host
 *    pointers are marked "host".  The caller owns every buffer, including
 *    the workspace, and keeps them alive until pdhg_destroy returns.  The
 *    library allocates no device memory; its only allocations are the host
 *    handle and the HIP graph objects it records.
 *  - `stream` is a hipStream_t passed as void*; NULL means the legacy
 *    default stream.  All work is enqueued on that stream; calls that
 *    return host values synchronize it.
 *  - Return codes: 0 success; >0 a non-error outcome; <0 an error (see
 *    PDHG_E_*).  No C++ exception crosses the ABI.  After an error in a
 *    call other than pdhg_create the handle stays usable.
 *  - One host thread at a time per handle.
 *  - All floating point is IEEE FP64; indices are int32 (m, n, nnz must be
 *    below 2^31).
 */
#ifndef PDHG_H
#define PDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define PDHG_OK 0
#define PDHG_NOT_CONVERGED 1  /* iteration budget used up without reaching tol */
#define PDHG_E_INVALID (-1)   /* bad argument, malformed CSR, l > u, NaN data  */
#define PDHG_E_WORKSPACE (-2) /* workspace missing, misaligned or too small    */
#define PDHG_E_HIP (-3)       /* a HIP runtime call failed                     */
#define PDHG_E_NUMERICAL (-4) /* NaN or Inf appeared in the iterates           */

/* restart schemes (Section 5 and Remark rem:flexible) */
#define PDHG_RESTART_NONE 0
#define PDHG_RESTART_ADAPTIVE 1 /* eq. adaptive-restart-scheme                    */
#define PDHG_RESTART_FLEXIBLE 2 /* adaptive, candidate may be the last iterate    */
#define PDHG_RESTART_FIXED 3    /* eq. define:t-star with t* = fixed_len          */

/* which KKT error the stopping test uses */
/* The primal-dual step inside Algorithm 1 (Section 2).  The batched solver
 * and the unrolled forward/backward passes run PDHG only. */
#define PDHG_METHOD_PDHG 0 /* eq. PDHG-update: two products per iteration      */
#define PDHG_METHOD_EGM 1  /* eq. extra-gradient-update: four products; the
                              window average is over the target points        */

#define PDHG_KKT_RELATIVE 0  /* max of the three relative residuals            */
#define PDHG_KKT_PAPER_ABS 1 /* ||(h - Kz)^+||_2, eq. define:K-and-h-for-lp    */
#define PDHG_KKT_MAX_ABS 2   /* max abs primal residual, dual residual, gap    */

/* points held by a handle */
#define PDHG_POINT_CURRENT 0  /* z^{n,t}                                       */
#define PDHG_POINT_AVERAGE 1  /* z-bar^{n,t}, mean of the window's iterates    */
#define PDHG_POINT_ANCHOR 2   /* z^{n,0}, the last restart point               */
#define PDHG_POINT_SOLUTION 3 /* the point that met tol in the last solve      */

typedef struct pdhg_lp {
    int64_t m;               /* rows of A (>= 0)                                */
    int64_t n;               /* columns of A (>= 1)                             */
    int64_t nnz;             /* stored entries; row_ptr[m] must equal nnz       */
    const int32_t *row_ptr;  /* device, m+1, CSR row starts, non-decreasing     */
    const int32_t *col_idx;  /* device, nnz, in [0, n); order within a row free */
    const double *vals;      /* device, nnz                                     */
    const double *c;         /* device, n                                       */
    const double *b;         /* device, m (may be NULL when m == 0)             */
    const double *l;         /* device, n, lower bounds (-inf allowed)          */
    const double *u;         /* device, n, upper bounds (+inf allowed), l <= u  */
    const int8_t *row_kind;  /* device, m, 0 (=) or 1 (>=); NULL: all equality  */
} pdhg_lp;

typedef struct pdhg_params {
    double eta;           /* step size; <= 0: 0.9 / sigma_max(A) by power iteration */
    double omega;         /* primal weight: primal step eta/omega, dual eta*omega   */
    double beta;          /* restart factor (exp(-1), Remark on the choice of beta) */
    int32_t check_period; /* iterations between checks (30)                         */
    int32_t tau0;         /* first-window length of the adaptive scheme (1)         */
    int32_t restart_mode; /* PDHG_RESTART_*                                         */
    int32_t fixed_len;    /* restart length for PDHG_RESTART_FIXED                  */
    int32_t kkt_kind;     /* PDHG_KKT_*                                             */
    int32_t power_iters;  /* power-iteration cap (1000)                             */
    double power_tol;     /* power-iteration relative stop (1e-10)                  */
    int32_t method;       /* PDHG_METHOD_*: the iteration inside Algorithm 1 (PDHG) */
} pdhg_params;

typedef struct pdhg_kkt {
    double kkt;           /* the value of the selected kkt_kind                 */
    double kkt_rel;       /* max(|p|/(1+|b|), |d|/(1+|c|), |gap|/(1+|pobj|+|dobj|)) */
    double primal_res;    /* |p|_2: b - Ax on = rows, (b - Ax)^+ on >= rows     */
    double dual_res;      /* |d|_2: reduced cost minus its projection on the sign set of its bounds */
    double pobj;          /* c'x                                                */
    double dobj;          /* b'y + sum_j (l_j lam_j^+ - u_j lam_j^-)            */
    double kkt_paper_abs; /* ||(h - Kz)^+||_2 with bound violations             */
    double kkt_max_abs;   /* max(|p|_2, |d|_2, |pobj - dobj|)                   */
} pdhg_kkt;

typedef struct pdhg_result {
    int32_t status;       /* PDHG_OK (converged) or PDHG_NOT_CONVERGED         */
    int32_t which_point;  /* PDHG_POINT_CURRENT / _AVERAGE that met tol, or -1 */
    int64_t iterations;   /* total iterations of the handle                    */
    int64_t restarts;     /* total restarts of the handle                      */
    double kkt;           /* selected KKT error of the returned point          */
    double pobj, dobj;
} pdhg_result;

typedef struct pdhg_info {
    double eta, tau, sigma;   /* step sizes in use                            */
    double sigma_max;         /* power-iteration estimate (0 if eta was given) */
    int64_t k;                /* total iterations                              */
    int64_t t;                /* iterations since the last restart             */
    int64_t restarts;         /* restarts so far                               */
    double rho_prev;          /* rho of the last restart point                 */
    int64_t checks;           /* checks so far                                 */
    int64_t power_iters_used; /* products used by the power iteration          */
    int32_t one_workgroup;    /* nonzero: pdhg_solve runs whole check periods
                                 of this LP in one workgroup (method PDHG,
                                 restarts other than fixed length, n + m <= 1024
                                 and the iteration vectors within 148 KiB of
                                 LDS); 1: every lane holds its matrix entries
                                 in registers, 2: the matrix is in LDS too,
                                 3: as 1, and each check runs on half the
                                 workgroup beside the next period's
                                 iterations on the other half (the same
                                 iterates and checks; every row within half
                                 the workgroup).
                                 0: one launch per product and check step.
                                 Environment: PDHG_TINY=0 at pdhg_create turns
                                 the path off, PDHG_TINY=lds asks for 2,
                                 PDHG_TINY_OVERLAP=0 keeps 1 instead of 3 */
    int32_t bound_classes;    /* distinct (l, u) pairs the primal update reads
                                 as a one-byte class per column (1..4), or 0:
                                 it reads l and u */
} pdhg_info;

/* One check, in the order the library performs it (14 doubles):
 *  k, t, restarts before, KKT at z, KKT at z-bar, r-bar = |z-bar - z^{n,0}|,
 *  rho at z-bar, r = |z - z^{n,0}|, rho at z (flexible, else -1),
 *  restarted (0/1), candidate (0 z-bar, 1 z), converged point (-1, 0, 1),
 *  rho_prev used by the test, lambda of the z-bar trust region. */
typedef struct pdhg_check_record {
    double v[14];
} pdhg_check_record;

typedef struct pdhg_handle pdhg_t;

/* Fill *p with the defaults above (eta auto, omega 1, beta exp(-1),
 * check_period 30, tau0 1, adaptive restarts, relative KKT,
 * 1000 power iterations, power_tol 1e-10, method PDHG). */
void pdhg_default_params(pdhg_params *p);

/* Device workspace (bytes, 256-byte aligned start required) that
 * pdhg_create needs for an LP of this size.  Returns 0 for sizes it
 * rejects (negative, n < 1, above int32 range).  When the vector a product
 * gathers is larger than one XCD's L2 (4 MiB; the environment variable
 * PDHG_SLAB_BYTES overrides the target), the workspace also holds a copy
 * of A or A' split into column slabs: keep that variable unchanged between
 * this call and pdhg_create. */
size_t pdhg_workspace_bytes(int64_t m, int64_t n, int64_t nnz);

/*
 * Build a solver for `lp` (setup step of the paper's experiments,
 * Section 7): validates the CSR (row_ptr[0] = 0, non-decreasing,
 * row_ptr[m] = nnz, 0 <= col_idx < n, no NaN in vals/c/b, l <= u, no
 * l = +inf or u = -inf) on the device, forms A' explicitly (entries of each
 * transposed row in increasing row of A), picks eta (power iteration when
 * prm->eta <= 0), and sets x = proj_X(0), y = 0.  `lp` and `prm` are host
 * structs read during the call; the device arrays they point to are read
 * again by later calls and must not change.  prm may be NULL (defaults).
 * Errors: PDHG_E_INVALID, PDHG_E_WORKSPACE, PDHG_E_HIP.  On error *out is
 * NULL.  Synchronizes the stream.
 */
int pdhg_create(const pdhg_lp *lp, const pdhg_params *prm, void *workspace,
                size_t workspace_bytes, void *stream, pdhg_t **out);

/* Run `iters` PDHG iterations (eq. PDHG-update + the average of
 * Algorithm 1) with no check.  With PDHG_RESTART_FIXED the outer loop
 * restarts whenever t reaches fixed_len.  Does not synchronize. */
int pdhg_step(pdhg_t *h, int64_t iters);

/* One check now: KKT at z and z-bar (stopping test against tol when
 * tol > 0), then the restart test of the configured scheme and the restart
 * itself (eq. adaptive-restart-scheme; Algorithm 1's restart line).
 * Outputs (host, each may be NULL): *converged, *restarted, *rho (rho at
 * z-bar), *rec.  Synchronizes. */
int pdhg_restart_check(pdhg_t *h, double tol, int32_t *converged,
                       int32_t *restarted, double *rho, pdhg_check_record *rec);

/* KKT error of a held point (PDHG_POINT_*), into *out (host).  Syncs. */
int pdhg_kkt_error(pdhg_t *h, int32_t which, pdhg_kkt *out);

/* Normalized duality gap rho_r at a held point (eq. rhorz), with r its
 * distance to the anchor z^{n,0} when r < 0, else the given r.  Outputs
 * host *rho, *r_used, *lambda (each may be NULL).  Syncs. */
int pdhg_gap(pdhg_t *h, int32_t which, double r, double *rho, double *r_used,
             double *lambda);

/* Restarted PDHG for up to `max_iters` more iterations, checking whenever
 * the total iteration count is a multiple of check_period; stops at the
 * first check where the KKT error of z or z-bar is <= tol (tol <= 0: never).
 * Returns PDHG_OK when converged, PDHG_NOT_CONVERGED when the budget ran
 * out, or an error.  *out (host, may be NULL) is filled either way.  The
 * check blocks run as a replayed HIP graph; the host reads one status word
 * per batch of blocks.  A block that directly follows a check takes its
 * first primal update from the A'y (or, after a restart at the average,
 * A'y-bar) the check computed, instead of a product: bitwise the same
 * update (PDHG_CHECK_REUSE=0 at pdhg_create runs the product). */
int pdhg_solve(pdhg_t *h, int64_t max_iters, double tol, pdhg_result *out);

/* Outcome of pdhg_autotune.  A product with slabs gathers one column slab
 * of its vector per launch (each slab meant to stay in one XCD's L2);
 * 1 = a single launch over all columns. */
typedef struct pdhg_tune {
    int32_t slabs_A, slabs_At;            /* slab counts in use for A x and A'y   */
    int32_t candidates_A, candidates_At;  /* counts timed (0: fixed or cached)    */
    int32_t tried_A[4], tried_At[4];      /* the slab counts timed                */
    double ms_A[4], ms_At[4];             /* mean time of one product each, ms    */
    int32_t from_cache, reserved;         /* 1: taken from an earlier tuning      */
    int32_t lanes_bias_A, lanes_bias_At;  /* lanes per row in use: -1, 0, +1 power
                                             of two from the block's rule        */
    double ms_lanes_A[3], ms_lanes_At[3]; /* one product with bias -1, 0, +1, ms
                                             (not filled when cached)            */
    int32_t threads_A, threads_At;        /* threads per workgroup in use, 256 or 128 */
    double ms_threads_A[2], ms_threads_At[2]; /* one product with 256 and with 128
                                                 threads, ms (not filled when cached) */
} pdhg_tune;

/* Per-matrix choice of the SpMV schedule of A x and A'y (Section 7's
 * products): first the column slabs (the tiles of the launches) -- times
 * `iters` products of the current point for each slab count 1, 2, 4, 8 the
 * workspace has room for (room exists when the gathered vector is larger
 * than one 4 MiB L2 slice) and keeps the fastest -- then the row split:
 * with that slab count, the lanes that reduce one row (a power of two near
 * each block's mean row length) one power of two lower, as the rule, and
 * one higher, keeping the fastest -- then the threads per workgroup (256,
 * or 128 with twice the entries in flight per thread), keeping the fastest.
 * Before any tuning a product runs 128 threads per workgroup when its launch
 * has at least 2048 blocks of at most 128 rows on average, else 256.  The
 * choice is remembered for the
 * process under a signature of the matrix (sizes and sampled row starts);
 * with use_cache != 0 a remembered choice is applied without timing.  The iterates, averages and counters are left as they are; the
 * products are written to scratch vectors.  Later solves follow the same
 * iterates up to the order of floating-point sums.  *out (host, may be
 * NULL).  Synchronizes.  PDHG_E_INVALID for iters outside 1..10000. */
int pdhg_autotune(pdhg_t *h, int32_t iters, int32_t use_cache, pdhg_tune *out);

/* Pins a schedule instead of timing one: slab counts (1, 2, 4 or 8, at
 * most what the workspace has room for; 1 is always allowed) and lanes-per-
 * row biases (-1, 0, +1) of A x and A'y.  Every schedule gives the same
 * iterates up to the order of floating-point sums.  PDHG_E_INVALID for a
 * value outside those sets.  No sync. */
int pdhg_set_schedule(pdhg_t *h, int32_t slabs_A, int32_t slabs_At, int32_t lanes_bias_A,
                      int32_t lanes_bias_At);

/* Bytes of device workspace pdhg_solve_many needs for `count` handles. */
size_t pdhg_solve_many_workspace_bytes(int32_t count);

/* pdhg_solve (Algorithm 1 with the Section 7 check schedule) on `count`
 * independent handles at once.  hs: host array of distinct handles, all
 * created on the current device.  Handles on the one-workgroup path
 * (pdhg_info.one_workgroup != 0) advance together: one launch runs whole
 * blocks of check_period iterations for all of them, one workgroup (one CU)
 * per LP; each handle follows exactly the iterates and checks of its own
 * pdhg_solve.  Other handles are solved one after another with pdhg_solve.
 * workspace: device memory of at least
 * pdhg_solve_many_workspace_bytes(count) bytes, owned by the caller, not
 * used by any other call while this one runs.  out: host array of `count`
 * results (may be NULL).  The shared launches go on the stream of hs[0];
 * every handle's stream is synchronized first, and the call synchronizes
 * before returning.  Returns PDHG_OK when every handle converged,
 * PDHG_NOT_CONVERGED when the budget ran out for at least one,
 * PDHG_E_INVALID for a bad argument (NULL or repeated handle, workspace
 * too small), or the first error met. */
int pdhg_solve_many(pdhg_t *const *hs, int32_t count, int64_t max_iters, double tol,
                    void *workspace, size_t workspace_bytes, pdhg_result *out);

/* Copy a held point (PDHG_POINT_*) into caller device buffers x (n) and
 * y (m), enqueued on the handle's stream.  Does not synchronize. */
int pdhg_get_iterate(pdhg_t *h, int32_t which, double *x, double *y);

/* Replace the current point and the anchor by device x (n), y (m), clear
 * the averaging window (t = 0).  Restart count and rho_prev are kept. */
int pdhg_set_iterate(pdhg_t *h, const double *x, const double *y);

/*
 * Checkpoint and resume (Algorithm 1's state).  The state of a handle is
 * everything the rest of a run depends on: the current point z^{n,t},
 * the anchor z^{n,0}, the running sums of the window (the average's
 * numerator), A x of the current point, the counters k, t, n (restarts)
 * and checks, rho of the last restart point, the step size eta and primal
 * weight omega, the last check's results (with the converged point) and
 * the check log.  pdhg_state_bytes: size of that state for this handle
 * (0 for NULL).  pdhg_get_state writes it into `state` (device, at least
 * pdhg_state_bytes bytes, 256-byte aligned, owned by the caller) on the
 * handle's stream and synchronizes.  pdhg_set_state loads such a state
 * into a handle created for the same LP (same sizes and matrix, same
 * method, restart scheme, check period and KKT kind; eta and omega are
 * taken from the state), synchronizing; the run then continues exactly as
 * the run it was taken from would have: the same iterates bit for bit.
 * The contents are opaque (vectors in the library's internal column
 * order).  Errors: PDHG_E_INVALID (NULL, a state of another LP or solver
 * configuration, or not written by pdhg_get_state), PDHG_E_WORKSPACE
 * (buffer too small or misaligned), PDHG_E_HIP.  The handle is unchanged
 * after an error of pdhg_set_state.
 */
size_t pdhg_state_bytes(pdhg_t *h);
int pdhg_get_state(pdhg_t *h, void *state, size_t bytes);
int pdhg_set_state(pdhg_t *h, const void *state, size_t bytes);

/* Scalars of the handle into *out (host).  Syncs. */
int pdhg_get_info(pdhg_t *h, pdhg_info *out);

/* Copy up to `max` most recent check records (oldest first) into host
 * `out`; *count receives how many were written.  The library keeps the
 * last 4096.  Syncs. */
int pdhg_get_check_log(pdhg_t *h, pdhg_check_record *out, int64_t max,
                       int64_t *count);

/* out = A in (transpose = 0; in n, out m) or A' in (transpose = 1; in m,
 * out n), with the library's SpMV kernels.  Device buffers; no sync. */
int pdhg_matvec(pdhg_t *h, int32_t transpose, const double *in, double *out);

/* Copy the device-built A' (CSR, entries in increasing row of A) into
 * caller device buffers: t_row_ptr (n+1), t_col_idx (nnz), t_vals (nnz),
 * perm (nnz; index in A of each entry of A'; may be NULL).  No sync. */
int pdhg_get_transpose(pdhg_t *h, int32_t *t_row_ptr, int32_t *t_col_idx,
                       double *t_vals, int32_t *perm);

/* Run `iters` PDHG iterations exactly as pdhg_step does (no fixed-length
 * restarts) with a HIP event recorded around every half-step on the
 * handle's stream, and return the mean duration in milliseconds of the
 * primal half-step (x+ from A'y, eq. PDHG-update) and of the dual half-step
 * (y+ from A x+); each is one kernel, or one per column slab where the
 * product runs over slabs (the last one adds the slabs' row sums and
 * applies the update).  For throughput measurement.  Syncs. */
int pdhg_time_iterations(pdhg_t *h, int64_t iters, double *ms_primal, double *ms_dual);

/* Measurement yardsticks for the roofline of the half-steps (no paper
 * step): the mean time in ms (host *ms) of `reps` (1..1000) launches of
 *  - pdhg_time_copy: the library's plain streaming copy dst[i] = src[i],
 *    i < n (device, 32-byte aligned, not overlapping): 16 n bytes of HBM
 *    traffic per launch when n is large;
 *  - pdhg_time_gather: a plain gather out[i] = val[i] * x[idx[i]], i < n
 *    (device; every idx[i] must index x; n < 2^31), the access pattern of a
 *    product's gathers without its rows and update.
 * One warm-up launch runs first; enqueued on `stream`, synchronizes.
 * Errors: PDHG_E_INVALID, PDHG_E_HIP. */
int pdhg_time_copy(const double *src, double *dst, int64_t n, int32_t reps, void *stream,
                   double *ms);
int pdhg_time_gather(const int32_t *idx, const double *val, const double *x, double *out,
                     int64_t n, int32_t reps, void *stream, double *ms);

/* Gathers alone, the request rate a product's gathers can reach with
 * nothing else in flight: each thread sums x at 4 indices and stores the
 * sum (pdhg_gather_only_outputs(n) doubles of `out`, device).  With `idx`
 * (device, n indices into x of xlen doubles) the indices are that stream;
 * with idx NULL they are Fibonacci hashes of the entry number into
 * [0, xlen), xlen a power of two, so no index stream is read and the
 * footprint is 8 xlen bytes.  Mean ms of `reps` (1..1000) launches after one
 * warm-up (host *ms), enqueued on `stream`, synchronizes.  Errors:
 * PDHG_E_INVALID (also for a hashed window that is not a power of two),
 * PDHG_E_HIP. */
int64_t pdhg_gather_only_outputs(int64_t n);
int pdhg_time_gather_only(const int32_t *idx, int64_t n, const double *x, int64_t xlen,
                          double *out, int32_t reps, void *stream, double *ms);

/* Primal-weight search of Section 7 (experimental setup).  For each of the
 * `count` weights omega[w] (host array; every omega > 0; 1 <= count <= 16)
 * run `iters` (>= 0) iterations of the handle's method (PDHG or
 * extragradient) without restarts from the initial point, with primal step
 * eta/omega[w] and dual step eta*omega[w] (eta of the handle).  The
 * copies run side by side: each product streams A or A' once for all of
 * them.  Then the KKT error of every copy's last iterate
 * goes to kkt[w] (host array of count; kkt[w].kkt = kkt_paper_abs, the
 * criterion of Section 7), and *best (host, may be NULL) gets the w with
 * the smallest kkt_paper_abs (NaN counts as +inf, ties go to the smaller
 * w; -1 when every copy broke down).  x_out (device, count*n, copy w at
 * offset w*n) and y_out (device, count*m) receive the last iterates and may
 * be NULL.  workspace: device, 256-byte aligned, at least
 * pdhg_weight_search_workspace_bytes(m, n, count) bytes, owned by the
 * caller and free again on return.  The handle's own iterates, counters
 * and weight are untouched.  Synchronizes.  Errors: PDHG_E_INVALID for a
 * bad argument, PDHG_E_WORKSPACE, PDHG_E_HIP. */
size_t pdhg_weight_search_workspace_bytes(int64_t m, int64_t n, int32_t count);
int pdhg_weight_search(pdhg_t *h, const double *omega, int32_t count, int64_t iters,
                       void *workspace, size_t workspace_bytes, pdhg_kkt *kkt,
                       int32_t *best, double *x_out, double *y_out);

/* Set the primal weight omega (> 0, finite) of the handle (Section 7:
 * primal step eta/omega, dual step eta*omega, and the omega-weighted norm
 * of the normalized duality gap), then start the method again from the
 * initial point: iterates, running sums, counters, restart state and the
 * check log are reset.  No sync. */
int pdhg_set_primal_weight(pdhg_t *h, double omega);

/* Release the host handle and its graphs (does not touch caller memory).
 * Synchronizes the stream first.  NULL is ignored. */
void pdhg_destroy(pdhg_t *h);

/*
 * Stand-alone linear trust region of Section 6.3.1 (Algorithm 2 solves the
 * same problem): for N coordinates with a_i = |g_i| >= 0 and distances
 * d_i in [0, +inf] to the bound each one moves toward, find
 *     lambda* = max { lambda >= 0 : sum_i min(lambda a_i, d_i)^2 <= r^2 }
 * and value = sum_i a_i min(lambda* a_i, d_i), the decrease of the linear
 * objective (lambda* = +inf when every d_i with a_i > 0 is finite and
 * sum d_i^2 <= r^2; value = 0 when r <= 0).  a, d: device, N.  Workspace:
 * device, pdhg_trust_region_workspace_bytes(N) bytes, 256-byte aligned.
 * Outputs host *value, *lambda.  Syncs.  Errors: PDHG_E_INVALID (N < 0,
 * negative or NaN a or d), PDHG_E_WORKSPACE, PDHG_E_HIP.
 */
size_t pdhg_trust_region_workspace_bytes(int64_t N);
int pdhg_linear_trust_region(int64_t N, const double *a, const double *d,
                             double r, void *workspace, size_t workspace_bytes,
                             void *stream, double *value, double *lambda);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * stand-alone linear trust region above with its scratch in a static
 * device array owned by the library (14 MiB on each GPU it runs on, held
 * until the process ends) instead of a caller workspace.  N is at most
 * PDHG_TR_STATIC_MAX_N (PDHG_E_INVALID beyond).  The call allocates
 * nothing.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (several streams or host threads) race and must be
 * serialized by the caller.  Other arguments, outputs, synchronization and
 * errors as pdhg_linear_trust_region.
 */
#define PDHG_TR_STATIC_MAX_N 262144
int pdhg_linear_trust_region_static(int64_t N, const double *a, const double *d, double r,
                                    void *stream, double *value, double *lambda);

/*
 * Batched solver: `count` independent LPs advanced by the same launches
 * (the LPs are concatenated into one block-diagonal system on the device).
 * Each LP keeps its own step sizes (power iteration per LP when its
 * eta <= 0), iteration and restart counters, restart state and stopping
 * test; an LP that reaches tol stops changing while the others continue.
 * `lps` and `prm` are host arrays of `count` structs (prm may be NULL for
 * defaults); restart_mode (none, adaptive or flexible), check_period and
 * kkt_kind must be equal across the batch.  Workspace and stream rules are
 * those of pdhg_create.  Sizes: host arrays m, n, nnz of `count` entries.
 * Inside each LP's own range the columns are held in an order of the
 * library's choosing (by entry count, then by first row); every call below
 * takes and returns column vectors in the caller's order.
 */
typedef struct pdhg_batch_handle pdhg_batch_t;
size_t pdhg_batch_workspace_bytes(int32_t count, const int64_t *m, const int64_t *n,
                                  const int64_t *nnz);
int pdhg_batch_create(int32_t count, const pdhg_lp *lps, const pdhg_params *prm,
                      void *workspace, size_t workspace_bytes, void *stream,
                      pdhg_batch_t **out);
/* `iters` PDHG iterations of every LP that has not converged (no checks). */
int pdhg_batch_step(pdhg_batch_t *h, int64_t iters);
/* Restarted PDHG on all LPs for up to max_iters more iterations with the
 * checks of pdhg_solve; returns PDHG_OK when every LP met tol.  results:
 * host array of `count` (may be NULL).  Graph-replayed like pdhg_solve. */
int pdhg_batch_solve(pdhg_batch_t *h, int64_t max_iters, double tol, pdhg_result *results);
/* Held point (PDHG_POINT_*) of LP `index` into device x (n_index), y (m_index). */
int pdhg_batch_get_iterate(pdhg_batch_t *h, int32_t index, int32_t which, double *x,
                           double *y);
int pdhg_batch_get_info(pdhg_batch_t *h, int32_t index, pdhg_info *out);
/* Last check records of LP `index` (the last 512 are kept). */
int pdhg_batch_get_check_log(pdhg_batch_t *h, int32_t index, pdhg_check_record *out,
                             int64_t max, int64_t *count);
void pdhg_batch_destroy(pdhg_batch_t *h);

/* SpMV schedule of the batch's products: `placement` 1 runs the merge-path
 * blocks of each LP on one XCD (largest LP first onto the least loaded
 * XCD), 0 runs the blocks in row order; `index16` 1 gathers through 16-bit
 * indices relative to each LP (available when every LP has at most 65,536
 * rows and columns), 0 through the 32-bit ones.  Both are set at creation
 * to (1, 1 when available). */
typedef struct pdhg_batch_tune {
    int32_t placement, index16;   /* the schedule in use                        */
    int32_t candidates, reserved; /* schedules timed                             */
    int32_t tried_placement[4], tried_index16[4];
    double ms[4];                 /* mean time of one A'y and one A x, ms       */
} pdhg_batch_tune;
/* Times `iters` pairs of products (A'y and A x of the current point, into
 * scratch vectors; the iterates, averages and counters stay as they are)
 * for each schedule and keeps the fastest.  *out (host, may be NULL).
 * Synchronizes.  PDHG_E_INVALID for iters outside 1..10000. */
int pdhg_batch_autotune(pdhg_batch_t *h, int32_t iters, pdhg_batch_tune *out);
/* Sets a schedule (see pdhg_batch_tune); PDHG_E_INVALID for a flag other
 * than 0 or 1, or index16 = 1 when 16-bit indices are not available.  No
 * schedule changes a result: every row is summed in the same order. */
int pdhg_batch_set_schedule(pdhg_batch_t *h, int32_t placement, int32_t index16);

/* Replace the problem data of the whole batch with device arrays in the
 * concatenated layout (c: sum n_i, b: sum m_i, vals: sum nnz_i, each LP's
 * entries in its own CSR order); the sparsity pattern and the step sizes
 * stay.  Enqueued, no sync. */
int pdhg_batch_set_data(pdhg_batch_t *h, const double *c, const double *b, const double *vals);

/*
 * Differentiation of K unrolled restarted-PDHG iterations.  The forward
 * call puts every LP back at its initial point and runs K iterations with
 * the configured restart checks (no stopping test), recording into `tape`
 * (device, pdhg_batch_tape_bytes(h, K) bytes, 256-byte aligned) a
 * checkpoint of (x, y, A x) at every check boundary (so at every restart)
 * and each check's restart decision; x_K (concatenated, sum n_i) goes to
 * device xK when given.  The backward call takes dL/dx_K (device,
 * concatenated) and writes dL/dc, dL/db and dL/d(values of A) (device,
 * concatenated; they are overwritten) through the PDHG update
 * (eq. PDHG-update), the running average and restarts of Algorithm 1 with
 * the restart decisions and projection masks of the forward pass held
 * fixed.  Each window between checkpoints is recomputed from its
 * checkpoint and swept in reverse.  The step sizes are constants.  The
 * backward call takes the tape and K of the last forward call, with no
 * solve, step or set_data since (else PDHG_E_INVALID); it may be repeated
 * on one forward.  The backward call recomputes the windows through the
 * batch's own iterate arrays and then puts back the state the forward call
 * ended in (x_K, y_K, the running sums and every LP's counters and
 * restart state; the tape holds a copy), so a later step or solve
 * continues from K exactly as it would have without the backward call.
 */
size_t pdhg_batch_tape_bytes(pdhg_batch_t *h, int64_t K);
int pdhg_batch_unrolled_forward(pdhg_batch_t *h, int64_t K, void *tape, size_t tape_bytes,
                                double *xK);
int pdhg_batch_unrolled_backward(pdhg_batch_t *h, int64_t K, void *tape, size_t tape_bytes,
                                 const double *dL_dxK, double *grad_c, double *grad_b,
                                 double *grad_vals);

/* Static text for a return code. */
const char *pdhg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PDHG_H */
