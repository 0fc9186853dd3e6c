/*
 * Plain FP64 CPU oracle for restarted PDHG on linear programs.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only through
 * the seeded input generator.
 *
 * Problem (the paper's standard form, Section 1 and eq. LP-primal, widened
 * to boxes and >= rows):
 *     min c'x  s.t.  A x = b  (rows of kind 0),  A x >= b (rows of kind 1),
 *                    l <= x <= u.
 * Saddle form (eq. LP-Lagrangian): L(x,y) = c'x - y'Ax + b'y over
 * X = {l <= x <= u} and Y = {y : y_i >= 0 for rows of kind 1}.
 * Operator F(z) = (grad_x L, -grad_y L) = (c - A'y, Ax - b)   (Section 1).
 *
 * Everything here follows the paper's statements directly, in the paper's
 * order, with no blocking, fusion or reordering:
 *   - PDHG step: eq. PDHG-update with f(x) = c'x + 1_X, the bilinear
 *     coupling y'(-A)x and g(y) = -b'y + 1_Y, primal step tau = eta/omega and
 *     dual step sigma = eta*omega (footnote to eq. PDHG-update; primal weight
 *     paragraph of Section 7).  The dual step forms A(2x+ - x) literally.
 *   - Extragradient step (the paper's second method): eq.
 *     extra-gradient-update with the same F, Z and step sizes; Algorithm 1
 *     averages its target points z~ (the averaging of Section 2).
 *   - Running average: Algorithm 1, average line, kept as the sum of the
 *     window's iterates (targets, for the extragradient method) divided by
 *     its length.
 *   - Restart schemes: Algorithm 1 with eq. adaptive-restart-scheme,
 *     eq. define:t-star (fixed length) and Remark rem:flexible.
 *   - Normalized duality gap: eq. rhorz with L(x,y~)-L(x~,y) = F(z)'(z-z~)
 *     (eq. bilinear-0), solved as the linear trust region of Section 6.3.1
 *     by Algorithm 2 (median elimination), widened from lower bounds to
 *     boxes by sending each coordinate toward the bound its gradient points
 *     at.  The median comes from a full sort (qsort), a library step.
 *   - KKT error: eq. define:K-and-h-for-lp rows, widened to boxes and >=
 *     rows, plus a relative variant; see orc_kkt_parts.
 *   - Step size: eta = 0.9 / sigma_max(A) with sigma_max from power
 *     iteration (Section 7; the printed formula multiplies by sigma_max,
 *     which contradicts the valid range eta <= 1/sigma_max of Proposition
 *     prop:assumption-one-holds, so the reciprocal is used).
 * Compile with -O2 -ffp-contract=off so that no fused multiply-add changes
 * the rounding of the written formulas.
 *
 * Built with -DORC_OPENMP -fopenmp, the same source runs the products and
 * the per-coordinate loops of an iteration on every host core (for the
 * CPU baseline): each parallel loop writes only its own outputs, and A'y
 * is taken row by row of an explicit A' whose rows keep the entries in
 * increasing row of A, the order in which the plain build accumulates
 * them.  Every sum (norms, KKT parts, the trust region) stays sequential.
 * The two builds therefore give bitwise equal results.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MODE_NONE 0
#define ORC_MODE_ADAPTIVE 1
#define ORC_MODE_FLEXIBLE 2
#define ORC_MODE_FIXED 3

#define ORC_METHOD_PDHG 0
#define ORC_METHOD_EGM 1

#ifdef ORC_OPENMP
#define ORC_PAR_FOR _Pragma("omp parallel for schedule(static, 2048)")
#else
#define ORC_PAR_FOR
#endif

#define ORC_KKT_RELATIVE 0
#define ORC_KKT_PAPER_ABS 1
#define ORC_KKT_MAX_ABS 2

/* One check record (doubles): see orc_check. */
#define ORC_REC 14

typedef struct orc {
    int64_t m, n, nnz;
    int32_t *rp, *ci;
    double *v;
    double *c, *b, *l, *u;
    int8_t *kind;
    double eta, omega, tau, sigma, beta, sigma_max;
    int32_t period, tau0, mode, fixed_len, kkt_kind, method;
    /* state */
    double *x, *y, *x0, *y0, *sx, *sy;
    int64_t k, t, nrst;
    double rho_prev;
    /* scratch */
    double *ax, *aty, *xa, *ya, *axa, *atya, *xn, *yn, *e, *ga, *gd, *xt, *yt;
    /* check log */
    double *log;
    int64_t log_len, log_cap;
    /* explicit A' for the row-parallel A'y of the ORC_OPENMP build */
    int32_t *trp, *tci;
    double *tv;
} orc_t;

/* ------------------------------------------------------------------ */
/* Products with A and A' (plain definitions).                         */
/* ------------------------------------------------------------------ */

/* out = A x : (A x)_i = sum_k A_ik x_k over the stored entries of row i. */
static void mat_vec(const orc_t *o, const double *x, double *out)
{
    ORC_PAR_FOR
    for (int64_t i = 0; i < o->m; ++i) {
        double s = 0.0;
        for (int32_t p = o->rp[i]; p < o->rp[i + 1]; ++p)
            s += o->v[p] * x[o->ci[p]];
        out[i] = s;
    }
}

/* out = A' y : (A'y)_j = sum_i A_ij y_i, accumulated in increasing i. */
static void mat_tvec(const orc_t *o, const double *y, double *out)
{
#ifdef ORC_OPENMP
    if (o->trp) {
        /* the same sums, one row of A' per column j, entries in increasing i */
        ORC_PAR_FOR
        for (int64_t j = 0; j < o->n; ++j) {
            double s = 0.0;
            for (int32_t q = o->trp[j]; q < o->trp[j + 1]; ++q)
                s += o->tv[q] * y[o->tci[q]];
            out[j] = s;
        }
        return;
    }
#endif
    for (int64_t j = 0; j < o->n; ++j) out[j] = 0.0;
    for (int64_t i = 0; i < o->m; ++i)
        for (int32_t p = o->rp[i]; p < o->rp[i + 1]; ++p)
            out[o->ci[p]] += o->v[p] * y[i];
}

static double clampd(double v, double lo, double hi)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* ------------------------------------------------------------------ */
/* CSR transpose (definition: entry (i,j) of A becomes entry (j,i)).    */
/* Entries of each transposed row come out in increasing original row.  */
/* perm[q] is the index in A of transposed entry q.                     */
/* ------------------------------------------------------------------ */
void orc_transpose(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                   const double *v, int32_t *trp, int32_t *tci, double *tv,
                   int32_t *perm)
{
    for (int64_t j = 0; j <= n; ++j) trp[j] = 0;
    for (int64_t p = 0; p < rp[m]; ++p) trp[ci[p] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) fill[j] = trp[j];
    for (int64_t i = 0; i < m; ++i)
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            int32_t q = fill[ci[p]]++;
            tci[q] = (int32_t)i;
            tv[q] = v[p];
            if (perm) perm[q] = p;
        }
    free(fill);
}

/* ------------------------------------------------------------------ */
/* Power iteration on A'A for sigma_max(A) (Section 7 step size).        */
/* Start 1/sqrt(n) in every coordinate; stop when the estimate changes  */
/* by at most tol relative, or after max_iters products.                */
/* ------------------------------------------------------------------ */
static double power_iter(const orc_t *o, int32_t max_iters, double tol)
{
    int64_t n = o->n;
    double *vv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(o->m > 0 ? o->m : 1));
    double *uu = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j) vv[j] = 1.0 / sqrt((double)n);
    double est = 0.0, prev = 0.0;
    for (int32_t it = 0; it < max_iters; ++it) {
        mat_vec(o, vv, w);
        mat_tvec(o, w, uu);
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += uu[j] * uu[j];
        s = sqrt(s); /* ||A'A v|| with ||v|| = 1 approaches sigma_max^2 */
        if (!(s > 0.0)) { est = 0.0; break; }
        for (int64_t j = 0; j < n; ++j) vv[j] = uu[j] / s;
        est = sqrt(s);
        if (it > 0 && fabs(est - prev) <= tol * est) break;
        prev = est;
    }
    free(vv); free(w); free(uu);
    return est;
}

double orc_power_iteration(int64_t m, int64_t n, const int32_t *rp,
                           const int32_t *ci, const double *v,
                           int32_t max_iters, double tol)
{
    orc_t o;
    memset(&o, 0, sizeof(o));
    o.m = m; o.n = n; o.rp = (int32_t *)rp; o.ci = (int32_t *)ci; o.v = (double *)v;
    return power_iter(&o, max_iters, tol);
}

/* ------------------------------------------------------------------ */
/* Linear trust region, Algorithm 2 (Appendix), in the g_i > 0 form.    */
/*                                                                      */
/* Each coordinate i is described by a_i = |g_i| >= 0 and the distance */
/* d_i in [0, inf] it may travel before it meets the bound its gradient */
/* points at.  With z~(lambda)_i moving by min(lambda a_i, d_i), the    */
/* problem is  max lambda : f(lambda) = sum_i min(lambda a_i, d_i)^2 <= */
/* r^2  (eq. lp-trust-region:lambda, eq. lp-trust-region:summation).    */
/* Coordinates with a_i = 0 never move and are left out.                */
/* Returns the decrease of the linear objective, sum_i a_i min(lambda*  */
/* a_i, d_i), and stores lambda* (inf when the whole box fits).         */
/* ------------------------------------------------------------------ */
static int cmp_double(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

double orc_trust_region(int64_t N, const double *a, const double *d, double r,
                        double *lambda_out)
{
    if (!(r > 0.0)) {
        if (lambda_out) *lambda_out = 0.0;
        return 0.0;
    }
    const double r2 = r * r;
    /* first line of Algorithm 2: the bound itself lies in the ball */
    int all_finite = 1;
    double dist2 = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(a[i] > 0.0)) continue;
        if (isinf(d[i])) all_finite = 0;
        else dist2 += d[i] * d[i];
    }
    if (all_finite && dist2 <= r2) {
        double val = 0.0;
        for (int64_t i = 0; i < N; ++i)
            if (a[i] > 0.0) val += a[i] * d[i];
        if (lambda_out) *lambda_out = INFINITY;
        return val;
    }
    /* breakpoints lambda^_i = d_i / a_i */
    double *bp = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double lam_lo = 0.0, lam_hi = INFINITY;
    double f_lo = 0.0, f_hi = 0.0;
    int64_t ni = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(a[i] > 0.0)) continue;
        bp[i] = d[i] / a[i];
        if (bp[i] <= lam_lo) f_lo += d[i] * d[i];
        else if (bp[i] >= lam_hi) f_hi += a[i] * a[i];
        else idx[ni++] = i;
    }
    while (ni > 0) {
        for (int64_t q = 0; q < ni; ++q) tmp[q] = bp[idx[q]];
        qsort(tmp, (size_t)ni, sizeof(double), cmp_double);
        double mid = tmp[(ni - 1) / 2]; /* a median of the open set */
        double f_mid = f_lo + f_hi * mid * mid;
        for (int64_t q = 0; q < ni; ++q) {
            int64_t i = idx[q];
            double s = mid * a[i];
            if (s > d[i]) s = d[i];
            f_mid += s * s;
        }
        int64_t keep = 0;
        if (f_mid < r2) {
            lam_lo = mid;
            for (int64_t q = 0; q < ni; ++q) {
                int64_t i = idx[q];
                if (bp[i] <= mid) f_lo += d[i] * d[i];
                else idx[keep++] = i;
            }
        } else {
            lam_hi = mid;
            for (int64_t q = 0; q < ni; ++q) {
                int64_t i = idx[q];
                if (bp[i] >= mid) f_hi += a[i] * a[i];
                else idx[keep++] = i;
            }
        }
        ni = keep;
    }
    double lam;
    if (f_hi > 0.0) {
        double num = r2 - f_lo;
        if (num < 0.0) num = 0.0;
        lam = sqrt(num / f_hi);
    } else {
        lam = INFINITY;
    }
    (void)lam_hi;
    double val = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        if (!(a[i] > 0.0)) continue;
        double s = lam * a[i];
        if (s > d[i]) s = d[i];
        val += a[i] * s;
    }
    free(bp); free(idx); free(tmp);
    if (lambda_out) *lambda_out = lam;
    return val;
}

/* ------------------------------------------------------------------ */
/* Normalized duality gap rho_r(z) for the LP (eq. rhorz, Section 6.3.2) */
/* at z = (x, y) given ax = A x and aty = A'y.  The norm is Euclidean in */
/* the primal-weight scaling ||z||^2 = omega ||x||^2 + ||y||^2 / omega,   */
/* which is the plain Euclidean norm of the rescaled space in the        */
/* footnote to eq. PDHG-update; omega = 1 gives the paper's experiments. */
/* r = 0 gives 0 (eq. rhor-zero is never needed by the restart test).    */
/* ------------------------------------------------------------------ */
static double gap_at(orc_t *o, const double *x, const double *y,
                     const double *ax, const double *aty, double r,
                     double *lambda_out)
{
    int64_t n = o->n, m = o->m;
    double sw = sqrt(o->omega);
    for (int64_t j = 0; j < n; ++j) {
        double g = o->c[j] - aty[j];
        double dist = 0.0;
        if (g > 0.0) dist = x[j] - o->l[j];      /* objective falls as x~_j falls */
        else if (g < 0.0) dist = o->u[j] - x[j]; /* objective falls as x~_j rises */
        if (dist < 0.0) dist = 0.0;
        o->ga[j] = fabs(g) / sw;
        o->gd[j] = dist * sw;
    }
    for (int64_t i = 0; i < m; ++i) {
        double g = ax[i] - o->b[i];
        double lo = o->kind[i] ? 0.0 : -INFINITY;
        double dist = 0.0;
        if (g > 0.0) dist = y[i] - lo;
        else if (g < 0.0) dist = INFINITY;
        if (dist < 0.0) dist = 0.0;
        o->ga[n + i] = fabs(g) * sw;
        o->gd[n + i] = dist / sw;
    }
    if (!(r > 0.0)) {
        if (lambda_out) *lambda_out = 0.0;
        return 0.0;
    }
    double val = orc_trust_region(n + m, o->ga, o->gd, r, lambda_out);
    return val / r;
}

/* ------------------------------------------------------------------ */
/* KKT error.  Rows of K z >= h (eq. define:K-and-h-for-lp) widened to  */
/* l <= x <= u and >= rows:                                             */
/*   primal residual p_i = b_i - (Ax)_i (kind 0), max(b_i - (Ax)_i, 0)  */
/*   (kind 1);                                                          */
/*   reduced cost rc = c - A'y; lam_j = projection of rc_j onto the     */
/*   sign set its finite bounds allow (both: R; lower only: [0,inf);    */
/*   upper only: (-inf,0]; none: {0}); dual residual d_j = rc_j - lam_j;*/
/*   pobj = c'x, dobj = b'y + sum_j (l_j max(lam_j,0) - u_j max(-lam_j,0));*/
/*   bound violations of x and of y on >= rows.                         */
/* With l = 0, u = inf and all rows equalities this is exactly h - Kz.  */
/* out[0] relative KKT = max(|p|/(1+|b|), |d|/(1+|c|),                  */
/*                           |pobj-dobj|/(1+|pobj|+|dobj|))             */
/* out[1] |p|, out[2] |d|, out[3] pobj, out[4] dobj,                    */
/* out[5] |(h - Kz)^+| (bound, primal, dual rows and (pobj-dobj)^+),    */
/* out[6] max(|p|, |d|, |pobj - dobj|).                                 */
/* ------------------------------------------------------------------ */
static void kkt_parts(const orc_t *o, const double *x, const double *y,
                      const double *ax, const double *aty, double *out)
{
    int64_t n = o->n, m = o->m;
    double pres2 = 0.0, dres2 = 0.0, bviol2 = 0.0, nb2 = 0.0, nc2 = 0.0;
    double pobj = 0.0, dobj = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double p = o->b[i] - ax[i];
        if (o->kind[i] && p < 0.0) p = 0.0;
        pres2 += p * p;
        if (o->kind[i] && y[i] < 0.0) bviol2 += y[i] * y[i];
        nb2 += o->b[i] * o->b[i];
        dobj += o->b[i] * y[i];
    }
    for (int64_t j = 0; j < n; ++j) {
        double rc = o->c[j] - aty[j];
        int lf = isfinite(o->l[j]), uf = isfinite(o->u[j]);
        double lam;
        if (lf && uf) lam = rc;
        else if (lf) lam = rc > 0.0 ? rc : 0.0;
        else if (uf) lam = rc < 0.0 ? rc : 0.0;
        else lam = 0.0;
        double dr = rc - lam;
        dres2 += dr * dr;
        if (lam > 0.0) dobj += o->l[j] * lam;
        if (lam < 0.0) dobj += o->u[j] * lam; /* -u_j * max(-lam_j, 0) */
        pobj += o->c[j] * x[j];
        nc2 += o->c[j] * o->c[j];
        double bv = 0.0;
        if (x[j] < o->l[j]) bv = o->l[j] - x[j];
        if (x[j] > o->u[j]) bv = x[j] - o->u[j];
        bviol2 += bv * bv;
    }
    double pres = sqrt(pres2), dres = sqrt(dres2);
    double gap = pobj - dobj;
    double rel_p = pres / (1.0 + sqrt(nb2));
    double rel_d = dres / (1.0 + sqrt(nc2));
    double rel_g = fabs(gap) / (1.0 + fabs(pobj) + fabs(dobj));
    double rel = rel_p;
    if (rel_d > rel) rel = rel_d;
    if (rel_g > rel) rel = rel_g;
    double gpos = gap > 0.0 ? gap : 0.0;
    double mx = pres;
    if (dres > mx) mx = dres;
    if (fabs(gap) > mx) mx = fabs(gap);
    out[0] = rel;
    out[1] = pres;
    out[2] = dres;
    out[3] = pobj;
    out[4] = dobj;
    out[5] = sqrt(bviol2 + pres2 + dres2 + gpos * gpos);
    out[6] = mx;
}

/* ------------------------------------------------------------------ */
/* Handle                                                              */
/* ------------------------------------------------------------------ */
static double *dalloc(int64_t k)
{
    return (double *)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
}

static double wnorm2(const orc_t *o, const double *x1, const double *y1,
                     const double *x2, const double *y2)
{
    double sx = 0.0, sy = 0.0;
    for (int64_t j = 0; j < o->n; ++j) { double d = x1[j] - x2[j]; sx += d * d; }
    for (int64_t i = 0; i < o->m; ++i) { double d = y1[i] - y2[i]; sy += d * d; }
    return o->omega * sx + sy / o->omega;
}

orc_t *orc_create(int64_t m, int64_t n, const int32_t *rp, const int32_t *ci,
                  const double *v, const double *c, const double *b,
                  const double *l, const double *u, const int8_t *kind,
                  double eta, double omega, double beta, int32_t period,
                  int32_t tau0, int32_t mode, int32_t fixed_len,
                  int32_t kkt_kind, int32_t power_iters, double power_tol)
{
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    int64_t nnz = rp[m];
    o->m = m; o->n = n; o->nnz = nnz;
    o->rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    o->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    o->v = dalloc(nnz);
    memcpy(o->rp, rp, sizeof(int32_t) * (size_t)(m + 1));
    if (nnz) memcpy(o->ci, ci, sizeof(int32_t) * (size_t)nnz);
    if (nnz) memcpy(o->v, v, sizeof(double) * (size_t)nnz);
    o->c = dalloc(n); o->b = dalloc(m); o->l = dalloc(n); o->u = dalloc(n);
    memcpy(o->c, c, sizeof(double) * (size_t)n);
    memcpy(o->b, b, sizeof(double) * (size_t)m);
    memcpy(o->l, l, sizeof(double) * (size_t)n);
    memcpy(o->u, u, sizeof(double) * (size_t)n);
    o->kind = (int8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
    if (kind) memcpy(o->kind, kind, (size_t)m);
    o->omega = omega > 0.0 ? omega : 1.0;
    o->beta = beta;
    o->period = period > 0 ? period : 30;
    o->tau0 = tau0 > 0 ? tau0 : 1;
    o->mode = mode;
    o->fixed_len = fixed_len;
    o->kkt_kind = kkt_kind;
#ifdef ORC_OPENMP
    o->trp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    o->tci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    o->tv = dalloc(nnz);
    orc_transpose(m, n, o->rp, o->ci, o->v, o->trp, o->tci, o->tv, NULL);
#endif
    o->sigma_max = 0.0;
    if (eta > 0.0) {
        o->eta = eta;
    } else {
        o->sigma_max = power_iter(o, power_iters > 0 ? power_iters : 1000,
                                  power_tol > 0.0 ? power_tol : 1e-10);
        o->eta = o->sigma_max > 0.0 ? 0.9 / o->sigma_max : 1.0;
    }
    o->tau = o->eta / o->omega;
    o->sigma = o->eta * o->omega;
    o->x = dalloc(n); o->y = dalloc(m); o->x0 = dalloc(n); o->y0 = dalloc(m);
    o->sx = dalloc(n); o->sy = dalloc(m);
    o->ax = dalloc(m); o->aty = dalloc(n); o->xa = dalloc(n); o->ya = dalloc(m);
    o->axa = dalloc(m); o->atya = dalloc(n); o->xn = dalloc(n); o->yn = dalloc(m);
    o->e = dalloc(n > m ? n : m);
    o->ga = dalloc(n + m); o->gd = dalloc(n + m);
    o->xt = dalloc(n); o->yt = dalloc(m);
    o->method = ORC_METHOD_PDHG;
    /* initial point (the paper leaves it open): x = proj_X(0), y = 0 */
    for (int64_t j = 0; j < n; ++j) {
        o->x[j] = clampd(0.0, o->l[j], o->u[j]);
        o->x0[j] = o->x[j];
    }
    o->k = 0; o->t = 0; o->nrst = 0; o->rho_prev = 0.0;
    o->log_cap = 0; o->log_len = 0; o->log = NULL;
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    free(o->rp); free(o->ci); free(o->v); free(o->c); free(o->b); free(o->l);
    free(o->u); free(o->kind); free(o->x); free(o->y); free(o->x0); free(o->y0);
    free(o->sx); free(o->sy); free(o->ax); free(o->aty); free(o->xa); free(o->ya);
    free(o->axa); free(o->atya); free(o->xn); free(o->yn); free(o->e);
    free(o->ga); free(o->gd); free(o->xt); free(o->yt); free(o->log);
    free(o->trp); free(o->tci); free(o->tv);
    free(o);
}

/* threads the parallel loops use (1 for the plain build) */
#ifdef ORC_OPENMP
#include <omp.h>
int32_t orc_threads(void) { return (int32_t)omp_get_max_threads(); }
#else
int32_t orc_threads(void) { return 1; }
#endif

/* scalar info: eta, tau, sigma, sigma_max, k, t, restarts, rho_prev */
void orc_info(const orc_t *o, double *out)
{
    out[0] = o->eta; out[1] = o->tau; out[2] = o->sigma; out[3] = o->sigma_max;
    out[4] = (double)o->k; out[5] = (double)o->t; out[6] = (double)o->nrst;
    out[7] = o->rho_prev;
}

/* z-bar of Algorithm 1; the empty window (t = 0) averages to z itself */
static void average(orc_t *o, double *xa, double *ya)
{
    if (o->t == 0) {
        memcpy(xa, o->x, sizeof(double) * (size_t)o->n);
        memcpy(ya, o->y, sizeof(double) * (size_t)o->m);
        return;
    }
    double tt = (double)o->t;
    ORC_PAR_FOR
    for (int64_t j = 0; j < o->n; ++j) xa[j] = o->sx[j] / tt;
    ORC_PAR_FOR
    for (int64_t i = 0; i < o->m; ++i) ya[i] = o->sy[i] / tt;
}

/* restart the outer loop of Algorithm 1 from the candidate (xc, yc) */
static void restart_to(orc_t *o, const double *xc, const double *yc, double rho)
{
    if (xc != o->x) memcpy(o->x, xc, sizeof(double) * (size_t)o->n);
    if (yc != o->y) memcpy(o->y, yc, sizeof(double) * (size_t)o->m);
    memcpy(o->x0, o->x, sizeof(double) * (size_t)o->n);
    memcpy(o->y0, o->y, sizeof(double) * (size_t)o->m);
    memset(o->sx, 0, sizeof(double) * (size_t)o->n);
    memset(o->sy, 0, sizeof(double) * (size_t)o->m);
    o->t = 0;
    o->nrst += 1;
    o->rho_prev = rho;
}

/* One PDHG step (eq. PDHG-update) for the LP saddle problem. */
static void pdhg_step1(orc_t *o)
{
    int64_t n = o->n, m = o->m;
    mat_tvec(o, o->y, o->aty);
    ORC_PAR_FOR
    for (int64_t j = 0; j < n; ++j)
        o->xn[j] = clampd(o->x[j] - o->tau * (o->c[j] - o->aty[j]), o->l[j], o->u[j]);
    ORC_PAR_FOR
    for (int64_t j = 0; j < n; ++j) o->e[j] = 2.0 * o->xn[j] - o->x[j];
    mat_vec(o, o->e, o->ax);
    ORC_PAR_FOR
    for (int64_t i = 0; i < m; ++i) {
        double yy = o->y[i] + o->sigma * (o->b[i] - o->ax[i]);
        if (o->kind[i] && yy < 0.0) yy = 0.0;
        o->yn[i] = yy;
    }
    memcpy(o->x, o->xn, sizeof(double) * (size_t)n);
    memcpy(o->y, o->yn, sizeof(double) * (size_t)m);
    ORC_PAR_FOR
    for (int64_t j = 0; j < n; ++j) o->sx[j] += o->x[j];
    ORC_PAR_FOR
    for (int64_t i = 0; i < m; ++i) o->sy[i] += o->y[i];
    o->t += 1;
    o->k += 1;
}

/*
 * One extragradient step (eq. extra-gradient-update) for the LP saddle
 * problem, F(z) = (c - A'y, Ax - b), with the step scaled per block as in
 * PDHG (primal tau, dual sigma): the target z~ = proj_Z(z - D F(z)), then
 * z+ = proj_Z(z - D F(z~)), D = diag(tau I, sigma I).  Four products with
 * A or A'.  Algorithm 1 averages the targets z~.
 */
static void egm_step1(orc_t *o)
{
    int64_t n = o->n, m = o->m;
    /* F at z */
    mat_tvec(o, o->y, o->aty);
    mat_vec(o, o->x, o->ax);
    for (int64_t j = 0; j < n; ++j)
        o->xt[j] = clampd(o->x[j] - o->tau * (o->c[j] - o->aty[j]), o->l[j], o->u[j]);
    for (int64_t i = 0; i < m; ++i) {
        double yy = o->y[i] - o->sigma * (o->ax[i] - o->b[i]);
        if (o->kind[i] && yy < 0.0) yy = 0.0;
        o->yt[i] = yy;
    }
    /* F at z~, applied from z */
    mat_tvec(o, o->yt, o->aty);
    mat_vec(o, o->xt, o->ax);
    for (int64_t j = 0; j < n; ++j)
        o->x[j] = clampd(o->x[j] - o->tau * (o->c[j] - o->aty[j]), o->l[j], o->u[j]);
    for (int64_t i = 0; i < m; ++i) {
        double yy = o->y[i] - o->sigma * (o->ax[i] - o->b[i]);
        if (o->kind[i] && yy < 0.0) yy = 0.0;
        o->y[i] = yy;
    }
    for (int64_t j = 0; j < n; ++j) o->sx[j] += o->xt[j];
    for (int64_t i = 0; i < m; ++i) o->sy[i] += o->yt[i];
    o->t += 1;
    o->k += 1;
}

/* 0: PDHG (eq. PDHG-update), 1: extragradient (eq. extra-gradient-update) */
void orc_set_method(orc_t *o, int32_t method)
{
    o->method = method == ORC_METHOD_EGM ? ORC_METHOD_EGM : ORC_METHOD_PDHG;
}

/* Inner iterations of Algorithm 1.  With fixed-length restarts
 * (eq. define:t-star) the outer loop restarts as soon as t reaches the
 * length, at any iteration. */
void orc_step(orc_t *o, int64_t iters)
{
    for (int64_t s = 0; s < iters; ++s) {
        if (o->method == ORC_METHOD_EGM) egm_step1(o);
        else pdhg_step1(o);
        if (o->mode == ORC_MODE_FIXED && o->fixed_len > 0 && o->t >= o->fixed_len) {
            average(o, o->xa, o->ya);
            restart_to(o, o->xa, o->ya, 0.0);
        }
    }
}

static double kkt_pick(const orc_t *o, const double *parts)
{
    if (o->kkt_kind == ORC_KKT_PAPER_ABS) return parts[5];
    if (o->kkt_kind == ORC_KKT_MAX_ABS) return parts[6];
    return parts[0];
}

/* KKT parts at the current point (which = 0), the average (1) or the
 * restart anchor z^{n,0} (2). */
void orc_kkt(orc_t *o, int32_t which, double *out)
{
    const double *x = o->x, *y = o->y;
    if (which == 1) { average(o, o->xa, o->ya); x = o->xa; y = o->ya; }
    if (which == 2) { x = o->x0; y = o->y0; }
    mat_vec(o, x, o->axa);
    mat_tvec(o, y, o->atya);
    kkt_parts(o, x, y, o->axa, o->atya, out);
}

/* rho at the current point (0), the average (1) or the anchor (2), with
 * the radius its distance to the anchor z^{n,0}, unless r >= 0 is given. */
double orc_gap(orc_t *o, int32_t which, double r, double *r_out, double *lambda_out)
{
    const double *x = o->x, *y = o->y;
    if (which == 1) { average(o, o->xa, o->ya); x = o->xa; y = o->ya; }
    if (which == 2) { x = o->x0; y = o->y0; }
    if (r < 0.0) r = sqrt(wnorm2(o, x, y, o->x0, o->y0));
    if (r_out) *r_out = r;
    mat_vec(o, x, o->axa);
    mat_tvec(o, y, o->atya);
    return gap_at(o, x, y, o->axa, o->atya, r, lambda_out);
}

static void log_push(orc_t *o, const double *rec)
{
    if (o->log_len + 1 > o->log_cap) {
        o->log_cap = o->log_cap ? 2 * o->log_cap : 64;
        o->log = (double *)realloc(o->log, sizeof(double) * ORC_REC * (size_t)o->log_cap);
    }
    memcpy(o->log + ORC_REC * o->log_len, rec, sizeof(double) * ORC_REC);
    o->log_len += 1;
}

/*
 * One check (termination, then the restart test of Algorithm 1).
 * Record (ORC_REC doubles):
 *  [0] k  [1] t  [2] restarts before  [3] KKT at z  [4] KKT at z-bar
 *  [5] r-bar = ||z-bar - z^{n,0}||  [6] rho at z-bar  [7] r = ||z - z^{n,0}||
 *  [8] rho at z (flexible only, else -1)  [9] restarted (0/1)
 *  [10] candidate (0 = z-bar, 1 = z)  [11] converged point (-1 none,
 *  0 = z, 1 = z-bar)  [12] rho_prev used by the test  [13] lambda at z-bar
 * Returns 1 when converged (tol > 0 and a KKT value at most tol).
 */
int32_t orc_check(orc_t *o, double tol, double *rec_out)
{
    double rec[ORC_REC];
    double pc[7], pa[7];
    for (int q = 0; q < ORC_REC; ++q) rec[q] = 0.0;
    rec[0] = (double)o->k; rec[1] = (double)o->t; rec[2] = (double)o->nrst;
    rec[8] = -1.0; rec[11] = -1.0; rec[12] = o->rho_prev;
    /* KKT at z (A x and A'y of the current point) */
    mat_vec(o, o->x, o->ax);
    mat_tvec(o, o->y, o->aty);
    kkt_parts(o, o->x, o->y, o->ax, o->aty, pc);
    /* KKT at the average */
    average(o, o->xa, o->ya);
    mat_vec(o, o->xa, o->axa);
    mat_tvec(o, o->ya, o->atya);
    kkt_parts(o, o->xa, o->ya, o->axa, o->atya, pa);
    double kc = kkt_pick(o, pc), ka = kkt_pick(o, pa);
    rec[3] = kc; rec[4] = ka;
    int32_t conv = 0;
    if (tol > 0.0 && (kc <= tol || ka <= tol)) {
        conv = 1;
        rec[11] = (ka <= kc) ? 1.0 : 0.0;
    }
    int adaptive = (o->mode == ORC_MODE_ADAPTIVE || o->mode == ORC_MODE_FLEXIBLE);
    if (!conv && adaptive && o->t > 0) {
        double ra = sqrt(wnorm2(o, o->xa, o->ya, o->x0, o->y0));
        double lam = 0.0;
        double rho_a = gap_at(o, o->xa, o->ya, o->axa, o->atya, ra, &lam);
        rec[5] = ra; rec[6] = rho_a; rec[13] = lam;
        double rho_c = rho_a;
        int cand_cur = 0;
        if (o->mode == ORC_MODE_FLEXIBLE) {
            double rc = sqrt(wnorm2(o, o->x, o->y, o->x0, o->y0));
            double rho_z = gap_at(o, o->x, o->y, o->ax, o->aty, rc, NULL);
            rec[7] = rc; rec[8] = rho_z;
            if (rho_z < rho_a) { cand_cur = 1; rho_c = rho_z; } /* strict, Remark rem:flexible */
        }
        int restart;
        if (o->nrst == 0) restart = (o->t >= o->tau0);
        else restart = (rho_c <= o->beta * o->rho_prev);
        rec[10] = (double)cand_cur;
        if (restart) {
            rec[9] = 1.0;
            if (cand_cur) restart_to(o, o->x, o->y, rho_c);
            else restart_to(o, o->xa, o->ya, rho_c);
        }
    }
    log_push(o, rec);
    if (rec_out) memcpy(rec_out, rec, sizeof(rec));
    return conv;
}

/*
 * Run up to `budget` more iterations, checking whenever the global
 * iteration count is a multiple of the check period (Section 7: the
 * restart test and the stopping test every 30 iterations).
 * result: [0] status (0 converged, 1 budget used) [1] k [2] restarts
 *         [3] KKT of the returned point [4] which (0 z, 1 z-bar, -1 none)
 *         [5] pobj [6] dobj
 * When converged, out_x/out_y (if given) receive the converged point.
 */
int32_t orc_solve(orc_t *o, int64_t budget, double tol, double *result,
                  double *out_x, double *out_y)
{
    int64_t k_end = o->k + budget;
    int32_t status = 1;
    double rec[ORC_REC];
    rec[11] = -1.0;
    while (o->k < k_end) {
        int64_t to_check = o->period - (o->k % o->period);
        int64_t s = k_end - o->k;
        if (to_check < s) s = to_check;
        orc_step(o, s);
        if (o->k % o->period == 0) {
            /* snapshot both points before the check may restart */
            average(o, o->xa, o->ya);
            if (orc_check(o, tol, rec)) { status = 0; break; }
        }
    }
    double parts[7] = {0};
    int which = (status == 0) ? (int)rec[11] : 0;
    if (status == 0 && which == 1) {
        mat_vec(o, o->xa, o->axa);
        mat_tvec(o, o->ya, o->atya);
        kkt_parts(o, o->xa, o->ya, o->axa, o->atya, parts);
        if (out_x) memcpy(out_x, o->xa, sizeof(double) * (size_t)o->n);
        if (out_y) memcpy(out_y, o->ya, sizeof(double) * (size_t)o->m);
    } else {
        mat_vec(o, o->x, o->ax);
        mat_tvec(o, o->y, o->aty);
        kkt_parts(o, o->x, o->y, o->ax, o->aty, parts);
        if (out_x) memcpy(out_x, o->x, sizeof(double) * (size_t)o->n);
        if (out_y) memcpy(out_y, o->y, sizeof(double) * (size_t)o->m);
    }
    if (result) {
        result[0] = (double)status;
        result[1] = (double)o->k;
        result[2] = (double)o->nrst;
        result[3] = kkt_pick(o, parts);
        result[4] = status == 0 ? (double)which : -1.0;
        result[5] = parts[3];
        result[6] = parts[4];
    }
    return status;
}

/* which: 0 current z, 1 average z-bar, 2 anchor z^{n,0}, 3 running sums */
void orc_get(orc_t *o, int32_t which, double *x, double *y)
{
    if (which == 0) {
        memcpy(x, o->x, sizeof(double) * (size_t)o->n);
        memcpy(y, o->y, sizeof(double) * (size_t)o->m);
    } else if (which == 1) {
        average(o, x, y);
    } else if (which == 2) {
        memcpy(x, o->x0, sizeof(double) * (size_t)o->n);
        memcpy(y, o->y0, sizeof(double) * (size_t)o->m);
    } else {
        memcpy(x, o->sx, sizeof(double) * (size_t)o->n);
        memcpy(y, o->sy, sizeof(double) * (size_t)o->m);
    }
}

/* Replace the current point (and the restart anchor) and clear the window;
 * the restart count and rho_prev are left as they are. */
void orc_set_point(orc_t *o, const double *x, const double *y)
{
    memcpy(o->x, x, sizeof(double) * (size_t)o->n);
    memcpy(o->y, y, sizeof(double) * (size_t)o->m);
    memcpy(o->x0, x, sizeof(double) * (size_t)o->n);
    memcpy(o->y0, y, sizeof(double) * (size_t)o->m);
    memset(o->sx, 0, sizeof(double) * (size_t)o->n);
    memset(o->sy, 0, sizeof(double) * (size_t)o->m);
    o->t = 0;
}

int64_t orc_log_len(const orc_t *o) { return o->log_len; }

void orc_log_copy(const orc_t *o, double *out)
{
    if (o->log_len)
        memcpy(out, o->log, sizeof(double) * ORC_REC * (size_t)o->log_len);
}

/* ------------------------------------------------------------------ */
/* Stand-alone pieces for tests: KKT and gap at arbitrary points.        */
/* ------------------------------------------------------------------ */
void orc_kkt_at(orc_t *o, const double *x, const double *y, double *out)
{
    mat_vec(o, x, o->axa);
    mat_tvec(o, y, o->atya);
    kkt_parts(o, x, y, o->axa, o->atya, out);
}

double orc_gap_at(orc_t *o, const double *x, const double *y, double r,
                  double *lambda_out)
{
    mat_vec(o, x, o->axa);
    mat_tvec(o, y, o->atya);
    return gap_at(o, x, y, o->axa, o->atya, r, lambda_out);
}

/* one PDHG step applied to an arbitrary point, leaving the handle's state */
void orc_pdhg_map(orc_t *o, const double *x, const double *y, double *xo, double *yo)
{
    int64_t n = o->n, m = o->m;
    mat_tvec(o, y, o->atya);
    for (int64_t j = 0; j < n; ++j)
        xo[j] = clampd(x[j] - o->tau * (o->c[j] - o->atya[j]), o->l[j], o->u[j]);
    for (int64_t j = 0; j < n; ++j) o->e[j] = 2.0 * xo[j] - x[j];
    mat_vec(o, o->e, o->axa);
    for (int64_t i = 0; i < m; ++i) {
        double yy = y[i] + o->sigma * (o->b[i] - o->axa[i]);
        if (o->kind[i] && yy < 0.0) yy = 0.0;
        yo[i] = yy;
    }
}

void orc_matvec(orc_t *o, const double *x, double *out) { mat_vec(o, x, out); }
void orc_matvec_t(orc_t *o, const double *y, double *out) { mat_tvec(o, y, out); }

/* ------------------------------------------------------------------ */
/* Differentiation of K unrolled restarted-PDHG iterations.             */
/*                                                                      */
/* The forward pass is the solve loop above from the initial point with */
/* no stopping test (checks still decide restarts).  Restart decisions  */
/* and projection masks are frozen; what remains is the chain rule     */
/* through eq. PDHG-update, the running average (Algorithm 1) and the   */
/* restart line of Algorithm 1:                                         */
/*   u = x - tau (c - A'y),   x+ = proj_X(u)    (derivative: 1 inside)  */
/*   w = 2 x+ - x,  v = y + sigma (b - A w),  y+ = proj_Y(v)            */
/*   S_x += x+, S_y += y+; at a restart to the average x = S_x / T      */
/* The loss is |x_K - x_target|^2 with x_K the primal point after K     */
/* iterations (including a restart at iteration K).                     */
/* ------------------------------------------------------------------ */
static void reinit(orc_t *o)
{
    for (int64_t j = 0; j < o->n; ++j) {
        o->x[j] = clampd(0.0, o->l[j], o->u[j]);
        o->x0[j] = o->x[j];
        o->sx[j] = 0.0;
    }
    for (int64_t i = 0; i < o->m; ++i) {
        o->y[i] = 0.0;
        o->y0[i] = 0.0;
        o->sy[i] = 0.0;
    }
    o->k = 0; o->t = 0; o->nrst = 0; o->rho_prev = 0.0; o->log_len = 0;
}

typedef struct {
    int64_t K;
    double *X, *Y;       /* iterate after step k, k = 0..K (row k) */
    int8_t *ev;          /* restart after step k: 0 none, 1 to average, 2 to current */
    int64_t *T;          /* window length of that restart */
    double **XR, **YR;   /* restart point after step k (when ev[k] == 1) */
} tape_t;

static void tape_free(tape_t *tp)
{
    if (tp->XR) for (int64_t k = 0; k <= tp->K; ++k) { free(tp->XR[k]); free(tp->YR[k]); }
    free(tp->X); free(tp->Y); free(tp->ev); free(tp->T); free(tp->XR); free(tp->YR);
}

/* forward pass recording the iterates and the restart events */
static void unrolled_forward(orc_t *o, int64_t K, tape_t *tp)
{
    int64_t n = o->n, m = o->m;
    tp->K = K;
    tp->X = dalloc((K + 1) * n);
    tp->Y = dalloc((K + 1) * (m > 0 ? m : 1));
    tp->ev = (int8_t *)calloc((size_t)(K + 1), 1);
    tp->T = (int64_t *)calloc((size_t)(K + 1), sizeof(int64_t));
    tp->XR = (double **)calloc((size_t)(K + 1), sizeof(double *));
    tp->YR = (double **)calloc((size_t)(K + 1), sizeof(double *));
    reinit(o);
    memcpy(tp->X, o->x, sizeof(double) * (size_t)n);
    memcpy(tp->Y, o->y, sizeof(double) * (size_t)m);
    for (int64_t k = 1; k <= K; ++k) {
        int64_t r0 = o->nrst;
        pdhg_step1(o);
        memcpy(tp->X + k * n, o->x, sizeof(double) * (size_t)n);
        memcpy(tp->Y + k * m, o->y, sizeof(double) * (size_t)m);
        int64_t tlen = o->t;
        if (o->mode == ORC_MODE_FIXED && o->fixed_len > 0 && o->t >= o->fixed_len) {
            average(o, o->xa, o->ya);
            restart_to(o, o->xa, o->ya, 0.0);
        } else if (o->k % o->period == 0) {
            double rec[ORC_REC];
            orc_check(o, 0.0, rec);
            if (o->nrst > r0 && rec[10] == 1.0) {
                tp->ev[k] = 2;
                tp->T[k] = tlen;
                continue;
            }
        }
        if (o->nrst > r0) {
            tp->ev[k] = 1;
            tp->T[k] = tlen;
            tp->XR[k] = dalloc(n);
            tp->YR[k] = dalloc(m);
            memcpy(tp->XR[k], o->x, sizeof(double) * (size_t)n);
            memcpy(tp->YR[k], o->y, sizeof(double) * (size_t)m);
        }
    }
}

static const double *tape_x_in(const tape_t *tp, int64_t k, int64_t n)
{   /* the primal point entering step k */
    return tp->ev[k - 1] == 1 ? tp->XR[k - 1] : tp->X + (k - 1) * n;
}

static const double *tape_y_in(const tape_t *tp, int64_t k, int64_t m)
{
    return tp->ev[k - 1] == 1 ? tp->YR[k - 1] : tp->Y + (k - 1) * m;
}

/*
 * Loss |x_K - x_target|^2 and its gradient with respect to c (n), b (m)
 * and the stored values of A (nnz, CSR order), by a reverse sweep over
 * the recorded iterates.  x_K (n) is returned in xK_out when given.
 */
double orc_unrolled_grad(orc_t *o, int64_t K, const double *x_target, double *gc,
                         double *gb, double *gA, double *xK_out)
{
    int64_t n = o->n, m = o->m;
    tape_t tp;
    memset(&tp, 0, sizeof(tp));
    unrolled_forward(o, K, &tp);
    const double *xK = o->x;
    double loss = 0.0;
    double *xh = dalloc(n), *yh = dalloc(m), *sxh = dalloc(n), *syh = dalloc(m);
    double *vh = dalloc(m), *wh = dalloc(n), *uh = dalloc(n), *au = dalloc(m);
    for (int64_t j = 0; j < n; ++j) {
        double d = xK[j] - x_target[j];
        loss += d * d;
        xh[j] = 2.0 * d;
    }
    if (xK_out) memcpy(xK_out, xK, sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) gc[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) gb[i] = 0.0;
    for (int64_t p = 0; p < o->nnz; ++p) gA[p] = 0.0;
    for (int64_t k = K; k >= 1; --k) {
        /* restart after step k: x = S_x / T (average) or the current point */
        if (tp.ev[k] == 1) {
            double T = (double)tp.T[k];
            for (int64_t j = 0; j < n; ++j) { sxh[j] = xh[j] / T; xh[j] = 0.0; }
            for (int64_t i = 0; i < m; ++i) { syh[i] = yh[i] / T; yh[i] = 0.0; }
        } else if (tp.ev[k] == 2) {
            for (int64_t j = 0; j < n; ++j) sxh[j] = 0.0;
            for (int64_t i = 0; i < m; ++i) syh[i] = 0.0;
        }
        const double *xin = tape_x_in(&tp, k, n), *yin = tape_y_in(&tp, k, m);
        const double *xout = tp.X + k * n, *yout = tp.Y + k * m;
        /* dual half-step */
        for (int64_t i = 0; i < m; ++i) {
            int inside = !o->kind[i] || yout[i] > 0.0;
            vh[i] = inside ? yh[i] + syh[i] : 0.0;
            gb[i] += o->sigma * vh[i];
        }
        mat_tvec(o, vh, wh);
        for (int64_t j = 0; j < n; ++j) wh[j] = -o->sigma * wh[j];
        /* primal half-step */
        for (int64_t j = 0; j < n; ++j) {
            double tot = xh[j] + sxh[j] + 2.0 * wh[j];
            int inside = o->l[j] < xout[j] && xout[j] < o->u[j];
            uh[j] = inside ? tot : 0.0;
            gc[j] += -o->tau * uh[j];
        }
        mat_vec(o, uh, au);
        for (int64_t i = 0; i < o->m; ++i)
            for (int32_t p = o->rp[i]; p < o->rp[i + 1]; ++p) {
                int32_t j = o->ci[p];
                double w = 2.0 * xout[j] - xin[j];
                gA[p] += -o->sigma * vh[i] * w + o->tau * yin[i] * uh[j];
            }
        for (int64_t j = 0; j < n; ++j) xh[j] = -wh[j] + uh[j];
        for (int64_t i = 0; i < m; ++i) yh[i] = vh[i] + o->tau * au[i];
    }
    free(xh); free(yh); free(sxh); free(syh); free(vh); free(wh); free(uh); free(au);
    tape_free(&tp);
    return loss;
}

/*
 * Tangent (forward-mode) derivative of x_K in the direction (dc, db, dA)
 * along the same frozen decisions; dxK (n).
 */
void orc_unrolled_tangent(orc_t *o, int64_t K, const double *dc, const double *db,
                          const double *dA, double *dxK)
{
    int64_t n = o->n, m = o->m;
    tape_t tp;
    memset(&tp, 0, sizeof(tp));
    unrolled_forward(o, K, &tp);
    double *xd = dalloc(n), *yd = dalloc(m), *sxd = dalloc(n), *syd = dalloc(m);
    double *t1 = dalloc(n), *t2 = dalloc(m), *xo = dalloc(n), *wd = dalloc(n);
    for (int64_t k = 1; k <= K; ++k) {
        const double *xin = tape_x_in(&tp, k, n), *yin = tape_y_in(&tp, k, m);
        const double *xout = tp.X + k * n, *yout = tp.Y + k * m;
        /* u' = x' - tau (c' - (dA' y + A' y')) */
        for (int64_t j = 0; j < n; ++j) t1[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            for (int32_t p = o->rp[i]; p < o->rp[i + 1]; ++p)
                t1[o->ci[p]] += dA[p] * yin[i] + o->v[p] * yd[i];
        for (int64_t j = 0; j < n; ++j) {
            double ud = xd[j] - o->tau * (dc[j] - t1[j]);
            int inside = o->l[j] < xout[j] && xout[j] < o->u[j];
            xo[j] = inside ? ud : 0.0;
            wd[j] = 2.0 * xo[j] - xd[j];
        }
        /* v' = y' + sigma (b' - (dA w + A w')) */
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int32_t p = o->rp[i]; p < o->rp[i + 1]; ++p) {
                int32_t j = o->ci[p];
                s += dA[p] * (2.0 * xout[j] - xin[j]) + o->v[p] * wd[j];
            }
            double vd = yd[i] + o->sigma * (db[i] - s);
            int inside = !o->kind[i] || yout[i] > 0.0;
            t2[i] = inside ? vd : 0.0;
        }
        memcpy(xd, xo, sizeof(double) * (size_t)n);
        memcpy(yd, t2, sizeof(double) * (size_t)m);
        for (int64_t j = 0; j < n; ++j) sxd[j] += xd[j];
        for (int64_t i = 0; i < m; ++i) syd[i] += yd[i];
        if (tp.ev[k] == 1) {
            double T = (double)tp.T[k];
            for (int64_t j = 0; j < n; ++j) { xd[j] = sxd[j] / T; sxd[j] = 0.0; }
            for (int64_t i = 0; i < m; ++i) { yd[i] = syd[i] / T; syd[i] = 0.0; }
        } else if (tp.ev[k] == 2) {
            for (int64_t j = 0; j < n; ++j) sxd[j] = 0.0;
            for (int64_t i = 0; i < m; ++i) syd[i] = 0.0;
        }
    }
    memcpy(dxK, xd, sizeof(double) * (size_t)n);
    free(xd); free(yd); free(sxd); free(syd); free(t1); free(t2); free(xo); free(wd);
    tape_free(&tp);
}

/* x_K of the same forward pass (for finite differences) */
void orc_unrolled_value(orc_t *o, int64_t K, double *xK)
{
    tape_t tp;
    memset(&tp, 0, sizeof(tp));
    unrolled_forward(o, K, &tp);
    memcpy(xK, o->x, sizeof(double) * (size_t)o->n);
    tape_free(&tp);
}

/* restart events of the last unrolled forward pass are visible through the
 * check log; this reports the iterations at which restarts happened */
int64_t orc_restart_iters(orc_t *o, int64_t K, int64_t *out, int64_t cap)
{
    tape_t tp;
    memset(&tp, 0, sizeof(tp));
    unrolled_forward(o, K, &tp);
    int64_t c = 0;
    for (int64_t k = 1; k <= K; ++k)
        if (tp.ev[k]) {
            if (c < cap) out[c] = k;
            ++c;
        }
    tape_free(&tp);
    return c;
}

/* Hash of every projection mask and restart event of the unrolled
 * forward pass: runs with equal hashes took the same piecewise-linear
 * branch, so finite differences between them see no kink. */
uint64_t orc_branch_signature(orc_t *o, int64_t K)
{
    tape_t tp;
    memset(&tp, 0, sizeof(tp));
    unrolled_forward(o, K, &tp);
    uint64_t h = 1469598103934665603ULL;
    for (int64_t k = 1; k <= K; ++k) {
        const double *xo = tp.X + k * o->n, *yo = tp.Y + k * o->m;
        for (int64_t j = 0; j < o->n; ++j) {
            uint64_t bit = (o->l[j] < xo[j] && xo[j] < o->u[j]) ? 1u : 0u;
            h = (h ^ bit) * 1099511628211ULL;
        }
        for (int64_t i = 0; i < o->m; ++i) {
            uint64_t bit = (!o->kind[i] || yo[i] > 0.0) ? 1u : 0u;
            h = (h ^ bit) * 1099511628211ULL;
        }
        h = (h ^ (uint64_t)tp.ev[k]) * 1099511628211ULL;
    }
    tape_free(&tp);
    return h;
}
