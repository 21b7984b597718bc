/*
 * Plain FP64 reference implementation of the Scylla LP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the library never calls, links or includes it, and it
 * shares no code with the library (its own transpose-free products, its own
 * preconditioner, its own residuals).
 *
 * What it computes (Mexi et al., "Scylla", Section 2 and Algorithm 1):
 *   - orc_precondition : diagonal preconditioning that the paper delegates to
 *                        PDLP (Section 2.1), read as 10 Ruiz rounds in the
 *                        infinity norm followed by one Pock-Chambolle
 *                        (alpha = 1) round; A itself is never rescaled.
 *   - orc_pdhg         : the PDHG inner loop of Algorithm 1 (primal step
 *                        d_x = A^T y - c_hat, projection on [l, u]; dual step
 *                        d_y = b - A(2 x+ - x), projection on the dual sign
 *                        cone), with diagonal step sizes, a relative-KKT
 *                        termination test (Section 2.2) and a KKT-based
 *                        restart-to-current scheme with primal-weight update
 *                        (Section 2.1 names restarts and step sizes without
 *                        detail; the constants are readings, listed below).
 *   - orc_kkt          : relative primal / dual / gap errors of (x, y) on the
 *                        original problem (Section 2.2).
 *   An optional diagonal Hessian q (the quadratic objectives Section 5
 *   proposes: diagonal-Hessian QPs, and the L2 distance of the objective
 *   update) enters the primal proximal step exactly and the KKT test through
 *   the reduced cost and both objectives.
 *   - orc_fix_propagate: fix-and-propagate rounding (Section 2.3).
 *   - orc_fix_propagate_batched: the same rounding with K variables fixed at
 *                        a time and synchronous propagation rounds (a
 *                        parallel form of Section 2.3; rules at the function).
 *
 * Readings where the paper is silent (each is restated in the design notes):
 *   - rows may be >=, <= or = (the paper writes only >=); the dual cone is
 *     R+ for >=, R- for <=, R for = (Lagrangian c^T x - y^T (A x - b)).
 *   - the start point is the projection of 0 (or of the warm start) onto the
 *     bounds and the dual cone.
 *   - step sizes: t = eta / omega, s = eta * omega on the preconditioned
 *     problem, eta = 0.99 by default; omega (the primal weight) starts at
 *     ||D_c c|| / ||D_r b|| and only changes at restarts.
 *   - KKT: rho_p = ||r_p|| / (1 + ||b||), rho_d = ||c_hat - A^T y - lambda||
 *     / (1 + ||c_hat||), rho_g = |P - D| / (1 + |P| + |D|); rel = max of the
 *     three; checked every R iterations, at 0 and at the iteration limit.
 *   - restart when E <= 0.2 E_r, or E <= 0.8 E_r and E > E_prev, or
 *     k - k_r >= 0.36 k; omega <- exp(0.5 ln(|dy|/|dx|) + 0.5 ln omega).
 *   - infeasibility (after PDLP; the paper has no infeasible relaxations):
 *     at every check after the first, with d = x - x_prev and v = y - y_prev
 *     the moves since the previous check, v is a dual ray (primal
 *     infeasible) when rho = b^T v + sum_j (l_j lam_j^+ + u_j lam_j^-) > 0
 *     for lam = proj_Lambda(-A^T v) and |A^T v + lam| (+ |v - proj_Y v|) <=
 *     infeas_tol * rho; d is a primal ray (dual infeasible) when c^T d < 0
 *     and the violation of A d against the row cones, of d against the
 *     bounds' recession cone (and |Q d|) is <= infeas_tol * |c^T d|.  The
 *     optimality test comes first.
 *   - "bounds stalling" (an exit of Algorithm 1's inner loop, not defined
 *     further): the primal and the dual objective, the two bounds on the
 *     LP optimum the iteration maintains, both move by at most
 *     stall_tol (1 + |value|) between consecutive checks, stall_checks
 *     checks in a row (tested after the optimality and infeasibility tests,
 *     before the iteration limit; off when stall_tol = 0).
 *   - adaptive step size ("update step sizes" in Algorithm 1, after PDLP):
 *     after the k-th iteration (k counted from 1 over the whole call), with
 *     dx = x+ - x and dy = y+ - y in the preconditioned metric,
 *     eta_bar = (omega |D_c^-1 dx|^2 + |D_r^-1 dy|^2 / omega) / (2 |dy^T A dx|)
 *     and eta <- min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta); the
 *     iterate is always kept (PDLP would retry a step with eta > eta_bar);
 *     eta_bar = infinity when dy^T A dx = 0, and eta stays when dx = dy = 0.
 *     eta starts at the eta parameter.
 *   - restart to the average (PDLP's restart candidates; option): z_avg is
 *     the running mean of the iterates produced since the last restart (or
 *     since the start), equal weights: the first iterate after a restart
 *     starts it, later ones update z_avg += (z - z_avg) / count.  At every check after the first the candidate
 *     is z_avg if its relative KKT error is below the current iterate's,
 *     else the current iterate (ties: current); its error E is what the
 *     termination test, the restart rule and E_prev use, and the candidate
 *     is what a restart restarts to and what an OPTIMAL or
 *     iteration-limit stop returns.  Infeasibility and stalling are tested
 *     on the current iterate.  A restart starts a new average.
 *
 * Build: gcc -O2 -std=c11 -shared -fPIC -o liboracle.so scylla_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t m, n;
    const int64_t *row_ptr; /* [m+1] */
    const int32_t *col_idx; /* [nnz] */
    const double *val;      /* [nnz] */
    const double *c;        /* [n] objective (the current c_hat) */
    const double *b;        /* [m] */
    const char *sense;      /* [m] 'G', 'L' or 'E' */
    const double *l, *u;    /* [n], may be -inf / +inf */
    const double *q;        /* [n] diagonal Hessian >= 0, or NULL (LP) */
} orc_lp;

typedef struct {
    double tol;          /* relative KKT tolerance */
    int64_t iter_limit;  /* number of PDHG iterations allowed */
    int32_t check_period;/* R */
    int32_t restarts;    /* 1: restart scheme on, 0: off */
    double eta;          /* step-size safety factor */
    int32_t ruiz_iters;  /* Ruiz rounds (10) */
    int32_t pock_chambolle; /* 1: one Pock-Chambolle round after Ruiz */
    double omega0;       /* > 0: use as primal weight, else from norms */
    int32_t adaptive;    /* 1: adaptive step size (PDLP's rule, no retry) */
    double infeas_tol;   /* > 0: infeasibility certificates at the checks */
    double stall_tol;    /* > 0: stop when the objective bounds stall */
    int32_t stall_checks;/* consecutive checks without a move that stop */
    int32_t restart_avg; /* 1: the average of the iterates since the last
                            restart is a candidate at every check */
} orc_params;

enum { ORC_OPTIMAL = 1, ORC_ITERATION_LIMIT = 2, ORC_NUMERICAL_ERROR = 4, ORC_PRIMAL_INFEASIBLE = 5,
       ORC_DUAL_INFEASIBLE = 6, ORC_STALLED = 7 };

typedef struct {
    int32_t status;
    int32_t restarts;
    int64_t iterations;
    double rel_kkt, rho_p, rho_d, rho_g, pobj, dobj, omega;
    double eta;          /* step-size factor in effect at the end */
} orc_result;

/* ------------------------------------------------------------------ helpers */
static double clampd(double v, double lo, double hi)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    return v;
}

/* Projection onto the dual sign cone of one row (Algorithm 1 dual step). */
static double proj_dual(double v, char sense)
{
    if (sense == 'G') return v > 0.0 ? v : 0.0;
    if (sense == 'L') return v < 0.0 ? v : 0.0;
    return v;
}

/* y = A x, plain row-by-row definition. */
static void mul_A(const orc_lp *lp, const double *x, double *ax)
{
    for (int32_t i = 0; i < lp->m; ++i) {
        double s = 0.0;
        for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
            s += lp->val[e] * x[lp->col_idx[e]];
        ax[i] = s;
    }
}

/* z = A^T y, by the definition z_j = sum_i a_ij y_i (accumulated row by row). */
static void mul_At(const orc_lp *lp, const double *y, double *z)
{
    for (int32_t j = 0; j < lp->n; ++j) z[j] = 0.0;
    for (int32_t i = 0; i < lp->m; ++i)
        for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
            z[lp->col_idx[e]] += lp->val[e] * y[i];
}

static double norm2(const double *v, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* ------------------------------------------------------- preconditioning */
/*
 * Diagonal scaling D_r, D_c with A~ = D_r A D_c (Section 2.1: PDLP's matrix
 * preconditioning).  Ruiz: each round divides row i by sqrt(max_j |a~_ij|)
 * and column j by sqrt(max_i |a~_ij|), both maxima taken from the same A~.
 * Pock-Chambolle (alpha = 1): divide row i by sqrt(sum_j |a~_ij|) and
 * column j by sqrt(sum_i |a~_ij|).  Zero rows / columns keep their scale.
 */
int orc_precondition(const orc_lp *lp, int32_t ruiz_iters, int32_t pc, double *dr, double *dc)
{
    const int32_t m = lp->m, n = lp->n;
    double *rs = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *cs = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!rs || !cs) { free(rs); free(cs); return -1; }
    for (int32_t i = 0; i < m; ++i) dr[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) dc[j] = 1.0;
    for (int32_t it = 0; it < ruiz_iters; ++it) {
        for (int32_t i = 0; i < m; ++i) rs[i] = 0.0;
        for (int32_t j = 0; j < n; ++j) cs[j] = 0.0;
        for (int32_t i = 0; i < m; ++i)
            for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) {
                int32_t j = lp->col_idx[e];
                double a = fabs(dr[i] * lp->val[e] * dc[j]);
                if (a > rs[i]) rs[i] = a;
                if (a > cs[j]) cs[j] = a;
            }
        for (int32_t i = 0; i < m; ++i) if (rs[i] > 0.0) dr[i] /= sqrt(rs[i]);
        for (int32_t j = 0; j < n; ++j) if (cs[j] > 0.0) dc[j] /= sqrt(cs[j]);
    }
    if (pc) {
        for (int32_t i = 0; i < m; ++i) rs[i] = 0.0;
        for (int32_t j = 0; j < n; ++j) cs[j] = 0.0;
        for (int32_t i = 0; i < m; ++i)
            for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) {
                int32_t j = lp->col_idx[e];
                double a = fabs(dr[i] * lp->val[e] * dc[j]);
                rs[i] += a;
                cs[j] += a;
            }
        for (int32_t i = 0; i < m; ++i) if (rs[i] > 0.0) dr[i] /= sqrt(rs[i]);
        for (int32_t j = 0; j < n; ++j) if (cs[j] > 0.0) dc[j] /= sqrt(cs[j]);
    }
    free(rs);
    free(cs);
    return 0;
}

/* ------------------------------------------------------------------- KKT */
/*
 * Relative KKT errors of (x, y) on the original, unscaled problem
 * (Section 2.2: primal and dual feasibility errors; the gap is included).
 *   r_p,i = max(b_i - (Ax)_i, 0) (G), max((Ax)_i - b_i, 0) (L), b_i - (Ax)_i (E)
 *   g = c - A^T y;  lambda_j = projection of g_j onto R (both bounds finite),
 *   R+ (only l finite), R- (only u finite), {0} (free);  r_d = g - lambda
 *   P = c^T x;  D = b^T y + sum_{l finite} l_j max(lambda_j, 0)
 *                         - sum_{u finite} u_j max(-lambda_j, 0)
 * out[0..7] = rel, rho_p, rho_d, rho_g, P, D, ||b||, ||c||.
 */
int orc_kkt(const orc_lp *lp, const double *x, const double *y, double *out)
{
    const int32_t m = lp->m, n = lp->n;
    double *ax = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *aty = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!ax || !aty) { free(ax); free(aty); return -1; }
    mul_A(lp, x, ax);
    mul_At(lp, y, aty);
    double rp2 = 0.0, rd2 = 0.0, pobj = 0.0, dobj = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        double r;
        if (lp->sense[i] == 'G') r = fmax(lp->b[i] - ax[i], 0.0);
        else if (lp->sense[i] == 'L') r = fmax(ax[i] - lp->b[i], 0.0);
        else r = lp->b[i] - ax[i];
        rp2 += r * r;
        dobj += lp->b[i] * y[i];
    }
    for (int32_t j = 0; j < n; ++j) {
        /* with a diagonal Hessian: reduced cost c + Q x - A^T y; primal
           objective c^T x + x^T Q x / 2; dual objective
           b^T y - x^T Q x / 2 + bound terms (the QP dual at the same x) */
        const double qx = lp->q ? lp->q[j] * x[j] : 0.0;
        double g = lp->c[j] + qx - aty[j];
        int lf = isfinite(lp->l[j]), uf = isfinite(lp->u[j]);
        double lam;
        if (lf && uf) lam = g;
        else if (lf) lam = fmax(g, 0.0);
        else if (uf) lam = fmin(g, 0.0);
        else lam = 0.0;
        double rd = g - lam;
        rd2 += rd * rd;
        pobj += lp->c[j] * x[j] + 0.5 * qx * x[j];
        dobj -= 0.5 * qx * x[j];
        if (lf && lam > 0.0) dobj += lp->l[j] * lam;
        if (uf && lam < 0.0) dobj += lp->u[j] * lam;
    }
    double bn = norm2(lp->b, m), cn = norm2(lp->c, n);
    double rho_p = sqrt(rp2) / (1.0 + bn);
    double rho_d = sqrt(rd2) / (1.0 + cn);
    double rho_g = fabs(pobj - dobj) / (1.0 + fabs(pobj) + fabs(dobj));
    double rel = rho_p;
    if (rho_d > rel) rel = rho_d;
    if (rho_g > rel) rel = rho_g;
    if (!isfinite(rho_p) || !isfinite(rho_d) || !isfinite(rho_g)) rel = NAN;
    out[0] = rel; out[1] = rho_p; out[2] = rho_d; out[3] = rho_g;
    out[4] = pobj; out[5] = dobj; out[6] = bn; out[7] = cn;
    free(ax);
    free(aty);
    return 0;
}

/* ------------------------------------------------------------------ PDHG */
/*
 * Algorithm 1, inner loop.  With D_r, D_c from orc_precondition, PDHG with
 * scalar steps t, s on the preconditioned problem is, in the original
 * variables, the diagonal-step iteration
 *     d_x  = A^T y - c_hat
 *     x+   = proj_[l,u](x + t D_c^2 d_x)
 *     d_y  = b - A(2 x+ - x)
 *     y+   = proj_Y(y + s D_r^2 d_y)
 * Every R iterations (and at k = 0 and k = iter_limit) the KKT test decides
 * termination and, if enabled, a restart to the current point.
 */
/* Certificate quantities of the moves d = x - xp, v = y - yp (see the
 * infeasibility reading above): out = {rho, dual-ray residual, c^T d,
 * primal-ray violation}. */
int orc_ray(const orc_lp *lp, const double *x, const double *y, const double *xp, const double *yp,
            double *out)
{
    const int32_t m = lp->m, n = lp->n;
    double *d = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *v = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *ad = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *atv = malloc(sizeof(double) * (n > 0 ? n : 1));
    if (!d || !v || !ad || !atv) { free(d); free(v); free(ad); free(atv); return -1; }
    for (int32_t j = 0; j < n; ++j) d[j] = x[j] - xp[j];
    for (int32_t i = 0; i < m; ++i) v[i] = y[i] - yp[i];
    mul_A(lp, d, ad);
    mul_At(lp, v, atv);
    double rho = 0.0, rd2 = 0.0, cd = 0.0, pv2 = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        const double vp = proj_dual(v[i], lp->sense[i]);
        rho += lp->b[i] * v[i];
        rd2 += (v[i] - vp) * (v[i] - vp);
        double viol;  /* A d against the row's recession cone */
        if (lp->sense[i] == 'G') viol = fmax(-ad[i], 0.0);
        else if (lp->sense[i] == 'L') viol = fmax(ad[i], 0.0);
        else viol = ad[i];
        pv2 += viol * viol;
    }
    for (int32_t j = 0; j < n; ++j) {
        const int lf = isfinite(lp->l[j]), uf = isfinite(lp->u[j]);
        const double g = -atv[j];
        double lam;
        if (lf && uf) lam = g;
        else if (lf) lam = fmax(g, 0.0);
        else if (uf) lam = fmin(g, 0.0);
        else lam = 0.0;
        const double r = atv[j] + lam;
        rd2 += r * r;
        if (lf && lam > 0.0) rho += lp->l[j] * lam;
        if (uf && lam < 0.0) rho += lp->u[j] * lam;
        cd += lp->c[j] * d[j];
        double bv;  /* d against the bounds' recession cone */
        if (lf && uf) bv = d[j];
        else if (lf) bv = fmin(d[j], 0.0);
        else if (uf) bv = fmax(d[j], 0.0);
        else bv = 0.0;
        pv2 += bv * bv;
        if (lp->q) pv2 += (lp->q[j] * d[j]) * (lp->q[j] * d[j]);
    }
    out[0] = rho;
    out[1] = sqrt(rd2);
    out[2] = cd;
    out[3] = sqrt(pv2);
    free(d); free(v); free(ad); free(atv);
    return 0;
}

int orc_pdhg_avg(const orc_lp *lp, const orc_params *p, const double *x0, const double *y0,
                 double *x, double *y, double *xa_out, double *ya_out, orc_result *res);

int orc_pdhg(const orc_lp *lp, const orc_params *p, const double *x0, const double *y0,
             double *x, double *y, orc_result *res)
{
    return orc_pdhg_avg(lp, p, x0, y0, x, y, NULL, NULL, res);
}

/* orc_pdhg that also returns the running averages (restart_avg) at the stop,
 * before any candidate replaced the iterate; xa_out / ya_out may be NULL. */
int orc_pdhg_avg(const orc_lp *lp, const orc_params *p, const double *x0, const double *y0,
                 double *x, double *y, double *xa_out, double *ya_out, orc_result *res)
{
    const int32_t m = lp->m, n = lp->n;
    const int32_t R = p->check_period > 0 ? p->check_period : 64;
    double *dr = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *dc = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *xn = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *xbar = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *aty = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *axb = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *xr = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *yr = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *yn = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *dxv = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *adx = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *xp = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *yp = malloc(sizeof(double) * (m > 0 ? m : 1));
    double *xa = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *ya = malloc(sizeof(double) * (m > 0 ? m : 1));
    int rc = 0;
    if (!dr || !dc || !xn || !xbar || !aty || !axb || !xr || !yr || !yn || !dxv || !adx || !xp || !yp ||
        !xa || !ya) {
        rc = -1;
        goto done;
    }
    orc_precondition(lp, p->ruiz_iters, p->pock_chambolle, dr, dc);

    /* start point: projection of the warm start (or of 0) */
    for (int32_t j = 0; j < n; ++j) x[j] = clampd(x0 ? x0[j] : 0.0, lp->l[j], lp->u[j]);
    for (int32_t i = 0; i < m; ++i) y[i] = proj_dual(y0 ? y0[i] : 0.0, lp->sense[i]);

    double omega;
    if (p->omega0 > 0.0) {
        omega = p->omega0;
    } else {
        double cs = 0.0, bs = 0.0;
        for (int32_t j = 0; j < n; ++j) cs += (dc[j] * lp->c[j]) * (dc[j] * lp->c[j]);
        for (int32_t i = 0; i < m; ++i) bs += (dr[i] * lp->b[i]) * (dr[i] * lp->b[i]);
        cs = sqrt(cs);
        bs = sqrt(bs);
        omega = (cs > 0.0 && bs > 0.0) ? cs / bs : 1.0;
    }
    double eta = p->eta;
    double t = eta / omega, s = eta * omega;

    int64_t k = 0, kr = 0;
    double Er = 0.0, Ep = 0.0;
    double pprev = 0.0, dprev = 0.0;
    int32_t nstall = 0;
    int32_t nrestart = 0;
    int64_t na = 0; /* iterates in the running average */
    double kkt[8] = {0}, kkta[8] = {0};
    memset(res, 0, sizeof(*res));
    for (;;) {
        if (k % R == 0 || k >= p->iter_limit) {
            orc_kkt(lp, x, y, kkt);
            if (!isfinite(kkt[0])) { res->status = ORC_NUMERICAL_ERROR; break; }
            /* the candidate: the running average when its error is lower */
            int use_avg = 0;
            if (p->restart_avg && na > 0) {
                orc_kkt(lp, xa, ya, kkta);
                use_avg = kkta[0] < kkt[0];
            }
            double E = use_avg ? kkta[0] : kkt[0];
            if (E <= p->tol) {
                if (use_avg) {
                    memcpy(x, xa, sizeof(double) * n);
                    memcpy(y, ya, sizeof(double) * m);
                    memcpy(kkt, kkta, sizeof(kkt));
                }
                res->status = ORC_OPTIMAL;
                break;
            }
            if (p->infeas_tol > 0.0 && k > 0) {
                double ray[4];
                orc_ray(lp, x, y, xp, yp, ray);
                if (ray[0] > 0.0 && ray[1] <= p->infeas_tol * ray[0]) { res->status = ORC_PRIMAL_INFEASIBLE; break; }
                if (ray[2] < 0.0 && ray[3] <= -p->infeas_tol * ray[2]) { res->status = ORC_DUAL_INFEASIBLE; break; }
            }
            memcpy(xp, x, sizeof(double) * n);
            memcpy(yp, y, sizeof(double) * m);
            if (p->stall_tol > 0.0) {
                /* bounds stalling: the primal objective kkt[4] and the dual
                   objective kkt[5] both within stall_tol (1 + |value|) of
                   their values at the previous check, stall_checks checks
                   in a row */
                if (k > 0) {
                    int still = fabs(kkt[4] - pprev) <= p->stall_tol * (1.0 + fabs(kkt[4])) &&
                                fabs(kkt[5] - dprev) <= p->stall_tol * (1.0 + fabs(kkt[5]));
                    nstall = still ? nstall + 1 : 0;
                    if (nstall >= p->stall_checks) { res->status = ORC_STALLED; break; }
                }
                pprev = kkt[4];
                dprev = kkt[5];
            }
            if (k >= p->iter_limit) {
                if (use_avg) {
                    memcpy(x, xa, sizeof(double) * n);
                    memcpy(y, ya, sizeof(double) * m);
                    memcpy(kkt, kkta, sizeof(kkt));
                }
                res->status = ORC_ITERATION_LIMIT;
                break;
            }
            if (k == 0) {
                Er = E;
                for (int32_t j = 0; j < n; ++j) xr[j] = x[j];
                for (int32_t i = 0; i < m; ++i) yr[i] = y[i];
            } else if (p->restarts) {
                int fire = (E <= 0.2 * Er) || (E <= 0.8 * Er && E > Ep) ||
                           ((double)(k - kr) >= 0.36 * (double)k);
                if (fire) {
                    if (use_avg) {
                        memcpy(x, xa, sizeof(double) * n);
                        memcpy(y, ya, sizeof(double) * m);
                    }
                    double dx2 = 0.0, dy2 = 0.0;
                    for (int32_t j = 0; j < n; ++j) {
                        double d = (x[j] - xr[j]) / dc[j];
                        dx2 += d * d;
                    }
                    for (int32_t i = 0; i < m; ++i) {
                        double d = (y[i] - yr[i]) / dr[i];
                        dy2 += d * d;
                    }
                    double dx = sqrt(dx2), dy = sqrt(dy2);
                    if (dx > 1e-10 && dy > 1e-10) {
                        omega = exp(0.5 * log(dy / dx) + 0.5 * log(omega));
                        t = eta / omega;
                        s = eta * omega;
                    }
                    for (int32_t j = 0; j < n; ++j) xr[j] = x[j];
                    for (int32_t i = 0; i < m; ++i) yr[i] = y[i];
                    Er = E;
                    kr = k;
                    na = 0;
                    ++nrestart;
                }
            }
            Ep = E;
        }
        /* primal step: d_x = A^T y - c_hat, x+ = proj_[l,u](x + t D_c^2 d_x) */
        mul_At(lp, y, aty);
        for (int32_t j = 0; j < n; ++j) {
            /* proximal step; with a diagonal Hessian the one-dimensional
               problem min q x^2/2 + (c - A^T y) x + |x - x_j|^2 / (2 t D_c^2)
               over [l, u] is solved exactly: minimiser, then clamp */
            double dx = aty[j] - lp->c[j];
            double v = x[j] + t * (dc[j] * dc[j]) * dx;
            if (lp->q) v /= 1.0 + t * (dc[j] * dc[j]) * lp->q[j];
            xn[j] = clampd(v, lp->l[j], lp->u[j]);
            xbar[j] = 2.0 * xn[j] - x[j];
        }
        /* dual step: d_y = b - A(2 x+ - x), y+ = proj_Y(y + s D_r^2 d_y) */
        mul_A(lp, xbar, axb);
        for (int32_t i = 0; i < m; ++i) {
            double dy = lp->b[i] - axb[i];
            yn[i] = proj_dual(y[i] + s * (dr[i] * dr[i]) * dy, lp->sense[i]);
        }
        ++k;
        if (p->adaptive) {
            /* local step bound from this iteration's move */
            double nx = 0.0, ny = 0.0, inter = 0.0;
            for (int32_t j = 0; j < n; ++j) {
                dxv[j] = xn[j] - x[j];
                double d = dxv[j] / dc[j];
                nx += d * d;
            }
            mul_A(lp, dxv, adx);
            for (int32_t i = 0; i < m; ++i) {
                double d = yn[i] - y[i];
                inter += d * adx[i];
                d /= dr[i];
                ny += d * d;
            }
            if (nx + ny > 0.0) {
                double grow = (1.0 + pow((double)k + 1.0, -0.6)) * eta;
                if (inter != 0.0) {
                    double ebar = (omega * nx + ny / omega) / (2.0 * fabs(inter));
                    double shrink = (1.0 - pow((double)k + 1.0, -0.3)) * ebar;
                    eta = shrink < grow ? shrink : grow;
                } else {
                    eta = grow;
                }
                t = eta / omega;
                s = eta * omega;
            }
        }
        for (int32_t j = 0; j < n; ++j) x[j] = xn[j];
        for (int32_t i = 0; i < m; ++i) y[i] = yn[i];
        if (p->restart_avg) {
            /* the first iterate after a restart starts the mean */
            ++na;
            for (int32_t j = 0; j < n; ++j) xa[j] = na == 1 ? x[j] : xa[j] + (x[j] - xa[j]) / (double)na;
            for (int32_t i = 0; i < m; ++i) ya[i] = na == 1 ? y[i] : ya[i] + (y[i] - ya[i]) / (double)na;
        }
    }
    if (xa_out) {
        if (na > 0) memcpy(xa_out, xa, sizeof(double) * n);
        else memset(xa_out, 0, sizeof(double) * n);
    }
    if (ya_out) {
        if (na > 0) memcpy(ya_out, ya, sizeof(double) * m);
        else memset(ya_out, 0, sizeof(double) * m);
    }
    res->iterations = k;
    res->restarts = nrestart;
    res->rel_kkt = kkt[0];
    res->rho_p = kkt[1];
    res->rho_d = kkt[2];
    res->rho_g = kkt[3];
    res->pobj = kkt[4];
    res->dobj = kkt[5];
    res->omega = omega;
    res->eta = eta;
done:
    free(dr); free(dc); free(xn); free(xbar); free(aty); free(axb); free(xr); free(yr);
    free(yn); free(dxv); free(adx); free(xp); free(yp); free(xa); free(ya);
    return rc;
}

/* ------------------------------------------------------ fix-and-propagate */
/*
 * Section 2.3.  Integer variables are fixed one at a time to an integer of
 * their current domain, each fixing followed by propagation of the rows that
 * contain the variable.  A row whose derived bounds would empty a domain (or
 * whose activity bounds already exclude b) is ignored for the rest of the
 * call and contributes nothing.  Variables left unfixed take the reference
 * value projected onto their domain.  The result is integral on I and inside
 * [l, u], not necessarily row-feasible.
 *
 * Readings: order = ascending distance to the nearest integer, ties by index;
 * value = reference rounded half down, clamped to the domain; integer bounds
 * derived by propagation are rounded inward with 1e-9 slack; a continuous
 * bound is applied only if it moves by more than 1e-9 (1 + |bound|).
 *
 * info[0] = 1 if every row holds at x_hat within 1e-6 (1 + |b_i|)
 * info[1] = number of ignored rows
 */
typedef struct {
    const orc_lp *lp;
    const uint8_t *is_int;
    double *L, *U;
    int32_t *col_ptr, *col_row; /* incidence: rows of each column */
    uint8_t *ignored, *queued;
    int32_t *queue;
    int64_t qhead, qtail, qcap;
} fp_state;

static void fp_push(fp_state *st, int32_t i)
{
    if (st->ignored[i] || st->queued[i]) return;
    st->queued[i] = 1;
    st->queue[st->qtail % st->qcap] = i;
    st->qtail++;
}

static void fp_touch_col(fp_state *st, int32_t j)
{
    for (int32_t e = st->col_ptr[j]; e < st->col_ptr[j + 1]; ++e) fp_push(st, st->col_row[e]);
}

/* Activity bounds of row i over the current domains: finite part and number
 * of infinite contributions. */
static void row_activity(const fp_state *st, int32_t i, double *minf, int *mininf,
                         double *maxf, int *maxinf)
{
    const orc_lp *lp = st->lp;
    double mn = 0.0, mx = 0.0;
    int ni = 0, xi = 0;
    for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) {
        int32_t j = lp->col_idx[e];
        double a = lp->val[e];
        if (a == 0.0) continue;
        double lo = a > 0 ? st->L[j] : st->U[j];
        double hi = a > 0 ? st->U[j] : st->L[j];
        if (isinf(lo)) ni++; else mn += a * lo;
        if (isinf(hi)) xi++; else mx += a * hi;
    }
    *minf = mn; *mininf = ni; *maxf = mx; *maxinf = xi;
}

/* Domains that row i derives for its variables (newL / newU per nonzero,
 * integer bounds rounded inward), against the current domains; returns 1 if
 * the row must be ignored (its activity bounds exclude b, or a derived
 * domain is empty). */
static int fp_row_bounds(const fp_state *st, int32_t i, double *newL, double *newU)
{
    const orc_lp *lp = st->lp;
    char sn = lp->sense[i];
    double bi = lp->b[i];
    double mn, mx;
    int ni, xi;
    row_activity(st, i, &mn, &ni, &mx, &xi);
    const double feas_tol = 1e-9 * (1.0 + fabs(bi));
    if ((sn == 'G' || sn == 'E') && xi == 0 && mx < bi - feas_tol) return 1;
    if ((sn == 'L' || sn == 'E') && ni == 0 && mn > bi + feas_tol) return 1;
    int64_t len = lp->row_ptr[i + 1] - lp->row_ptr[i];
    for (int64_t q = 0; q < len; ++q) {
        int64_t e = lp->row_ptr[i] + q;
        int32_t j = lp->col_idx[e];
        double a = lp->val[e];
        double lo = st->L[j], hi = st->U[j];
        newL[q] = lo;
        newU[q] = hi;
        if (a == 0.0) continue;
        /* a x_j >= b - (max activity of the other terms)   (G / E rows) */
        if (sn == 'G' || sn == 'E') {
            double own = a > 0 ? hi : lo; /* the term's contribution to max */
            int own_inf = isinf(own) ? 1 : 0; /* isinf may return -1 for -inf */
            int others_inf = xi - own_inf;
            if (others_inf == 0) {
                double rest = mx - (own_inf ? 0.0 : a * own);
                double bnd = (bi - rest) / a;
                if (a > 0) newL[q] = fmax(newL[q], bnd);
                else newU[q] = fmin(newU[q], bnd);
            }
        }
        /* a x_j <= b - (min activity of the other terms)   (L / E rows) */
        if (sn == 'L' || sn == 'E') {
            double own = a > 0 ? lo : hi;
            int own_inf = isinf(own) ? 1 : 0; /* isinf may return -1 for -inf */
            int others_inf = ni - own_inf;
            if (others_inf == 0) {
                double rest = mn - (own_inf ? 0.0 : a * own);
                double bnd = (bi - rest) / a;
                if (a > 0) newU[q] = fmin(newU[q], bnd);
                else newL[q] = fmax(newL[q], bnd);
            }
        }
        if (st->is_int[j]) {
            if (newL[q] > lo) newL[q] = ceil(newL[q] - 1e-9);
            if (newU[q] < hi) newU[q] = floor(newU[q] + 1e-9);
        }
        if (newL[q] > newU[q] + 1e-9 * (1.0 + fabs(newU[q]))) return 1;
    }
    return 0;
}

/* Propagate one row; returns 0 if fine, 1 if the row must be ignored. */
static int fp_row(fp_state *st, int32_t i, int32_t *changed, int32_t *nchanged,
                  double *newL, double *newU)
{
    const orc_lp *lp = st->lp;
    if (fp_row_bounds(st, i, newL, newU)) return 1;
    *nchanged = 0;
    int64_t len = lp->row_ptr[i + 1] - lp->row_ptr[i];
    for (int64_t q = 0; q < len; ++q) {
        int64_t e = lp->row_ptr[i] + q;
        int32_t j = lp->col_idx[e];
        int ch = 0;
        double lo = st->L[j], hi = st->U[j];
        double nl = newL[q], nu = newU[q];
        if (nl > nu) nl = nu; /* within tolerance: collapse */
        if (st->is_int[j]) {
            if (nl > lo) { st->L[j] = nl; ch = 1; }
            if (nu < hi) { st->U[j] = nu; ch = 1; }
        } else {
            if (nl > lo + 1e-9 * (1.0 + fabs(lo)) || (isinf(lo) && isfinite(nl))) { st->L[j] = nl; ch = 1; }
            if (nu < hi - 1e-9 * (1.0 + fabs(hi)) || (isinf(hi) && isfinite(nu))) { st->U[j] = nu; ch = 1; }
        }
        if (ch) changed[(*nchanged)++] = j;
    }
    return 0;
}

static void fp_propagate(fp_state *st, int32_t *changed, double *newL, double *newU)
{
    while (st->qhead < st->qtail) {
        int32_t i = st->queue[st->qhead % st->qcap];
        st->qhead++;
        st->queued[i] = 0;
        if (st->ignored[i]) continue;
        int32_t nch = 0;
        if (fp_row(st, i, changed, &nch, newL, newU)) {
            st->ignored[i] = 1;
            continue;
        }
        for (int32_t q = 0; q < nch; ++q) fp_touch_col(st, changed[q]);
    }
}

/* Integers take their (fixed) lower bound, continuous variables the
 * reference value projected onto their domain; info[0] = 1 if every row holds
 * at x_hat within 1e-6 (1 + |b_i|), info[1] = number of ignored rows. */
static void fp_finish(const orc_lp *lp, const uint8_t *is_int, const double *xbar, const double *L,
                      const double *U, const uint8_t *ignored, double *xhat, int32_t *info)
{
    const int32_t m = lp->m, n = lp->n;
    for (int32_t j = 0; j < n; ++j) {
        if (is_int[j]) xhat[j] = L[j];
        else xhat[j] = clampd(xbar[j], L[j], U[j]);
    }
    int ok = 1;
    int32_t nign = 0;
    for (int32_t i = 0; i < m; ++i) {
        nign += ignored[i];
        double a = 0.0;
        for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) a += lp->val[e] * xhat[lp->col_idx[e]];
        double tol = 1e-6 * (1.0 + fabs(lp->b[i]));
        char sn = lp->sense[i];
        if ((sn == 'G' || sn == 'E') && a < lp->b[i] - tol) ok = 0;
        if ((sn == 'L' || sn == 'E') && a > lp->b[i] + tol) ok = 0;
    }
    info[0] = ok;
    info[1] = nign;
}

static double frac_dist(double v)
{
    double f = v - floor(v);
    return f < 1.0 - f ? f : 1.0 - f;
}

static const double *g_sort_key;
static int cmp_frac(const void *a, const void *b)
{
    int32_t ia = *(const int32_t *)a, ib = *(const int32_t *)b;
    double fa = g_sort_key[ia], fb = g_sort_key[ib];
    if (fa < fb) return -1;
    if (fa > fb) return 1;
    return ia < ib ? -1 : (ia > ib);
}

int orc_fix_propagate(const orc_lp *lp, const uint8_t *is_int, const double *xbar,
                      double *xhat, int32_t *info)
{
    const int32_t m = lp->m, n = lp->n;
    const int64_t nnz = lp->row_ptr[m];
    fp_state st;
    memset(&st, 0, sizeof(st));
    st.lp = lp;
    st.is_int = is_int;
    st.L = malloc(sizeof(double) * (n + 1));
    st.U = malloc(sizeof(double) * (n + 1));
    st.col_ptr = calloc((size_t)n + 1, sizeof(int32_t));
    st.col_row = malloc(sizeof(int32_t) * (nnz + 1));
    st.ignored = calloc((size_t)m + 1, 1);
    st.queued = calloc((size_t)m + 1, 1);
    st.qcap = (int64_t)m + 1;
    st.queue = malloc(sizeof(int32_t) * st.qcap);
    int64_t maxlen = 1;
    for (int32_t i = 0; i < m; ++i) {
        int64_t len = lp->row_ptr[i + 1] - lp->row_ptr[i];
        if (len > maxlen) maxlen = len;
    }
    int32_t *changed = malloc(sizeof(int32_t) * maxlen);
    double *newL = malloc(sizeof(double) * maxlen);
    double *newU = malloc(sizeof(double) * maxlen);
    int32_t *order = malloc(sizeof(int32_t) * (n + 1));
    double *key = malloc(sizeof(double) * (n + 1));
    int32_t *fill = malloc(sizeof(int32_t) * (n + 1));
    if (!st.L || !st.U || !st.col_ptr || !st.col_row || !st.ignored || !st.queued || !st.queue ||
        !changed || !newL || !newU || !order || !key || !fill)
        return -1;
    /* row incidence of each column */
    for (int64_t e = 0; e < nnz; ++e) st.col_ptr[lp->col_idx[e] + 1]++;
    for (int32_t j = 0; j < n; ++j) st.col_ptr[j + 1] += st.col_ptr[j];
    for (int32_t j = 0; j < n; ++j) fill[j] = st.col_ptr[j];
    for (int32_t i = 0; i < m; ++i)
        for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
            st.col_row[fill[lp->col_idx[e]]++] = i;
    /* domains */
    int32_t nint = 0;
    for (int32_t j = 0; j < n; ++j) {
        st.L[j] = lp->l[j];
        st.U[j] = lp->u[j];
        if (is_int[j]) {
            if (isfinite(st.L[j])) st.L[j] = ceil(st.L[j] - 1e-9);
            if (isfinite(st.U[j])) st.U[j] = floor(st.U[j] + 1e-9);
            order[nint++] = j;
            key[j] = frac_dist(xbar[j]);
        }
    }
    g_sort_key = key;
    qsort(order, (size_t)nint, sizeof(int32_t), cmp_frac);
    for (int32_t q = 0; q < nint; ++q) {
        int32_t j = order[q];
        if (st.L[j] == st.U[j]) continue; /* fixed by an earlier propagation */
        double v = ceil(xbar[j] - 0.5);   /* round half down */
        v = clampd(v, st.L[j], st.U[j]);
        st.L[j] = st.U[j] = v;
        fp_touch_col(&st, j);
        fp_propagate(&st, changed, newL, newU);
    }
    fp_finish(lp, is_int, xbar, st.L, st.U, st.ignored, xhat, info);
    free(st.L); free(st.U); free(st.col_ptr); free(st.col_row); free(st.ignored);
    free(st.queued); free(st.queue); free(changed); free(newL); free(newU);
    free(order); free(key); free(fill);
    return 0;
}

/* ---------------------------------------------- batched fix-and-propagate */
/*
 * A parallel form of the procedure above (Section 2.3), for a device that
 * evaluates many rows at once; it is not the paper's order of work.  The
 * next K unfixed integer variables of the same fixing order are fixed
 * together, each to its rounded reference value clamped to its domain, and
 * propagation then runs in synchronous rounds.  In a round every active row
 * is evaluated against the domains at the start of the round, with the
 * activity bounds, derived bounds, integer rounding and emptiness tests of
 * the sequential procedure; a row failing them is ignored for the rest of
 * the call.  Per variable, the derived bounds of the surviving rows that
 * would change it (integer: any tightening; continuous: by more than
 * 1e-9 (1 + |bound|), or from infinite to finite) are combined by max (lower)
 * and min (upper).  Where the combined domain of a variable is empty by more
 * than 1e-9 (1 + |upper|), every row that would change that variable is
 * ignored and the combination is taken again without them (dropping rows
 * only widens the combined domains, so once is enough); a crossing within
 * that tolerance sets both bounds to max(upper, old lower).  The variables
 * whose domain changed make their non-ignored rows active for the next
 * round.  A batch ends when no row is active or after max_rounds rounds.
 * With K = 1, exact arithmetic and no ignored row, both procedures end with
 * the same domains: the greatest common fixpoint of the row propagators,
 * whatever the order in which the rows are evaluated.
 */
static int fpb_lower_changes(int is_int, double lo, double nl)
{
    if (is_int) return nl > lo;
    return nl > lo + 1e-9 * (1.0 + fabs(lo)) || (isinf(lo) && isfinite(nl));
}

static int fpb_upper_changes(int is_int, double hi, double nu)
{
    if (is_int) return nu < hi;
    return nu < hi - 1e-9 * (1.0 + fabs(hi)) || (isinf(hi) && isfinite(nu));
}

/* Folds the derived bounds of row i into the combined domains NL / NU
 * (touched variables are listed once per round in `touched`). */
static void fpb_fold_row(const fp_state *st, int32_t i, const double *cl, const double *cu,
                         double *NL, double *NU, int32_t *vmark, int32_t stamp, int32_t *touched,
                         int32_t *ntouched)
{
    const orc_lp *lp = st->lp;
    for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) {
        const int32_t j = lp->col_idx[e];
        const double nl = cl[e], nu = cu[e];
        const int tl = fpb_lower_changes(st->is_int[j], st->L[j], nl);
        const int tu = fpb_upper_changes(st->is_int[j], st->U[j], nu);
        if (!tl && !tu) continue;
        if (vmark[j] != stamp) {
            vmark[j] = stamp;
            touched[(*ntouched)++] = j;
        }
        if (tl && nl > NL[j]) NL[j] = nl;
        if (tu && nu < NU[j]) NU[j] = nu;
    }
}

/* ignored_out: [m] or NULL, receives 1 for every ignored row. */
int orc_fix_propagate_batched(const orc_lp *lp, const uint8_t *is_int, const double *xbar, int32_t K,
                              int32_t max_rounds, double *xhat, int32_t *info, uint8_t *ignored_out)
{
    const int32_t m = lp->m, n = lp->n;
    const int64_t nnz = lp->row_ptr[m];
    if (K < 1 || max_rounds < 1) return -1;
    fp_state st;
    memset(&st, 0, sizeof(st));
    st.lp = lp;
    st.is_int = is_int;
    st.L = malloc(sizeof(double) * (n + 1));
    st.U = malloc(sizeof(double) * (n + 1));
    st.col_ptr = calloc((size_t)n + 1, sizeof(int32_t));
    st.col_row = malloc(sizeof(int32_t) * (nnz + 1));
    st.ignored = calloc((size_t)m + 1, 1);
    double *NL = malloc(sizeof(double) * (n + 1)), *NU = malloc(sizeof(double) * (n + 1));
    double *cl = malloc(sizeof(double) * (nnz + 1)), *cu = malloc(sizeof(double) * (nnz + 1));
    int32_t *active = malloc(sizeof(int32_t) * (m + 1)), *next = malloc(sizeof(int32_t) * (m + 1));
    int32_t *rmark = malloc(sizeof(int32_t) * (m + 1));
    uint8_t *bad = calloc((size_t)m + 1, 1);
    int32_t *vmark = malloc(sizeof(int32_t) * (n + 1)), *touched = malloc(sizeof(int32_t) * (n + 1));
    int32_t *order = malloc(sizeof(int32_t) * (n + 1)), *fill = malloc(sizeof(int32_t) * (n + 1));
    double *key = malloc(sizeof(double) * (n + 1));
    if (!st.L || !st.U || !st.col_ptr || !st.col_row || !st.ignored || !NL || !NU || !cl || !cu ||
        !active || !next || !rmark || !bad || !vmark || !touched || !order || !fill || !key)
        return -1;
    for (int64_t e = 0; e < nnz; ++e) st.col_ptr[lp->col_idx[e] + 1]++;
    for (int32_t j = 0; j < n; ++j) st.col_ptr[j + 1] += st.col_ptr[j];
    for (int32_t j = 0; j < n; ++j) fill[j] = st.col_ptr[j];
    for (int32_t i = 0; i < m; ++i)
        for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e)
            st.col_row[fill[lp->col_idx[e]]++] = i;
    int32_t nint = 0;
    for (int32_t j = 0; j < n; ++j) {
        st.L[j] = lp->l[j];
        st.U[j] = lp->u[j];
        if (is_int[j]) {
            if (isfinite(st.L[j])) st.L[j] = ceil(st.L[j] - 1e-9);
            if (isfinite(st.U[j])) st.U[j] = floor(st.U[j] + 1e-9);
            order[nint++] = j;
            key[j] = frac_dist(xbar[j]);
        }
        NL[j] = st.L[j];
        NU[j] = st.U[j];
        vmark[j] = -1;
    }
    for (int32_t i = 0; i < m; ++i) rmark[i] = -1;
    g_sort_key = key;
    qsort(order, (size_t)nint, sizeof(int32_t), cmp_frac);
    int32_t stamp = 0;
    int32_t p = 0;
    while (p < nint) {
        /* the batch: the next K variables of the order that are not fixed */
        int32_t nsel = 0;
        ++stamp;
        int32_t nact = 0;
        while (nsel < K && p < nint) {
            const int32_t j = order[p++];
            if (st.L[j] == st.U[j]) continue;
            const double v = clampd(ceil(xbar[j] - 0.5), st.L[j], st.U[j]);
            st.L[j] = st.U[j] = NL[j] = NU[j] = v;
            ++nsel;
            for (int32_t e = st.col_ptr[j]; e < st.col_ptr[j + 1]; ++e) {
                const int32_t i = st.col_row[e];
                if (!st.ignored[i] && rmark[i] != stamp) {
                    rmark[i] = stamp;
                    active[nact++] = i;
                }
            }
        }
        for (int32_t round = 0; round < max_rounds && nact > 0; ++round) {
            /* every active row against the domains at the start of the round */
            for (int32_t a = 0; a < nact; ++a) {
                const int32_t i = active[a];
                const int64_t e0 = lp->row_ptr[i];
                if (fp_row_bounds(&st, i, cl + e0, cu + e0)) st.ignored[i] = 1;
            }
            ++stamp;
            int32_t ntouched = 0;
            for (int32_t a = 0; a < nact; ++a)
                if (!st.ignored[active[a]])
                    fpb_fold_row(&st, active[a], cl, cu, NL, NU, vmark, stamp, touched, &ntouched);
            /* rows that would change a variable whose combined domain is empty */
            int conflict = 0;
            for (int32_t a = 0; a < nact; ++a) {
                const int32_t i = active[a];
                if (st.ignored[i]) continue;
                for (int64_t e = lp->row_ptr[i]; e < lp->row_ptr[i + 1]; ++e) {
                    const int32_t j = lp->col_idx[e];
                    if (!(NL[j] > NU[j] + 1e-9 * (1.0 + fabs(NU[j])))) continue;
                    if (fpb_lower_changes(is_int[j], st.L[j], cl[e]) ||
                        fpb_upper_changes(is_int[j], st.U[j], cu[e])) {
                        bad[i] = 1;
                        conflict = 1;
                    }
                }
            }
            if (conflict) {
                for (int32_t a = 0; a < nact; ++a)
                    if (bad[active[a]]) {
                        bad[active[a]] = 0;
                        st.ignored[active[a]] = 1;
                    }
                for (int32_t t = 0; t < ntouched; ++t) {
                    NL[touched[t]] = st.L[touched[t]];
                    NU[touched[t]] = st.U[touched[t]];
                }
                ++stamp;
                ntouched = 0;
                for (int32_t a = 0; a < nact; ++a)
                    if (!st.ignored[active[a]])
                        fpb_fold_row(&st, active[a], cl, cu, NL, NU, vmark, stamp, touched, &ntouched);
            }
            /* new domains; their rows are the next round's active rows */
            ++stamp;
            int32_t nnext = 0;
            for (int32_t t = 0; t < ntouched; ++t) {
                const int32_t j = touched[t];
                double nl = NL[j], nu = NU[j];
                if (nl > nu) nl = nu = fmax(nu, st.L[j]);
                const int ch = nl != st.L[j] || nu != st.U[j];
                st.L[j] = NL[j] = nl;
                st.U[j] = NU[j] = nu;
                if (!ch) continue;
                for (int32_t e = st.col_ptr[j]; e < st.col_ptr[j + 1]; ++e) {
                    const int32_t i = st.col_row[e];
                    if (!st.ignored[i] && rmark[i] != stamp) {
                        rmark[i] = stamp;
                        next[nnext++] = i;
                    }
                }
            }
            int32_t *sw = active;
            active = next;
            next = sw;
            nact = nnext;
        }
    }
    fp_finish(lp, is_int, xbar, st.L, st.U, st.ignored, xhat, info);
    if (ignored_out) memcpy(ignored_out, st.ignored, (size_t)m);
    free(st.L); free(st.U); free(st.col_ptr); free(st.col_row); free(st.ignored);
    free(NL); free(NU); free(cl); free(cu); free(active); free(next); free(rmark); free(bad);
    free(vmark); free(touched); free(order); free(fill); free(key);
    return 0;
}
