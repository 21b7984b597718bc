// Host fix-and-propagate rounding (Section 2.3) used by the pump loop.
//
// Integer variables are fixed one at a time, in order of increasing
// distance of the reference value to the nearest integer (ties by index), to
// the reference rounded half down and clamped to the current domain; every
// fixing is followed by activity-based bound propagation over the rows that
// contain the fixed variable, processed first-in first-out.  A row whose
// activity bounds already exclude its right-hand side, or whose derived
// bounds would empty a domain, is ignored for the rest of the call and
// changes nothing.  Remaining continuous variables take the reference value
// projected onto their (tightened) domain.  The result is integral on the
// integer variables and inside [l, u] (Section 2.3), not necessarily
// row-feasible.  Exact logic: with integer data every activity is an exact
// sum in double precision.
#include <cmath>
#include <math.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "fixprop.h"

namespace scy {

namespace {

constexpr double kIntSlack = 1e-9;   // slack when rounding derived integer bounds
constexpr double kContMove = 1e-9;   // relative move that counts as a tightening
constexpr double kFeasTol = 1e-6;    // row check of the final point

struct Activity {
    double lo = 0.0, hi = 0.0;  // finite parts of min / max activity
    int lo_inf = 0, hi_inf = 0; // number of infinite contributions
};

// Contribution of a_ij x_j to the min / max activity of a row.
inline void contrib(double c, double lo, double hi, double &mn, double &mx, int &mn_inf, int &mx_inf)
{
    const double at_min = c > 0 ? lo : hi, at_max = c > 0 ? hi : lo;
    mn_inf = isinf(at_min) ? 1 : 0;
    mx_inf = isinf(at_max) ? 1 : 0;
    mn = mn_inf ? 0.0 : c * at_min;
    mx = mx_inf ? 0.0 : c * at_max;
}

Activity activity(const FPProblem &P, const FPDomain *D, int32_t i)
{
    Activity a;
    for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) {
        const double c = P.val[e];
        if (c == 0.0) continue;
        const FPDomain &d = D[P.col[e]];
        const double at_min = c > 0 ? d.L : d.U;
        const double at_max = c > 0 ? d.U : d.L;
        if (isinf(at_min)) a.lo_inf++;
        else a.lo += c * at_min;
        if (isinf(at_max)) a.hi_inf++;
        else a.hi += c * at_max;
    }
    return a;
}

// |a_ij| (U_j - L_j) with an undefined product (0 * inf) taken as infinite.
inline double reach_of(double c, const FPDomain &d)
{
    const double r = fabs(c) * (d.U - d.L);
    return isnan(r) ? INFINITY : r;
}

class Rounder {
public:
    Rounder(const FPProblem &P, const uint8_t *is_int, const FPPrep &prep)
        : P_(P), is_int_(is_int), exact_(prep.exact), row_(prep.rows), dom_(prep.dom)
    {
        lo_new_.resize(prep.maxlen);
        hi_new_.resize(prep.maxlen);
    }

    void run(const double *xref, double *xhat)
    {
        // integer variables by distance to the nearest integer, ties by
        // index: the integral ones first (already in index order), then the
        // others sorted by (distance, index)
        std::vector<std::pair<double, int32_t>> order, frac;
        order.reserve(P_.n);
        for (int32_t j = 0; j < P_.n; ++j)
            if (is_int_[j]) {
                const double f = xref[j] - floor(xref[j]);
                const double d = std::min(f, 1.0 - f);
                if (d == 0.0) order.emplace_back(d, j);
                else frac.emplace_back(isnan(d) ? INFINITY : d, j);
            }
        std::sort(frac.begin(), frac.end());
        order.insert(order.end(), frac.begin(), frac.end());
        for (const auto &o : order) {
            const int32_t j = o.second;
            if (dom_[j].L == dom_[j].U) continue;
            double v = ceil(xref[j] - 0.5);  // round half down
            // clamp to the domain (a NaN reference takes the lower bound)
            if (!(v >= dom_[j].L)) v = dom_[j].L;
            if (!(v <= dom_[j].U)) v = dom_[j].U;
            set_bounds(j, v, v);
            enqueue_rows_of(j);
            drain();
        }
        for (int32_t j = 0; j < P_.n; ++j)
            xhat[j] = is_int_[j] ? dom_[j].L : std::min(std::max(xref[j], dom_[j].L), dom_[j].U);
    }

    int32_t ignored_rows() const
    {
        int32_t k = 0;
        for (const FPRow &r : row_) k += r.ignored;
        return k;
    }

private:
    // New bounds of x_j; keeps the row activities current in exact mode.
    void set_bounds(int32_t j, double lo, double hi)
    {
        FPDomain &d = dom_[j];
        if (exact_) {
            for (int32_t e = P_.cptr[j]; e < P_.cptr[j + 1]; ++e) {
                const double c = P_.cval[e];
                if (c == 0.0) continue;
                double mn0, mx0, mn1, mx1;
                int a0, b0, a1, b1;
                contrib(c, d.L, d.U, mn0, mx0, a0, b0);
                contrib(c, lo, hi, mn1, mx1, a1, b1);
                FPRow &R = row_[P_.crow[e]];
                R.lo += mn1 - mn0;
                R.hi += mx1 - mx0;
                R.lo_inf += a1 - a0;
                R.hi_inf += b1 - b0;
            }
        }
        d.L = lo;
        d.U = hi;
    }

    // Exact mode: true when the row can neither tighten a bound nor be
    // ignored.  All activities are exact integers, so a slack of at least
    // the reach on the row's side proves that every derived bound lies
    // outside the current domain; the margin covers the one rounding of
    // the slack itself.
    static bool idle(const FPRow &R)
    {
        const double margin = 1e-9 * (1.0 + fabs(R.b) + R.reach);
        if (R.sense == 'G' || R.sense == 'E') {
            if (R.hi_inf != 0 || !(R.hi - R.b >= R.reach + margin)) return false;
        }
        if (R.sense == 'L' || R.sense == 'E') {
            if (R.lo_inf != 0 || !(R.b - R.lo >= R.reach + margin)) return false;
        }
        return true;
    }

    void enqueue_rows_of(int32_t j)
    {
        for (int32_t e = P_.cptr[j]; e < P_.cptr[j + 1]; ++e) {
            const int32_t i = P_.crow[e];
            FPRow &R = row_[i];
            if (!R.ignored && !R.queued) {
                R.queued = 1;
                queue_.push_back(i);
            }
        }
    }

    void drain()
    {
        while (head_ < queue_.size()) {
            const int32_t i = queue_[head_++];
            FPRow &R = row_[i];
            R.queued = 0;
            if (R.ignored) continue;
            changed_.clear();
            if (!propagate_row(i, R)) {
                R.ignored = 1;
                continue;
            }
            for (int32_t j : changed_) enqueue_rows_of(j);
        }
        queue_.clear();
        head_ = 0;
    }

    // Returns false if row i must be ignored; otherwise applies its bounds.
    bool propagate_row(int32_t i, FPRow &R)
    {
        if (exact_ && idle(R)) return true;
        const char s = R.sense;
        const double b = R.b;
        const bool ge = s == 'G' || s == 'E', le = s == 'L' || s == 'E';
        Activity act;
        if (exact_) {
            act.lo = R.lo;
            act.hi = R.hi;
            act.lo_inf = R.lo_inf;
            act.hi_inf = R.hi_inf;
        } else {
            act = activity(P_, dom_.data(), i);
        }
        const double tol = kIntSlack * (1.0 + fabs(b));
        if (ge && act.hi_inf == 0 && act.hi < b - tol) return false;
        if (le && act.lo_inf == 0 && act.lo > b + tol) return false;
        const int32_t e0 = P_.ptr[i], len = P_.ptr[i + 1] - e0;
        double reach_now = 0.0;
        for (int32_t q = 0; q < len; ++q) {
            const int32_t j = P_.col[e0 + q];
            const double c = P_.val[e0 + q];
            const FPDomain d = dom_[j];
            double lo = d.L, hi = d.U;
            if (exact_) reach_now = std::max(reach_now, reach_of(c, d));
            if (c != 0.0) {
                if (ge) {  // c x_j >= b - (max activity of the other terms)
                    const double mine = c > 0 ? d.U : d.L;
                    const bool mine_inf = isinf(mine);
                    if (act.hi_inf - (mine_inf ? 1 : 0) == 0) {
                        const double rest = act.hi - (mine_inf ? 0.0 : c * mine);
                        const double bound = (b - rest) / c;
                        if (c > 0) lo = std::max(lo, bound);
                        else hi = std::min(hi, bound);
                    }
                }
                if (le) {  // c x_j <= b - (min activity of the other terms)
                    const double mine = c > 0 ? d.L : d.U;
                    const bool mine_inf = isinf(mine);
                    if (act.lo_inf - (mine_inf ? 1 : 0) == 0) {
                        const double rest = act.lo - (mine_inf ? 0.0 : c * mine);
                        const double bound = (b - rest) / c;
                        if (c > 0) hi = std::min(hi, bound);
                        else lo = std::max(lo, bound);
                    }
                }
                if (is_int_[j]) {
                    if (lo > d.L) lo = ceil(lo - kIntSlack);
                    if (hi < d.U) hi = floor(hi + kIntSlack);
                }
                if (lo > hi + kIntSlack * (1.0 + fabs(hi))) return false;  // would empty the domain
            }
            lo_new_[q] = lo;
            hi_new_[q] = hi;
        }
        // domains only shrink, so the reach measured now bounds every later one
        if (exact_) R.reach = std::min(R.reach, reach_now);
        for (int32_t q = 0; q < len; ++q) {
            const int32_t j = P_.col[e0 + q];
            double lo = lo_new_[q], hi = hi_new_[q];
            if (lo > hi) lo = hi;
            bool moved = false;
            const FPDomain d = dom_[j];
            double nl = d.L, nu = d.U;
            if (is_int_[j]) {
                if (lo > nl) { nl = lo; moved = true; }
                if (hi < nu) { nu = hi; moved = true; }
            } else {
                const double l0 = d.L, u0 = d.U;
                if (lo > l0 + kContMove * (1.0 + fabs(l0)) || (isinf(l0) && isfinite(lo))) { nl = lo; moved = true; }
                if (hi < u0 - kContMove * (1.0 + fabs(u0)) || (isinf(u0) && isfinite(hi))) { nu = hi; moved = true; }
            }
            if (moved) {
                set_bounds(j, nl, nu);
                changed_.push_back(j);
            }
        }
        return true;
    }

    const FPProblem &P_;
    const uint8_t *is_int_;
    const bool exact_;
    std::vector<FPRow> row_;
    std::vector<FPDomain> dom_;
    std::vector<double> lo_new_, hi_new_;
    std::vector<int32_t> queue_, changed_;
    size_t head_ = 0;
};

}  // namespace

void build_incidence(FPProblem &P, std::vector<int32_t> &cptr, std::vector<int32_t> &crow,
                     std::vector<double> &cval)
{
    cptr.assign((size_t)P.n + 1, 0);
    for (int32_t e = P.ptr[0]; e < P.ptr[P.m]; ++e) cptr[P.col[e] + 1]++;
    for (int32_t j = 0; j < P.n; ++j) cptr[j + 1] += cptr[j];
    crow.resize(cptr[P.n]);
    cval.resize(cptr[P.n]);
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (int32_t i = 0; i < P.m; ++i)
        for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) {
            const int32_t k = fill[P.col[e]]++;
            crow[k] = i;
            cval[k] = P.val[e];
        }
    P.cptr = cptr.data();
    P.crow = crow.data();
    P.cval = cval.data();
}

bool rows_satisfied(const FPProblem &P, const double *x, double tol)
{
    for (int32_t i = 0; i < P.m; ++i) {
        double a = 0.0;
        for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) a += P.val[e] * x[P.col[e]];
        const double t = tol * (1.0 + fabs(P.b[i]));
        const char s = P.sense[i];
        if (!std::isfinite(a)) return false;  // a non-finite activity satisfies no row
        if ((s == 'G' || s == 'E') && a < P.b[i] - t) return false;
        if ((s == 'L' || s == 'E') && a > P.b[i] + t) return false;
    }
    return true;
}

void fp_prepare(const FPProblem &P, const uint8_t *is_int, FPPrep &prep)
{
    prep.dom.resize(P.n);
    bool all_int = true;
    for (int32_t j = 0; j < P.n; ++j) {
        double L = P.l[j], U = P.u[j];
        if (is_int[j]) {
            if (isfinite(L)) L = ceil(L - kIntSlack);
            if (isfinite(U)) U = floor(U + kIntSlack);
        } else {
            all_int = false;
        }
        prep.dom[j] = FPDomain{L, U};
    }
    prep.rows.assign(P.m, FPRow());
    prep.maxlen = 1;
    for (int32_t i = 0; i < P.m; ++i) {
        prep.rows[i].b = P.b[i];
        prep.rows[i].sense = P.sense[i];
        prep.maxlen = std::max(prep.maxlen, P.ptr[i + 1] - P.ptr[i]);
    }
    // Exact mode: with integer variables, integer coefficients and integer
    // bounds every activity is an exact sum in double precision, so row
    // activities can be kept up to date incrementally (equal to a
    // recomputation bit for bit), and a row whose slack exceeds
    // max_j |a_ij| (U_j - L_j) can tighten nothing and is skipped.
    bool exact = all_int;
    for (int32_t e = P.ptr[0]; e < P.ptr[P.m] && exact; ++e) {
        const double c = P.val[e];
        exact = c == floor(c) && fabs(c) < 1e6;
    }
    for (int32_t j = 0; j < P.n && exact; ++j) {
        const FPDomain &d = prep.dom[j];
        exact = (!isfinite(d.L) || fabs(d.L) < 1e6) && (!isfinite(d.U) || fabs(d.U) < 1e6);
    }
    prep.exact = exact;
    if (exact) {
        for (int32_t i = 0; i < P.m; ++i) {
            FPRow &R = prep.rows[i];
            const Activity a = activity(P, prep.dom.data(), i);
            R.lo = a.lo;
            R.hi = a.hi;
            R.lo_inf = a.lo_inf;
            R.hi_inf = a.hi_inf;
            for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e)
                R.reach = std::max(R.reach, reach_of(P.val[e], prep.dom[P.col[e]]));
        }
    }
    prep.ready = true;
}

void fix_and_propagate(const FPProblem &P, const uint8_t *is_int, const FPPrep &prep, const double *xref,
                       double *xhat, int32_t *feasible, int32_t *ignored)
{
    Rounder r(P, is_int, prep);
    r.run(xref, xhat);
    *feasible = rows_satisfied(P, xhat, kFeasTol) ? 1 : 0;
    *ignored = r.ignored_rows();
}

}  // namespace scy
