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

class Rounder {
public:
    Rounder(const FPProblem &P, const uint8_t *is_int) : P_(P), is_int_(is_int)
    {
        L_.assign(P.l, P.l + P.n);
        U_.assign(P.u, P.u + P.n);
        bool all_int = true;
        for (int32_t j = 0; j < P.n; ++j)
            if (is_int_[j]) {
                if (isfinite(L_[j])) L_[j] = ceil(L_[j] - kIntSlack);
                if (isfinite(U_[j])) U_[j] = floor(U_[j] + kIntSlack);
            } else {
                all_int = false;
            }
        ignored_.assign(P.m, 0);
        in_queue_.assign(P.m, 0);
        size_t maxlen = 1;
        for (int32_t i = 0; i < P.m; ++i) maxlen = std::max<size_t>(maxlen, P.ptr[i + 1] - P.ptr[i]);
        lo_new_.resize(maxlen);
        hi_new_.resize(maxlen);
        // Fast path: with integer variables, integer coefficients and integer
        // bounds every activity is an exact sum in double precision, so row
        // activities can be kept up to date incrementally (equal to a
        // recomputation bit for bit), and a row whose slack exceeds
        // max_j |a_ij| (u_j - l_j) can tighten nothing and is skipped.
        exact_ = all_int;
        for (int32_t e = P.ptr[0]; e < P.ptr[P.m] && exact_; ++e) {
            const double c = P.val[e];
            exact_ = c == floor(c) && fabs(c) < 1e6;
        }
        for (int32_t j = 0; j < P.n && exact_; ++j)
            exact_ = (!isfinite(L_[j]) || fabs(L_[j]) < 1e6) && (!isfinite(U_[j]) || fabs(U_[j]) < 1e6);
        if (exact_) {
            act_.resize(P.m);
            reach_.assign(P.m, 0.0);
            for (int32_t i = 0; i < P.m; ++i) {
                act_[i] = activity(i);
                for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) {
                    const int32_t j = P.col[e];
                    const double r = fabs(P.val[e]) * (U_[j] - L_[j]);
                    reach_[i] = std::max(reach_[i], isnan(r) ? INFINITY : r);
                }
            }
        }
    }

    void run(const double *xref, double *xhat)
    {
        std::vector<int32_t> ints;
        std::vector<double> dist(P_.n, 0.0);
        for (int32_t j = 0; j < P_.n; ++j)
            if (is_int_[j]) {
                ints.push_back(j);
                const double f = xref[j] - floor(xref[j]);
                dist[j] = std::min(f, 1.0 - f);
            }
        std::stable_sort(ints.begin(), ints.end(), [&](int32_t a, int32_t b) {
            return dist[a] < dist[b] || (dist[a] == dist[b] && a < b);
        });
        for (int32_t j : ints) {
            if (L_[j] == U_[j]) continue;
            double v = ceil(xref[j] - 0.5);  // round half down
            v = std::min(std::max(v, L_[j]), U_[j]);
            set_bounds(j, v, v);
            enqueue_rows_of(j);
            drain();
        }
        for (int32_t j = 0; j < P_.n; ++j)
            xhat[j] = is_int_[j] ? L_[j] : std::min(std::max(xref[j], L_[j]), U_[j]);
    }

    int32_t ignored_rows() const { return (int32_t)std::count(ignored_.begin(), ignored_.end(), (uint8_t)1); }

private:
    // Contribution of a_ij x_j to the min / max activity of a row.
    static void contrib(double c, double lo, double hi, double &mn, double &mx, int &mn_inf, int &mx_inf)
    {
        const double at_min = c > 0 ? lo : hi, at_max = c > 0 ? hi : lo;
        mn_inf = isinf(at_min) ? 1 : 0;
        mx_inf = isinf(at_max) ? 1 : 0;
        mn = mn_inf ? 0.0 : c * at_min;
        mx = mx_inf ? 0.0 : c * at_max;
    }

    // New bounds of x_j; keeps the row activities current on the fast path.
    void set_bounds(int32_t j, double lo, double hi)
    {
        if (exact_) {
            for (int32_t e = P_.cptr[j]; e < P_.cptr[j + 1]; ++e) {
                const int32_t i = P_.crow[e];
                const double c = P_.cval[e];
                if (c == 0.0) continue;
                double mn0, mx0, mn1, mx1;
                int a0, b0, a1, b1;
                contrib(c, L_[j], U_[j], mn0, mx0, a0, b0);
                contrib(c, lo, hi, mn1, mx1, a1, b1);
                Activity &A = act_[i];
                A.lo += mn1 - mn0;
                A.hi += mx1 - mx0;
                A.lo_inf += a1 - a0;
                A.hi_inf += b1 - b0;
            }
        }
        L_[j] = lo;
        U_[j] = hi;
    }

    // Fast path: true when row i can neither tighten a bound nor be ignored.
    bool idle(int32_t i) const
    {
        const Activity &A = act_[i];
        const char s = P_.sense[i];
        const double b = P_.b[i];
        const double margin = 1e-9 * (1.0 + fabs(b) + reach_[i]);
        if (s == 'G' || s == 'E') {
            if (A.hi_inf != 0 || !(A.hi - b >= reach_[i] + margin)) return false;
        }
        if (s == 'L' || s == 'E') {
            if (A.lo_inf != 0 || !(b - A.lo >= reach_[i] + margin)) return false;
        }
        return true;
    }

    void enqueue_rows_of(int32_t j)
    {
        for (int32_t e = P_.cptr[j]; e < P_.cptr[j + 1]; ++e) {
            const int32_t i = P_.crow[e];
            if (!ignored_[i] && !in_queue_[i]) {
                in_queue_[i] = 1;
                queue_.push_back(i);
            }
        }
    }

    void drain()
    {
        while (head_ < queue_.size()) {
            const int32_t i = queue_[head_++];
            in_queue_[i] = 0;
            if (ignored_[i]) continue;
            changed_.clear();
            if (!propagate_row(i)) {
                ignored_[i] = 1;
                continue;
            }
            for (int32_t j : changed_) enqueue_rows_of(j);
        }
        queue_.clear();
        head_ = 0;
    }

    Activity activity(int32_t i) const
    {
        Activity a;
        for (int32_t e = P_.ptr[i]; e < P_.ptr[i + 1]; ++e) {
            const double c = P_.val[e];
            if (c == 0.0) continue;
            const int32_t j = P_.col[e];
            const double at_min = c > 0 ? L_[j] : U_[j];
            const double at_max = c > 0 ? U_[j] : L_[j];
            if (isinf(at_min)) a.lo_inf++;
            else a.lo += c * at_min;
            if (isinf(at_max)) a.hi_inf++;
            else a.hi += c * at_max;
        }
        return a;
    }

    // Returns false if row i must be ignored; otherwise applies its bounds.
    bool propagate_row(int32_t i)
    {
        if (exact_ && idle(i)) return true;
        const char s = P_.sense[i];
        const double b = P_.b[i];
        const bool ge = s == 'G' || s == 'E', le = s == 'L' || s == 'E';
        const Activity act = exact_ ? act_[i] : activity(i);
        const double tol = kIntSlack * (1.0 + fabs(b));
        if (ge && act.hi_inf == 0 && act.hi < b - tol) return false;
        if (le && act.lo_inf == 0 && act.lo > b + tol) return false;
        const int32_t e0 = P_.ptr[i], len = P_.ptr[i + 1] - e0;
        for (int32_t q = 0; q < len; ++q) {
            const int32_t j = P_.col[e0 + q];
            const double c = P_.val[e0 + q];
            double lo = L_[j], hi = U_[j];
            if (c != 0.0) {
                if (ge) {  // c x_j >= b - (max activity of the other terms)
                    const double mine = c > 0 ? U_[j] : L_[j];
                    const bool mine_inf = isinf(mine);
                    if (act.hi_inf - (mine_inf ? 1 : 0) == 0) {
                        const double rest = act.hi - (mine_inf ? 0.0 : c * mine);
                        const double bound = (b - rest) / c;
                        if (c > 0) lo = std::max(lo, bound);
                        else hi = std::min(hi, bound);
                    }
                }
                if (le) {  // c x_j <= b - (min activity of the other terms)
                    const double mine = c > 0 ? L_[j] : U_[j];
                    const bool mine_inf = isinf(mine);
                    if (act.lo_inf - (mine_inf ? 1 : 0) == 0) {
                        const double rest = act.lo - (mine_inf ? 0.0 : c * mine);
                        const double bound = (b - rest) / c;
                        if (c > 0) hi = std::min(hi, bound);
                        else lo = std::max(lo, bound);
                    }
                }
                if (is_int_[j]) {
                    if (lo > L_[j]) lo = ceil(lo - kIntSlack);
                    if (hi < U_[j]) hi = floor(hi + kIntSlack);
                }
                if (lo > hi + kIntSlack * (1.0 + fabs(hi))) return false;  // would empty the domain
            }
            lo_new_[q] = lo;
            hi_new_[q] = hi;
        }
        for (int32_t q = 0; q < len; ++q) {
            const int32_t j = P_.col[e0 + q];
            double lo = lo_new_[q], hi = hi_new_[q];
            if (lo > hi) lo = hi;
            bool moved = false;
            double nl = L_[j], nu = U_[j];
            if (is_int_[j]) {
                if (lo > nl) { nl = lo; moved = true; }
                if (hi < nu) { nu = hi; moved = true; }
            } else {
                const double l0 = L_[j], u0 = U_[j];
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
    bool exact_ = false;
    std::vector<Activity> act_;   // fast path: current row activities
    std::vector<double> reach_;   // fast path: max_j |a_ij| (u_j - l_j) at the start
    std::vector<double> L_, U_, lo_new_, hi_new_;
    std::vector<uint8_t> ignored_, in_queue_;
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
        if ((s == 'G' || s == 'E') && a < P.b[i] - t) return false;
        if ((s == 'L' || s == 'E') && a > P.b[i] + t) return false;
    }
    return true;
}

void fix_and_propagate(const FPProblem &P, const uint8_t *is_int, const double *xref, double *xhat,
                       int32_t *feasible, int32_t *ignored)
{
    Rounder r(P, is_int);
    r.run(xref, xhat);
    *feasible = rows_satisfied(P, xhat, kFeasTol) ? 1 : 0;
    *ignored = r.ignored_rows();
}

}  // namespace scy
