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
        for (int32_t j = 0; j < P.n; ++j)
            if (is_int_[j]) {
                if (isfinite(L_[j])) L_[j] = ceil(L_[j] - kIntSlack);
                if (isfinite(U_[j])) U_[j] = floor(U_[j] + kIntSlack);
            }
        ignored_.assign(P.m, 0);
        in_queue_.assign(P.m, 0);
        size_t maxlen = 1;
        for (int32_t i = 0; i < P.m; ++i) maxlen = std::max<size_t>(maxlen, P.ptr[i + 1] - P.ptr[i]);
        lo_new_.resize(maxlen);
        hi_new_.resize(maxlen);
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
            L_[j] = U_[j] = v;
            enqueue_rows_of(j);
            drain();
        }
        for (int32_t j = 0; j < P_.n; ++j)
            xhat[j] = is_int_[j] ? L_[j] : std::min(std::max(xref[j], L_[j]), U_[j]);
    }

    int32_t ignored_rows() const { return (int32_t)std::count(ignored_.begin(), ignored_.end(), (uint8_t)1); }

private:
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
        const char s = P_.sense[i];
        const double b = P_.b[i];
        const bool ge = s == 'G' || s == 'E', le = s == 'L' || s == 'E';
        const Activity act = activity(i);
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
            if (is_int_[j]) {
                if (lo > L_[j]) { L_[j] = lo; moved = true; }
                if (hi < U_[j]) { U_[j] = hi; moved = true; }
            } else {
                const double l0 = L_[j], u0 = U_[j];
                if (lo > l0 + kContMove * (1.0 + fabs(l0)) || (isinf(l0) && isfinite(lo))) { L_[j] = lo; moved = true; }
                if (hi < u0 - kContMove * (1.0 + fabs(u0)) || (isinf(u0) && isfinite(hi))) { U_[j] = hi; moved = true; }
            }
            if (moved) changed_.push_back(j);
        }
        return true;
    }

    const FPProblem &P_;
    const uint8_t *is_int_;
    std::vector<double> L_, U_, lo_new_, hi_new_;
    std::vector<uint8_t> ignored_, in_queue_;
    std::vector<int32_t> queue_, changed_;
    size_t head_ = 0;
};

}  // namespace

void build_incidence(FPProblem &P, std::vector<int32_t> &cptr, std::vector<int32_t> &crow)
{
    cptr.assign((size_t)P.n + 1, 0);
    for (int32_t e = P.ptr[0]; e < P.ptr[P.m]; ++e) cptr[P.col[e] + 1]++;
    for (int32_t j = 0; j < P.n; ++j) cptr[j + 1] += cptr[j];
    crow.resize(cptr[P.n]);
    std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
    for (int32_t i = 0; i < P.m; ++i)
        for (int32_t e = P.ptr[i]; e < P.ptr[i + 1]; ++e) crow[fill[P.col[e]]++] = i;
    P.cptr = cptr.data();
    P.crow = crow.data();
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
