// Batched fix-and-propagate on the device: a parallel form of the rounding
// of Section 2.3.  One workgroup rounds one instance.  The next K unfixed
// integer variables of the fixing order (ascending distance of the reference
// value to the nearest integer, ties by index) are fixed together to their
// reference values rounded half down and clamped to their domains; then
// propagation runs in synchronous rounds over the rows of the variables that
// changed.  A round evaluates every active row against the domains at its
// start (activity bounds, derived bounds, integer bounds rounded inward with
// 1e-9 slack, a row that excludes b or empties a domain is ignored for good),
// folds the derived bounds that would change a variable (integer: any
// tightening; continuous: by more than 1e-9 (1 + |bound|) or from infinite to
// finite) into per-variable max / min with 64-bit atomics on an
// order-preserving code of the doubles (so the result does not depend on the
// order of the rows), ignores every row that would change a variable whose
// combined domain is empty by more than 1e-9 (1 + |upper|) and folds again
// without them, pins a crossing within that tolerance to max(upper, old
// lower), and makes the rows of the changed variables active.  A batch ends
// with no active row or after max_rounds rounds.  All arithmetic is FP64 in
// the order the definition gives (no contraction), so the result is exact:
// equal to a sequential evaluation of the same rules.
#include "batch.h"

#include <cmath>
#include <rocprim/device/device_segmented_radix_sort.hpp>

// products and sums exactly as written: every activity and derived bound must
// round like a plain sequential evaluation
#pragma clang fp contract(off)

namespace {

struct FPBArgs {
    const int32_t *rptr;    // [M + 1] row pointers (global nonzero offsets)
    const int32_t *col;     // [NNZ] global column of each nonzero
    const double *val;      // [NNZ]
    const int32_t *cptr;    // [N + 1] column incidence pointers
    const int32_t *crow;    // [NNZ] global row of each incidence
    const double *b;        // [M]
    const uint8_t *sense;   // [M] 'G' / 'L' / 'E'
    const double *l, *u;    // [N] bounds as given
    const uint8_t *isint;   // [N]
    const double *xbar;     // [N] reference values
    const int32_t *order;   // [N] per instance: its integer columns in fixing order first
    const int32_t *row_off, *col_off;  // [count + 1]
    const int32_t *nint;    // [count] integer columns per instance
    const uint8_t *want;    // [count] or NULL
    double *L, *U;          // [N] domains
    unsigned long long *cL, *cU;  // [N] combined bounds of a round (codes)
    int32_t *vstamp;        // [N] last fold that listed the variable
    int32_t *rstamp;        // [M] last activation of the row
    uint8_t *ign, *bad;     // [M] ignored rows; rows caught by a conflict
    int32_t *act, *nxt;     // [M] active rows (per instance at its row offset)
    int32_t *touched;       // [N] variables folded in a round (at the column offset)
    double *xhat;           // [N]
    int32_t *info;          // [2 count] feasible, ignored rows
    int32_t K, max_rounds;
};

// Order-preserving 64-bit code of a double (NaN excluded): unsigned order of
// the codes equals the order of the values, -0 below +0.
__device__ __forceinline__ unsigned long long fpb_enc(double d)
{
    const unsigned long long w = (unsigned long long)__double_as_longlong(d);
    return (w >> 63) ? ~w : (w | 0x8000000000000000ull);
}

__device__ __forceinline__ double fpb_dec(unsigned long long c)
{
    const unsigned long long w = (c >> 63) ? (c & 0x7fffffffffffffffull) : ~c;
    return __longlong_as_double((long long)w);
}

__device__ __forceinline__ unsigned long long fpb_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void fpb_store(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct RowAct {
    double mn, mx;  // finite parts of the minimum / maximum activity
    int ni, xi;     // infinite contributions to each
};

// Activity bounds of row i over the current domains, nonzeros in row order.
__device__ RowAct fpb_activity(const FPBArgs &a, int i)
{
    RowAct r{0.0, 0.0, 0, 0};
    for (int e = a.rptr[i]; e < a.rptr[i + 1]; ++e) {
        const double v = a.val[e];
        if (v == 0.0) continue;
        const int j = a.col[e];
        const double lo = v > 0 ? a.L[j] : a.U[j];
        const double hi = v > 0 ? a.U[j] : a.L[j];
        if (isinf(lo)) r.ni++;
        else r.mn += v * lo;
        if (isinf(hi)) r.xi++;
        else r.mx += v * hi;
    }
    return r;
}

// Domain [nl, nu] that a row (sense sn, right-hand side bi, activity r)
// derives for one variable with coefficient v != 0 and domain [lo, hi].
__device__ __forceinline__ void fpb_derive(char sn, double bi, const RowAct &r, double v, double lo, double hi,
                                           bool isint, double &nl, double &nu)
{
    nl = lo;
    nu = hi;
    if (sn == 'G' || sn == 'E') {  // v x_j >= b - (max activity of the other terms)
        const double own = v > 0 ? hi : lo;
        const int own_inf = isinf(own) ? 1 : 0;
        if (r.xi - own_inf == 0) {
            const double rest = r.mx - (own_inf ? 0.0 : v * own);
            const double bnd = (bi - rest) / v;
            if (v > 0) nl = fmax(nl, bnd);
            else nu = fmin(nu, bnd);
        }
    }
    if (sn == 'L' || sn == 'E') {  // v x_j <= b - (min activity of the other terms)
        const double own = v > 0 ? lo : hi;
        const int own_inf = isinf(own) ? 1 : 0;
        if (r.ni - own_inf == 0) {
            const double rest = r.mn - (own_inf ? 0.0 : v * own);
            const double bnd = (bi - rest) / v;
            if (v > 0) nu = fmin(nu, bnd);
            else nl = fmax(nl, bnd);
        }
    }
    if (isint) {
        if (nl > lo) nl = ceil(nl - 1e-9);
        if (nu < hi) nu = floor(nu + 1e-9);
    }
}

__device__ __forceinline__ bool fpb_lower_changes(bool isint, double lo, double nl)
{
    if (isint) return nl > lo;
    return nl > lo + 1e-9 * (1.0 + fabs(lo)) || (isinf(lo) && isfinite(nl));
}

__device__ __forceinline__ bool fpb_upper_changes(bool isint, double hi, double nu)
{
    if (isint) return nu < hi;
    return nu < hi - 1e-9 * (1.0 + fabs(hi)) || (isinf(hi) && isfinite(nu));
}

// True if row i must be ignored against the current domains; r receives its
// activity bounds.
__device__ bool fpb_row_fails(const FPBArgs &a, int i, RowAct &r)
{
    r = fpb_activity(a, i);
    const char sn = (char)a.sense[i];
    const double bi = a.b[i];
    const double feas_tol = 1e-9 * (1.0 + fabs(bi));
    if ((sn == 'G' || sn == 'E') && r.xi == 0 && r.mx < bi - feas_tol) return true;
    if ((sn == 'L' || sn == 'E') && r.ni == 0 && r.mn > bi + feas_tol) return true;
    for (int e = a.rptr[i]; e < a.rptr[i + 1]; ++e) {
        const double v = a.val[e];
        if (v == 0.0) continue;
        const int j = a.col[e];
        double nl, nu;
        fpb_derive(sn, bi, r, v, a.L[j], a.U[j], a.isint[j] != 0, nl, nu);
        if (nl > nu + 1e-9 * (1.0 + fabs(nu))) return true;
    }
    return false;
}

// Folds the bounds row i derives that would change a variable into the
// combined bounds; lists each such variable once per fold stamp.
__device__ void fpb_fold(const FPBArgs &a, int i, const RowAct &r, int stamp, int32_t *touched, int *ntouched)
{
    const char sn = (char)a.sense[i];
    const double bi = a.b[i];
    for (int e = a.rptr[i]; e < a.rptr[i + 1]; ++e) {
        const double v = a.val[e];
        if (v == 0.0) continue;
        const int j = a.col[e];
        const double lo = a.L[j], hi = a.U[j];
        const bool ii = a.isint[j] != 0;
        double nl, nu;
        fpb_derive(sn, bi, r, v, lo, hi, ii, nl, nu);
        const bool tl = fpb_lower_changes(ii, lo, nl), tu = fpb_upper_changes(ii, hi, nu);
        if (!tl && !tu) continue;
        if (atomicExch(&a.vstamp[j], stamp) != stamp) touched[atomicAdd(ntouched, 1)] = j;
        if (tl) atomicMax(&a.cL[j], fpb_enc(nl));
        if (tu) atomicMin(&a.cU[j], fpb_enc(nu));
    }
}

// True if row i would change a variable whose combined domain is empty.
__device__ bool fpb_conflicts(const FPBArgs &a, int i, const RowAct &r)
{
    const char sn = (char)a.sense[i];
    const double bi = a.b[i];
    for (int e = a.rptr[i]; e < a.rptr[i + 1]; ++e) {
        const double v = a.val[e];
        if (v == 0.0) continue;
        const int j = a.col[e];
        const double NL = fpb_dec(fpb_load(&a.cL[j])), NU = fpb_dec(fpb_load(&a.cU[j]));
        if (!(NL > NU + 1e-9 * (1.0 + fabs(NU)))) continue;
        const double lo = a.L[j], hi = a.U[j];
        const bool ii = a.isint[j] != 0;
        double nl, nu;
        fpb_derive(sn, bi, r, v, lo, hi, ii, nl, nu);
        if (fpb_lower_changes(ii, lo, nl) || fpb_upper_changes(ii, hi, nu)) return true;
    }
    return false;
}

// Activates the non-ignored rows of column j (once per stamp).
__device__ __forceinline__ void fpb_activate(const FPBArgs &a, int j, int stamp, int32_t *list, int *n)
{
    for (int e = a.cptr[j]; e < a.cptr[j + 1]; ++e) {
        const int i = a.crow[e];
        if (!a.ign[i] && atomicExch(&a.rstamp[i], stamp) != stamp) list[atomicAdd(n, 1)] = i;
    }
}

// One workgroup per instance.  Every loop is bounded: a batch consumes at
// least one entry of the order, a batch runs at most max_rounds rounds, the
// row lists hold each row at most once per stamp.  Control values come from
// LDS after a barrier, so all threads take the same path through the
// barriers.
template <int NT>
__global__ __launch_bounds__(NT) void k_fp_batched(const FPBArgs a)
{
    constexpr int NW = NT / 64;
    __shared__ int s_wtot[NW];
    __shared__ int s_newp, s_nact, s_nnext, s_ntouched, s_conflict, s_bad, s_nign;
    const int q = blockIdx.x;
    if (a.want && !a.want[q]) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r0 = a.row_off[q], r1 = a.row_off[q + 1], c0 = a.col_off[q], c1 = a.col_off[q + 1];
    const int nint = a.nint[q];
    for (int j = c0 + tid; j < c1; j += NT) {
        double lo = a.l[j], hi = a.u[j];
        if (a.isint[j]) {
            if (isfinite(lo)) lo = ceil(lo - 1e-9);
            if (isfinite(hi)) hi = floor(hi + 1e-9);
        }
        a.L[j] = lo;
        a.U[j] = hi;
        fpb_store(&a.cL[j], fpb_enc(lo));
        fpb_store(&a.cU[j], fpb_enc(hi));
        a.vstamp[j] = -1;
    }
    for (int i = r0 + tid; i < r1; i += NT) {
        a.rstamp[i] = -1;
        a.ign[i] = 0;
        a.bad[i] = 0;
    }
    int32_t *act = a.act + r0, *nxt = a.nxt + r0;
    int32_t *touched = a.touched + c0;
    const int32_t *order = a.order + c0;
    int stamp = 0, p = 0;
    __syncthreads();
    while (p < nint) {
        // ---- the batch: the next K unfixed variables of the order
        ++stamp;
        const int fix_stamp = stamp;
        if (tid == 0) s_nact = 0;
        __syncthreads();
        int nsel = 0;
        while (nsel < a.K && p < nint) {
            const int idx = p + tid;
            int j = -1;
            bool unfixed = false;
            if (idx < nint) {
                j = order[idx];
                unfixed = a.L[j] != a.U[j];
            }
            const unsigned long long m = __ballot(unfixed);
            if (lane == 0) s_wtot[w] = __popcll(m);
            if (tid == 0) s_newp = -1;
            __syncthreads();
            int before = 0, total = 0;
            for (int k = 0; k < NW; ++k) {
                const int cnt = s_wtot[k];
                if (k < w) before += cnt;
                total += cnt;
            }
            const int rank = before + __popcll(m & ((1ull << lane) - 1ull));
            const int need = a.K - nsel;
            if (unfixed && rank < need) {
                const double lo = a.L[j], hi = a.U[j];
                double v = ceil(a.xbar[j] - 0.5);  // rounded half down
                if (!(v >= lo)) v = lo;  // a NaN reference takes the lower bound
                if (!(v <= hi)) v = hi;
                a.L[j] = v;
                a.U[j] = v;
                fpb_store(&a.cL[j], fpb_enc(v));
                fpb_store(&a.cU[j], fpb_enc(v));
                fpb_activate(a, j, fix_stamp, act, &s_nact);
                if (rank == need - 1) s_newp = idx + 1;
            }
            __syncthreads();
            if (total >= need) {
                nsel = a.K;
                p = s_newp;
            } else {
                nsel += total;
                p = min(p + NT, nint);
            }
            __syncthreads();
        }
        int nact = s_nact;
        __syncthreads();
        // ---- synchronous propagation rounds
        for (int round = 0; round < a.max_rounds && nact > 0; ++round) {
            ++stamp;
            const int fold1 = stamp;
            if (tid == 0) {
                s_ntouched = 0;
                s_conflict = 0;
                s_nnext = 0;
            }
            __syncthreads();
            for (int t = tid; t < nact; t += NT) {
                const int i = act[t];
                RowAct r;
                if (fpb_row_fails(a, i, r)) {
                    a.ign[i] = 1;
                    continue;
                }
                fpb_fold(a, i, r, fold1, touched, &s_ntouched);
            }
            __syncthreads();
            // is any combined domain empty?  (rare: only then are the rows
            // behind it looked for)
            for (int t = tid, nt = s_ntouched; t < nt; t += NT) {
                const int j = touched[t];
                const double NL = fpb_dec(fpb_load(&a.cL[j])), NU = fpb_dec(fpb_load(&a.cU[j]));
                if (NL > NU + 1e-9 * (1.0 + fabs(NU))) atomicOr(&s_conflict, 1);
            }
            __syncthreads();
            if (s_conflict) {
                for (int t = tid; t < nact; t += NT) {
                    const int i = act[t];
                    if (a.ign[i]) continue;
                    const RowAct r = fpb_activity(a, i);
                    if (fpb_conflicts(a, i, r)) a.bad[i] = 1;
                }
                __syncthreads();
                const int nt = s_ntouched;
                for (int t = tid; t < nact; t += NT) {
                    const int i = act[t];
                    if (a.bad[i]) {
                        a.bad[i] = 0;
                        a.ign[i] = 1;
                    }
                }
                for (int t = tid; t < nt; t += NT) {
                    const int j = touched[t];
                    fpb_store(&a.cL[j], fpb_enc(a.L[j]));
                    fpb_store(&a.cU[j], fpb_enc(a.U[j]));
                }
                ++stamp;
                const int fold2 = stamp;
                __syncthreads();
                if (tid == 0) s_ntouched = 0;
                __syncthreads();
                for (int t = tid; t < nact; t += NT) {
                    const int i = act[t];
                    if (a.ign[i]) continue;
                    const RowAct r = fpb_activity(a, i);
                    fpb_fold(a, i, r, fold2, touched, &s_ntouched);
                }
                __syncthreads();
            }
            ++stamp;
            const int push = stamp;
            const int nt = s_ntouched;
            for (int t = tid; t < nt; t += NT) {
                const int j = touched[t];
                const double lo = a.L[j], hi = a.U[j];
                double nl = fpb_dec(fpb_load(&a.cL[j])), nu = fpb_dec(fpb_load(&a.cU[j]));
                if (nl > nu) nl = nu = fmax(nu, lo);
                a.L[j] = nl;
                a.U[j] = nu;
                fpb_store(&a.cL[j], fpb_enc(nl));
                fpb_store(&a.cU[j], fpb_enc(nu));
                if (nl != lo || nu != hi) fpb_activate(a, j, push, nxt, &s_nnext);
            }
            __syncthreads();
            nact = s_nnext;
            int32_t *sw = act;
            act = nxt;
            nxt = sw;
            __syncthreads();
        }
    }
    // ---- the rounding, and its report
    for (int j = c0 + tid; j < c1; j += NT) {
        const double lo = a.L[j], hi = a.U[j];
        double v = lo;
        if (!a.isint[j]) {
            v = a.xbar[j];
            if (v < lo) v = lo;
            if (v > hi) v = hi;
        }
        a.xhat[j] = v;
    }
    if (tid == 0) {
        s_bad = 0;
        s_nign = 0;
    }
    __syncthreads();
    int nign = 0, bad = 0;
    for (int i = r0 + tid; i < r1; i += NT) {
        nign += a.ign[i];
        double s = 0.0;
        for (int e = a.rptr[i]; e < a.rptr[i + 1]; ++e) s += a.val[e] * a.xhat[a.col[e]];
        const double bi = a.b[i], tol = 1e-6 * (1.0 + fabs(bi));
        const char sn = (char)a.sense[i];
        if (!isfinite(s)) bad = 1;  // a non-finite activity satisfies no row
        if ((sn == 'G' || sn == 'E') && s < bi - tol) bad = 1;
        if ((sn == 'L' || sn == 'E') && s > bi + tol) bad = 1;
    }
    if (nign) atomicAdd(&s_nign, nign);
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (tid == 0) {
        a.info[2 * q] = s_bad ? 0 : 1;
        a.info[2 * q + 1] = s_nign;
    }
}

// Sort keys: the distance of the reference value to the nearest integer for
// integer columns (1 for a non-finite value: after the finite ones, before
// any continuous column), 2 (after every integer) for continuous ones;
// values: the column index, so that a stable sort breaks ties by index.
template <class V>
__global__ __launch_bounds__(256) void k_fp_keys(const V *x, const double *xin, const uint8_t *isint, int32_t N,
                                                 double *xbar, double *key, int32_t *idx)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double v = xin ? xin[j] : (double)x[j];
    xbar[j] = v;
    const double f = v - floor(v);
    key[j] = isint[j] ? (isfinite(v) ? (f < 1.0 - f ? f : 1.0 - f) : 1.0) : 2.0;
    idx[j] = j;
}

}  // namespace

namespace scy {

static void fp_setup(scylla_batch *h)
{
    FPDev &d = h->fpd;
    if (d.ready) return;
    const int32_t M = h->M, N = h->N, count = h->count;
    const HostOrient &o = h->orow.host;
    const size_t nnz = (size_t)o.ptr[M];
    std::vector<int32_t> col(nnz), cptr((size_t)N + 1, 0), crow(nnz);
    for (size_t e = 0; e < nnz; ++e) col[e] = (int32_t)(h->fmt == FMT_PACKED ? (o.ent[e] & o.mask) : o.ent[e]);
    for (size_t e = 0; e < nnz; ++e) cptr[(size_t)col[e] + 1]++;
    for (int32_t j = 0; j < N; ++j) cptr[j + 1] += cptr[j];
    {
        std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
        for (int32_t i = 0; i < M; ++i)
            for (int32_t e = o.ptr[i]; e < o.ptr[i + 1]; ++e) crow[fill[col[e]]++] = i;
    }
    const hipStream_t s = h->stream;
    upload(d.rptr, o.ptr, s);
    upload(d.col, col, s);
    upload(d.val, h->hval, s);
    upload(d.cptr, cptr, s);
    upload(d.crow, crow, s);
    upload(d.rowoff, h->row_off, s);
    upload(d.coloff, h->col_off, s);
    const size_t n1 = (size_t)std::max(N, 1), m1 = (size_t)std::max(M, 1);
    d.nint.alloc((size_t)count * 4);
    d.isint.alloc(n1);
    d.want.alloc((size_t)std::max(count, 1));
    for (DevMem *v : {&d.xbar, &d.key, &d.key2, &d.L, &d.U, &d.xhat}) v->alloc(n1 * 8);
    for (DevMem *v : {&d.cL, &d.cU}) v->alloc(n1 * 8);
    for (DevMem *v : {&d.ord0, &d.ord, &d.vst, &d.chg}) v->alloc(n1 * 4);
    for (DevMem *v : {&d.rst, &d.act, &d.nxt}) v->alloc(m1 * 4);
    for (DevMem *v : {&d.ign, &d.bad}) v->alloc(m1);
    d.info.alloc((size_t)std::max(count, 1) * 8);
    size_t bytes = 0;
    if (N > 0)
        HIPC(rocprim::segmented_radix_sort_pairs(nullptr, bytes, d.key.as<double>(), d.key2.as<double>(),
                                             d.ord0.as<int32_t>(), d.ord.as<int32_t>(), (unsigned)N,
                                             (unsigned)count, d.coloff.as<int32_t>(), d.coloff.as<int32_t>() + 1,
                                             0, 64, s));
    d.tmp.alloc(std::max<size_t>(bytes, 16));
    d.tmp_bytes = bytes;
    HIPC(hipStreamSynchronize(s));
    d.ready = true;
}

void fp_batched(scylla_batch *h, const uint8_t *is_int, const double *xbar, int32_t K, int32_t max_rounds,
                const uint8_t *want, double *xhat, int32_t *info, uint8_t *ignored)
{
    if (K < 1) throw_err(-EINVAL, "fix-and-propagate batch size must be >= 1");
    if (max_rounds < 1) throw_err(-EINVAL, "fix-and-propagate max_rounds must be >= 1");
    if (!is_int || !xhat || !info) throw_err(-EINVAL, "is_int, xhat and info must not be NULL");
    const int32_t M = h->M, N = h->N, count = h->count;
    if (xbar)
        for (int32_t j = 0; j < N; ++j)
            if (!std::isfinite(xbar[j])) throw_err(-EINVAL, "reference values must be finite");
    fp_setup(h);
    FPDev &d = h->fpd;
    const hipStream_t s = h->stream;
    std::vector<int32_t> nint(count, 0);
    for (int32_t q = 0; q < count; ++q)
        for (int32_t j = h->col_off[q]; j < h->col_off[q + 1]; ++j) nint[q] += is_int[j] ? 1 : 0;
    std::vector<uint8_t> ii(is_int, is_int + N);
    for (auto &v : ii) v = v ? 1 : 0;
    if (N > 0) HIPC(hipMemcpyAsync(d.isint.p, ii.data(), (size_t)N, hipMemcpyHostToDevice, s));
    if (count > 0) HIPC(hipMemcpyAsync(d.nint.p, nint.data(), (size_t)count * 4, hipMemcpyHostToDevice, s));
    if (want && count > 0) HIPC(hipMemcpyAsync(d.want.p, want, (size_t)count, hipMemcpyHostToDevice, s));
    if (xbar && N > 0) HIPC(hipMemcpyAsync(d.xbar.p, xbar, (size_t)N * 8, hipMemcpyHostToDevice, s));
    if (N > 0) {
        const double *xin = xbar ? d.xbar.as<double>() : nullptr;
        const dim3 g((unsigned)((N + 255) / 256));
        if (h->precision == SCYLLA_FP64)
            k_fp_keys<double><<<g, 256, 0, s>>>(h->x.as<double>(), xin, d.isint.as<uint8_t>(), N,
                                                d.xbar.as<double>(), d.key.as<double>(), d.ord0.as<int32_t>());
        else
            k_fp_keys<float><<<g, 256, 0, s>>>(h->x.as<float>(), xin, d.isint.as<uint8_t>(), N,
                                               d.xbar.as<double>(), d.key.as<double>(), d.ord0.as<int32_t>());
        HIPC(hipGetLastError());
        size_t bytes = d.tmp_bytes;
        HIPC(rocprim::segmented_radix_sort_pairs(d.tmp.p, bytes, d.key.as<double>(), d.key2.as<double>(),
                                                 d.ord0.as<int32_t>(), d.ord.as<int32_t>(), (unsigned)N,
                                                 (unsigned)count, d.coloff.as<int32_t>(),
                                                 d.coloff.as<int32_t>() + 1, 0, 64, s));
    }
    FPBArgs a{};
    a.rptr = d.rptr.as<int32_t>();
    a.col = d.col.as<int32_t>();
    a.val = d.val.as<double>();
    a.cptr = d.cptr.as<int32_t>();
    a.crow = d.crow.as<int32_t>();
    a.b = h->b64.as<double>();
    a.sense = h->sense.as<uint8_t>();
    a.l = h->l64.as<double>();
    a.u = h->u64.as<double>();
    a.isint = d.isint.as<uint8_t>();
    a.xbar = d.xbar.as<double>();
    a.order = d.ord.as<int32_t>();
    a.row_off = d.rowoff.as<int32_t>();
    a.col_off = d.coloff.as<int32_t>();
    a.nint = d.nint.as<int32_t>();
    a.want = want ? d.want.as<uint8_t>() : nullptr;
    a.L = d.L.as<double>();
    a.U = d.U.as<double>();
    a.cL = d.cL.as<unsigned long long>();
    a.cU = d.cU.as<unsigned long long>();
    a.vstamp = d.vst.as<int32_t>();
    a.rstamp = d.rst.as<int32_t>();
    a.ign = d.ign.as<uint8_t>();
    a.bad = d.bad.as<uint8_t>();
    a.act = d.act.as<int32_t>();
    a.nxt = d.nxt.as<int32_t>();
    a.touched = d.chg.as<int32_t>();
    a.xhat = d.xhat.as<double>();
    a.info = d.info.as<int32_t>();
    a.K = K;
    a.max_rounds = max_rounds;
    if (count > 0) {
        k_fp_batched<256><<<dim3((unsigned)count), dim3(256), 0, s>>>(a);
        HIPC(hipGetLastError());
    }
    std::vector<double> hx((size_t)N);
    std::vector<int32_t> hi((size_t)count * 2);
    std::vector<uint8_t> hg(ignored ? (size_t)M : 0);
    if (N > 0) HIPC(hipMemcpyAsync(hx.data(), d.xhat.p, (size_t)N * 8, hipMemcpyDeviceToHost, s));
    if (count > 0) HIPC(hipMemcpyAsync(hi.data(), d.info.p, (size_t)count * 8, hipMemcpyDeviceToHost, s));
    if (ignored && M > 0) HIPC(hipMemcpyAsync(hg.data(), d.ign.p, (size_t)M, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int32_t q = 0; q < count; ++q) {
        if (want && !want[q]) continue;
        const int32_t c0 = h->col_off[q], c1 = h->col_off[q + 1];
        memcpy(xhat + c0, hx.data() + c0, sizeof(double) * (size_t)(c1 - c0));
        info[2 * q] = hi[2 * q];
        info[2 * q + 1] = hi[2 * q + 1];
        if (ignored) {
            const int32_t r0 = h->row_off[q], r1 = h->row_off[q + 1];
            memcpy(ignored + r0, hg.data() + r0, (size_t)(r1 - r0));
        }
    }
}

}  // namespace scy

extern "C" int scylla_batch_fix_propagate(scylla_batch *h, const uint8_t *is_int, const double *xbar, int32_t K,
                                          int32_t max_rounds, double *xhat, int32_t *info, uint8_t *ignored)
{
    return guarded([&]() -> int {
        if (!h) throw_err(-EINVAL, "handle is NULL");
        if (!xhat || !info) throw_err(-EINVAL, "xhat and info must not be NULL");
        std::vector<uint8_t> ii((size_t)h->N, 1);
        if (is_int)
            for (int32_t j = 0; j < h->N; ++j) ii[j] = is_int[j] ? 1 : 0;
        fp_batched(h, ii.data(), xbar, K, max_rounds, nullptr, xhat, info, ignored);
        return 0;
    });
}
