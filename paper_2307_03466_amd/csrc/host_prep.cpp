// Host-side preparation of a batch of LPs: input validation, concatenation
// into one block-diagonal matrix, the explicit transposed copy used by the
// column pass (so A^T y needs no atomics), exact compact value formats, and
// the tile plans both passes launch over.  Plain C++, no GPU calls.
#include <errno.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "scylla_internal.h"

namespace scy {

// Runs fn(k) for k in [0, n) on up to 16 host threads in contiguous,
// dynamically handed-out chunks.  Every k writes only its own outputs, so
// results do not depend on the schedule.
template <class F>
static void parallel_chunks(int64_t n, int64_t chunk, F &&fn)
{
    if (n <= 0) return;
    const int64_t nchunks = (n + chunk - 1) / chunk;
    const int nt = (int)std::min<int64_t>(nchunks, std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (int64_t c = next++; c < nchunks; c = next++)
            for (int64_t k = c * chunk, e = std::min(n, k + chunk); k < e; ++k) fn(k);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

static int fail(std::string &err, const char *fmt, long long a = 0, long long b = 0)
{
    char buf[256];
    snprintf(buf, sizeof(buf), fmt, a, b);
    err = buf;
    return -EINVAL;
}

int validate_lp(const scylla_lp *lp, std::string &err)
{
    if (!lp) return fail(err, "lp is NULL");
    const scylla_csr &A = lp->A;
    if (A.m < 0 || A.n < 1) return fail(err, "need m >= 0 and n >= 1 (m=%lld, n=%lld)", A.m, A.n);
    if (A.nnz < 0 || A.nnz >= 0x7fffffffLL) return fail(err, "nnz out of range (%lld)", A.nnz);
    if (!A.row_ptr) return fail(err, "row_ptr is NULL");
    if (A.nnz > 0 && (!A.col_idx || !A.val)) return fail(err, "col_idx/val is NULL");
    if (!lp->c || !lp->l || !lp->u) return fail(err, "c, l or u is NULL");
    if (A.m > 0 && (!lp->b || !lp->senses)) return fail(err, "b or senses is NULL");
    if (A.row_ptr[0] != 0) return fail(err, "row_ptr[0] = %lld, expected 0", A.row_ptr[0]);
    if (A.row_ptr[A.m] != A.nnz)
        return fail(err, "row_ptr[m] = %lld differs from nnz = %lld", A.row_ptr[A.m], A.nnz);
    for (int32_t i = 0; i < A.m; ++i) {
        int64_t a = A.row_ptr[i], b = A.row_ptr[i + 1];
        if (b < a) return fail(err, "row_ptr decreases at row %lld", i);
        int32_t prev = -1;
        for (int64_t e = a; e < b; ++e) {
            int32_t j = A.col_idx[e];
            if (j < 0 || j >= A.n) return fail(err, "col_idx out of range at nonzero %lld (%lld)", e, j);
            if (j <= prev) return fail(err, "col_idx not strictly increasing in row %lld", i);
            prev = j;
            if (!isfinite(A.val[e])) return fail(err, "non-finite matrix value at nonzero %lld", e);
        }
        char s = lp->senses[i];
        if (s != 'G' && s != 'L' && s != 'E') return fail(err, "bad sense %lld at row %lld", (unsigned char)s, i);
        if (!isfinite(lp->b[i])) return fail(err, "non-finite b at row %lld", i);
    }
    for (int32_t j = 0; j < A.n; ++j) {
        double l = lp->l[j], u = lp->u[j];
        if (isnan(l) || isnan(u)) return fail(err, "NaN bound at column %lld", j);
        if (l > u) return fail(err, "l > u at column %lld", j);
        if (l == INFINITY || u == -INFINITY) return fail(err, "infeasible infinite bound at column %lld", j);
        if (!isfinite(lp->c[j])) return fail(err, "non-finite objective at column %lld", j);
    }
    return 0;
}

uint16_t f64_to_bf16_exact(double v, bool &exact)
{
    float f = (float)v;
    uint32_t w;
    memcpy(&w, &f, 4);
    exact = ((double)f == v) && ((w & 0xffffu) == 0u);
    return (uint16_t)(w >> 16);
}

static int32_t bits_for(int64_t maxval)
{
    int32_t b = 1;
    while (b < 31 && ((int64_t)1 << b) <= maxval) ++b;
    return b;
}

int build_orientations(const scylla_lp *lps, int32_t count, int32_t precision, HostOrient &csr,
                       HostOrient &csc, int32_t &fmt, std::vector<int32_t> &row_off,
                       std::vector<int32_t> &col_off, std::string &err)
{
    int64_t M = 0, N = 0, NNZ = 0;
    row_off.assign(count + 1, 0);
    col_off.assign(count + 1, 0);
    for (int32_t q = 0; q < count; ++q) {
        row_off[q] = (int32_t)M;
        col_off[q] = (int32_t)N;
        M += lps[q].A.m;
        N += lps[q].A.n;
        NNZ += lps[q].A.nnz;
        if (M >= 0x7fffffffLL || N >= 0x7fffffffLL || NNZ >= 0x7fffffffLL)
            return fail(err, "batch too large: totals must stay below 2^31 - 1");
    }
    row_off[count] = (int32_t)M;
    col_off[count] = (int32_t)N;

    // storage format: FP64 path stores FP64; FP32 path picks the most compact
    // exact format for every value of the batch
    const int32_t sh_r = bits_for(N > 1 ? N - 1 : 1);  // CSR words hold column ids
    const int32_t sh_c = bits_for(M > 1 ? M - 1 : 1);  // CSC words hold row ids
    if (precision == SCYLLA_FP64) {
        fmt = FMT_F64;
    } else {
        const int32_t sh = std::max(sh_r, sh_c);
        const int64_t vmax = ((int64_t)1 << (31 - sh)) - 1, vmin = -((int64_t)1 << (31 - sh));
        bool packed = sh <= 30, bf16 = true;
        for (int32_t q = 0; q < count && (packed || bf16); ++q) {
            const scylla_csr &A = lps[q].A;
            for (int64_t e = 0; e < A.nnz; ++e) {
                double v = A.val[e];
                if (packed && !(v == floor(v) && v >= (double)vmin && v <= (double)vmax)) packed = false;
                bool ex;
                f64_to_bf16_exact(v, ex);
                if (!ex) bf16 = false;
                if (!packed && !bf16) break;
            }
        }
        fmt = packed ? FMT_PACKED : (bf16 ? FMT_BF16 : FMT_F32);
    }

    csr.rows = (int32_t)M;
    csc.rows = (int32_t)N;
    csr.ptr.assign(M + 1, 0);
    csc.ptr.assign(N + 1, 0);
    csr.ent.resize(NNZ);
    csc.ent.resize(NNZ);
    std::vector<double> cval(NNZ), rval(NNZ);
    std::vector<int32_t> crow(NNZ);
    // CSR (global column ids)
    int64_t e_out = 0;
    for (int32_t q = 0; q < count; ++q) {
        const scylla_csr &A = lps[q].A;
        for (int32_t i = 0; i < A.m; ++i) {
            for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1]; ++e) {
                csr.ent[e_out] = (uint32_t)(A.col_idx[e] + col_off[q]);
                rval[e_out] = A.val[e];
                ++e_out;
            }
            csr.ptr[row_off[q] + i + 1] = (int32_t)e_out;
        }
    }
    // CSC by a stable counting sort over the CSR entries (row order), so the
    // rows of every column are increasing
    for (int64_t e = 0; e < NNZ; ++e) csc.ptr[csr.ent[e] + 1]++;
    for (int64_t j = 0; j < N; ++j) csc.ptr[j + 1] += csc.ptr[j];
    {
        std::vector<int32_t> fill(csc.ptr.begin(), csc.ptr.end() - 1);
        for (int64_t i = 0; i < M; ++i)
            for (int32_t e = csr.ptr[i]; e < csr.ptr[i + 1]; ++e) {
                int32_t pos = fill[csr.ent[e]]++;
                csc.ent[pos] = (uint32_t)i;
                cval[pos] = rval[e];
            }
    }
    auto finish = [&](HostOrient &o, std::vector<double> &vals, int32_t sh) {
        if (fmt == FMT_PACKED) {
            o.shift = sh;
            o.mask = (sh >= 32) ? 0xffffffffu : ((1u << sh) - 1u);
            for (int64_t e = 0; e < NNZ; ++e)
                o.ent[e] |= ((uint32_t)(int32_t)vals[e]) << sh;
        } else if (fmt == FMT_BF16) {
            o.v16.resize(NNZ);
            bool ex;
            for (int64_t e = 0; e < NNZ; ++e) o.v16[e] = f64_to_bf16_exact(vals[e], ex);
        } else if (fmt == FMT_F32) {
            o.v32.resize(NNZ);
            for (int64_t e = 0; e < NNZ; ++e) o.v32[e] = (float)vals[e];
        } else {
            o.v64 = vals;
        }
    };
    finish(csr, rval, sh_r);
    finish(csc, cval, sh_c);
    return 0;
}

void plan_tiles(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                int32_t chunk, int32_t max_rows, TilePlan &plan, const uint8_t *skip)
{
    const int32_t count = (int32_t)inst_off.size() - 1;
    plan.chunk = chunk;
    plan.tiles.clear();
    plan.longs.clear();
    plan.nslots = 0;
    plan.t_begin.assign(count, 0);
    plan.t_end.assign(count, 0);
    plan.l_begin.assign(count, 0);
    plan.l_end.assign(count, 0);
    for (int32_t q = 0; q < count; ++q) {
        plan.t_begin[q] = (int32_t)(plan.tiles.size() / 4);
        plan.l_begin[q] = (int32_t)(plan.longs.size() / 4);
        int32_t r = inst_off[q];
        const int32_t rend = (skip && skip[q]) ? r : inst_off[q + 1];
        while (r < rend) {
            int32_t len = ptr[r + 1] - ptr[r];
            if (len > chunk) {
                int32_t nseg = (len + chunk - 1) / chunk;
                plan.longs.insert(plan.longs.end(), {r, plan.nslots, nseg, q});
                for (int32_t s = 0; s < nseg; ++s) {
                    int32_t a = ptr[r] + s * chunk;
                    int32_t b = std::min(a + chunk, ptr[r + 1]);
                    plan.tiles.insert(plan.tiles.end(), {a, b, q, plan.nslots + s});
                }
                plan.nslots += nseg;
                ++r;
                continue;
            }
            int32_t start = r, nz = 0;
            while (r < rend && r - start < max_rows) {
                int32_t l2 = ptr[r + 1] - ptr[r];
                if (l2 > chunk || nz + l2 > chunk) break;
                nz += l2;
                ++r;
            }
            plan.tiles.insert(plan.tiles.end(), {start, r, q, -1});
        }
        plan.t_end[q] = (int32_t)(plan.tiles.size() / 4);
        plan.l_end[q] = (int32_t)(plan.longs.size() / 4);
    }
}

static inline int32_t entry_index(const HostOrient &o, int32_t fmt, int64_t e)
{
    return fmt == FMT_PACKED ? (int32_t)(o.ent[e] & o.mask) : (int32_t)o.ent[e];
}

void build_blocked(const HostOrient &o, int32_t fmt, int32_t gather_size, int32_t B, BlockedHost &out)
{
    const int32_t rows = o.rows;
    const int64_t nnz = (int64_t)o.ent.size();
    out.B = B;
    out.bounds.assign(B + 1, 0);
    for (int32_t b = 0; b <= B; ++b) out.bounds[b] = (int32_t)(((int64_t)gather_size * b) / B);
    // count nonzeros per (block, row)
    out.bptr.assign((size_t)B * (rows + 1), 0);
    parallel_chunks(rows, 4096, [&](int64_t k) {
        const int32_t i = (int32_t)k;
        int32_t b = 0;
        for (int32_t e = o.ptr[i]; e < o.ptr[i + 1]; ++e) {
            const int32_t g = entry_index(o, fmt, e);
            while (g >= out.bounds[b + 1]) ++b;
            out.bptr[(size_t)b * (rows + 1) + i + 1]++;
        }
    });
    int64_t base = 0;
    for (int32_t b = 0; b < B; ++b) {
        int32_t *p = out.bptr.data() + (size_t)b * (rows + 1);
        p[0] = (int32_t)base;
        for (int32_t i = 0; i < rows; ++i) p[i + 1] += p[i];
        base = p[rows];
    }
    out.ent.resize(nnz);
    if (fmt == FMT_BF16) out.v16.resize(nnz);
    if (fmt == FMT_F32) out.v32.resize(nnz);
    if (fmt == FMT_F64) out.v64.resize(nnz);
    parallel_chunks(rows, 4096, [&](int64_t k) {
        const int32_t i = (int32_t)k;
        int32_t b = 0, pos = out.bptr[i];
        for (int32_t e = o.ptr[i]; e < o.ptr[i + 1]; ++e) {
            const int32_t g = entry_index(o, fmt, e);
            if (g >= out.bounds[b + 1]) {
                while (g >= out.bounds[b + 1]) ++b;
                pos = out.bptr[(size_t)b * (rows + 1) + i];
            }
            out.ent[pos] = o.ent[e];
            if (fmt == FMT_BF16) out.v16[pos] = o.v16[e];
            if (fmt == FMT_F32) out.v32[pos] = o.v32[e];
            if (fmt == FMT_F64) out.v64[pos] = o.v64[e];
            ++pos;
        }
    });
}

void plan_blocked(const BlockedHost &bh, int32_t rows, const std::vector<int32_t> &inst_off, int32_t chunk,
                  int32_t max_rows, BlockedPlan &plan)
{
    const int32_t B = bh.B, XCD = 8, G = XCD / B;
    const int32_t count = (int32_t)inst_off.size() - 1;
    plan.chunk = chunk;
    plan.tiles.clear();
    plan.longs.clear();
    plan.nslots = 0;
    std::vector<std::vector<int32_t>> per_xcd(XCD);
    for (int32_t b = 0; b < B; ++b) {
        std::vector<int32_t> ptr(bh.bptr.begin() + (size_t)b * (rows + 1),
                                 bh.bptr.begin() + (size_t)(b + 1) * (rows + 1));
        TilePlan tp;
        plan_tiles(ptr, inst_off, chunk, max_rows, tp);
        const int32_t ntile = (int32_t)(tp.tiles.size() / 4);
        for (int32_t k = 0; k < ntile; ++k) {
            const int32_t *t = tp.tiles.data() + 4 * k;
            const int32_t slot = t[3] >= 0 ? t[3] + plan.nslots : -1;
            auto &dst = per_xcd[b + (k % G) * B];
            dst.insert(dst.end(), {t[0], t[1], t[2] | (b << 24), slot});
        }
        for (size_t q = 0; q < tp.longs.size(); q += 4)
            plan.longs.insert(plan.longs.end(),
                              {tp.longs[q], tp.longs[q + 1] + plan.nslots, tp.longs[q + 2], tp.longs[q + 3] | (b << 24)});
        plan.nslots += tp.nslots;
    }
    size_t K = 0;
    for (auto &v : per_xcd) K = std::max(K, v.size() / 4);
    plan.tiles.assign(K * XCD * 4, 0);
    for (size_t j = 0; j < K; ++j)
        for (int32_t x = 0; x < XCD; ++x) {
            int32_t *d = plan.tiles.data() + 4 * (j * XCD + x);
            if (4 * j < per_xcd[x].size()) {
                for (int c = 0; c < 4; ++c) d[c] = per_xcd[x][4 * j + c];
            } else {
                d[0] = d[1] = d[2] = 0;
                d[3] = -1;
            }
        }
    // combine tiles: up to 256 rows of one instance each
    plan.ctiles.clear();
    plan.ct_begin.assign(count, 0);
    plan.ct_end.assign(count, 0);
    for (int32_t q = 0; q < count; ++q) {
        plan.ct_begin[q] = (int32_t)(plan.ctiles.size() / 4);
        for (int32_t r = inst_off[q]; r < inst_off[q + 1]; r += 256)
            plan.ctiles.insert(plan.ctiles.end(), {r, std::min(r + 256, inst_off[q + 1]), q, -1});
        plan.ct_end[q] = (int32_t)(plan.ctiles.size() / 4);
    }
}

// Cuts the sub-tiles [t0, t1) of one instance (nz(t) nonzeros each) into
// k = ceil(total / group_nnz) runs of about total / k nonzeros and appends
// their boundaries t0 < c1 < ... < t1 to cuts: the tiles of a pass run at
// the same time, so the longest one sets its duration, and runs of exactly
// group_nnz would leave a short last tile per instance.
template <class NZ>
static void balanced_runs(int32_t t0, int32_t t1, int64_t group_nnz, NZ nz, std::vector<int32_t> &cuts)
{
    cuts.assign(1, t0);
    int64_t total = 0;
    for (int32_t t = t0; t < t1; ++t) total += nz(t);
    const int64_t k = std::max<int64_t>(1, (total + group_nnz - 1) / std::max<int64_t>(group_nnz, 1));
    int64_t acc = 0, j = 1;
    for (int32_t t = t0; t < t1; ++t) {
        acc += nz(t);
        bool cut = false;
        while (j < k && acc * k >= j * total) {
            ++j;
            cut = true;
        }
        if (cut && t + 1 < t1) cuts.push_back(t + 1);
    }
    cuts.push_back(t1);
}

void plan_staged(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, int32_t max_vec, int32_t sub_chunk, int32_t group_nnz,
                 int32_t rest_chunk, StagedPlan &plan)
{
    const int32_t count = (int32_t)inst_off.size() - 1;
    plan.tiles.clear();
    plan.staged.assign(count, 0);
    plan.max_vec = 0;
    std::vector<uint8_t> not_staged(count, 1);
    for (int32_t q = 0; q < count; ++q) {
        const int32_t glen = gofs[q + 1] - gofs[q];
        if (glen > max_vec || inst_off[q + 1] == inst_off[q]) continue;
        bool short_rows = true;
        for (int32_t r = inst_off[q]; r < inst_off[q + 1] && short_rows; ++r)
            short_rows = ptr[r + 1] - ptr[r] <= sub_chunk;
        if (!short_rows) continue;
        plan.staged[q] = 1;
        not_staged[q] = 0;
        plan.max_vec = std::max(plan.max_vec, glen);
    }
    plan_tiles(ptr, inst_off, sub_chunk, 4 * 1024, plan.sub, not_staged.data());
    std::vector<int32_t> cuts;
    for (int32_t q = 0; q < count; ++q) {
        if (!plan.staged[q] || plan.sub.t_end[q] == plan.sub.t_begin[q]) continue;
        balanced_runs(plan.sub.t_begin[q], plan.sub.t_end[q], group_nnz, [&](int32_t t) {
            const int32_t *d = plan.sub.tiles.data() + 4 * t;
            return (int64_t)(ptr[d[1]] - ptr[d[0]]);
        }, cuts);
        for (size_t c = 0; c + 1 < cuts.size(); ++c) plan.tiles.insert(plan.tiles.end(), {cuts[c], cuts[c + 1], q, -1});
    }
    plan_tiles(ptr, inst_off, rest_chunk, 1024, plan.rest, plan.staged.data());
}

void build_sliced(const HostOrient &o, int32_t fmt, const std::vector<int32_t> &inst_off,
                  const std::vector<int32_t> &gofs, const std::vector<uint8_t> &candidate, int32_t max_vec,
                  int32_t max_slices, int32_t sub_chunk, SlicedPlan &plan)
{
    const int32_t count = (int32_t)inst_off.size() - 1;
    const int32_t rows = o.rows;
    plan = SlicedPlan();
    plan.sliced.assign(count, 0);
    // slice count per instance: enough for its gathered vector; the slice
    // arrays are sized for the longest qualifying instance
    int64_t longest = 0;
    std::vector<uint8_t> ok(count, 0);
    for (int32_t q = 0; q < count; ++q) {
        const int64_t glen = gofs[q + 1] - gofs[q];
        if (!candidate[q] || glen <= max_vec || glen > (int64_t)max_slices * max_vec) continue;
        if (inst_off[q + 1] == inst_off[q]) continue;
        bool short_rows = true;
        for (int32_t r = inst_off[q]; r < inst_off[q + 1] && short_rows; ++r)
            short_rows = o.ptr[r + 1] - o.ptr[r] <= sub_chunk;
        if (!short_rows) continue;
        ok[q] = 1;
        longest = std::max(longest, glen);
    }
    if (longest == 0) return;
    const int32_t S = (int32_t)((longest + max_vec - 1) / max_vec);
    plan.S = S;
    plan.Sq.assign(count, 0);
    for (int32_t q = 0; q < count; ++q) {
        plan.sliced[q] = ok[q];
        if (ok[q]) plan.Sq[q] = (int32_t)((gofs[q + 1] - gofs[q] + max_vec - 1) / max_vec);
    }
    // entries of sliced instances regrouped by slice
    auto slice_of = [&](int32_t q, int32_t g) {
        const int64_t glen = gofs[q + 1] - gofs[q], rel = g - gofs[q];
        const int32_t Sq = plan.Sq[q];
        int32_t s = (int32_t)((rel * Sq) / glen);
        // s is the slice with glen*s/Sq <= rel < glen*(s+1)/Sq
        while (s > 0 && (glen * s) / Sq > rel) --s;
        while (s + 1 < Sq && (glen * (s + 1)) / Sq <= rel) ++s;
        return s;
    };
    plan.bptr.assign((size_t)S * (rows + 1), 0);
    parallel_chunks(count, 1, [&](int64_t k) {
        const int32_t q = (int32_t)k;
        if (!ok[q]) return;
        for (int32_t i = inst_off[q]; i < inst_off[q + 1]; ++i)
            for (int32_t e = o.ptr[i]; e < o.ptr[i + 1]; ++e)
                plan.bptr[(size_t)slice_of(q, entry_index(o, fmt, e)) * (rows + 1) + i + 1]++;
    });
    int64_t base = 0;
    for (int32_t s = 0; s < S; ++s) {
        int32_t *p = plan.bptr.data() + (size_t)s * (rows + 1);
        p[0] = (int32_t)base;
        for (int32_t i = 0; i < rows; ++i) p[i + 1] += p[i];
        base = p[rows];
    }
    plan.ent.resize(base);
    if (fmt == FMT_BF16) plan.v16.resize(base);
    if (fmt == FMT_F32) plan.v32.resize(base);
    if (fmt == FMT_F64) plan.v64.resize(base);
    parallel_chunks(count, 1, [&](int64_t k) {
        const int32_t q = (int32_t)k;
        if (!ok[q]) return;
        std::vector<int32_t> fill(S);
        for (int32_t i = inst_off[q]; i < inst_off[q + 1]; ++i) {
            for (int32_t s = 0; s < S; ++s) fill[s] = plan.bptr[(size_t)s * (rows + 1) + i];
            for (int32_t e = o.ptr[i]; e < o.ptr[i + 1]; ++e) {
                const int32_t pos = fill[slice_of(q, entry_index(o, fmt, e))]++;
                plan.ent[pos] = o.ent[e];
                if (fmt == FMT_BF16) plan.v16[pos] = o.v16[e];
                if (fmt == FMT_F32) plan.v32[pos] = o.v32[e];
                if (fmt == FMT_F64) plan.v64[pos] = o.v64[e];
            }
        }
    });
    for (int32_t q = 0; q < count; ++q) {
        if (!ok[q]) continue;
        const int64_t glen = gofs[q + 1] - gofs[q];
        const int32_t Sq = plan.Sq[q];
        for (int32_t s = 0; s < Sq; ++s)
            plan.max_slice = std::max<int32_t>(plan.max_slice, (int32_t)((glen * (s + 1)) / Sq - (glen * s) / Sq));
    }
}

void tile_sliced(const std::vector<int32_t> &inst_off, int32_t rows, int32_t sub_chunk, int32_t group_nnz,
                 SlicedPlan &plan)
{
    const int32_t count = (int32_t)inst_off.size() - 1;
    const int32_t S = plan.S;
    const std::vector<uint8_t> &ok = plan.sliced;
    plan.tiles.clear();
    plan.sub.clear();
    plan.ctiles.clear();
    if (S == 0) return;
    // sub-tiles per slice, grouped per (instance, slice)
    std::vector<uint8_t> skip(count);
    for (int32_t s = 0; s < S; ++s) {
        // instances with fewer slices have none here
        for (int32_t q = 0; q < count; ++q) skip[q] = (ok[q] && s < plan.Sq[q]) ? 0 : 1;
        std::vector<int32_t> ptr(plan.bptr.begin() + (size_t)s * (rows + 1),
                                 plan.bptr.begin() + (size_t)(s + 1) * (rows + 1));
        TilePlan tp;
        plan_tiles(ptr, inst_off, sub_chunk, 4 * 1024, tp, skip.data());
        const int32_t sub0 = (int32_t)(plan.sub.size() / 4);
        plan.sub.insert(plan.sub.end(), tp.tiles.begin(), tp.tiles.end());
        std::vector<int32_t> cuts;
        for (int32_t q = 0; q < count; ++q) {
            if (skip[q] || tp.t_end[q] == tp.t_begin[q]) continue;
            balanced_runs(tp.t_begin[q], tp.t_end[q], group_nnz, [&](int32_t t) {
                const int32_t *d = tp.tiles.data() + 4 * t;
                return (int64_t)(ptr[d[1]] - ptr[d[0]]);
            }, cuts);
            for (size_t c = 0; c + 1 < cuts.size(); ++c)
                plan.tiles.insert(plan.tiles.end(), {sub0 + cuts[c], sub0 + cuts[c + 1], q | (s << 24), -2});
        }
    }
    for (int32_t q = 0; q < count; ++q) {
        if (!ok[q]) continue;
        for (int32_t r = inst_off[q]; r < inst_off[q + 1]; r += 256)
            plan.ctiles.insert(plan.ctiles.end(), {r, std::min(r + 256, inst_off[q + 1]), q, -1});
    }
}

void plan_direct(const std::vector<int32_t> &ptr, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, int32_t max_vec, int32_t group_nnz, int32_t lanes_min,
                 int32_t per_lane, std::vector<uint8_t> &direct, std::vector<int32_t> &tiles)
{
    const int32_t count = (int32_t)inst_off.size() - 1;
    direct.assign(count, 0);
    tiles.clear();
    std::vector<int32_t> cuts;
    for (int32_t q = 0; q < count; ++q) {
        const int32_t r0 = inst_off[q], r1 = inst_off[q + 1];
        if (r1 == r0 || gofs[q + 1] - gofs[q] > max_vec) continue;
        direct[q] = 1;
        balanced_runs(r0, r1, group_nnz, [&](int32_t r) { return (int64_t)(ptr[r + 1] - ptr[r]); }, cuts);
        for (size_t c = 0; c + 1 < cuts.size(); ++c) {
            int32_t longest = 0;
            for (int32_t r = cuts[c]; r < cuts[c + 1]; ++r) longest = std::max(longest, ptr[r + 1] - ptr[r]);
            // lanes per row: enough that the longest row needs at most four
            // rounds of per_lane nonzeros per lane
            int32_t L = std::max(1, std::min(64, lanes_min));
            while (L < 64 && (int64_t)longest > 4LL * per_lane * L) L <<= 1;
            tiles.insert(tiles.end(), {cuts[c], cuts[c + 1], q, L});
        }
    }
}

void plan_sliced(const HostOrient &o, int32_t fmt, const std::vector<int32_t> &inst_off,
                 const std::vector<int32_t> &gofs, const std::vector<uint8_t> &candidate, int32_t max_vec,
                 int32_t max_slices, int32_t sub_chunk, int32_t group_nnz, SlicedPlan &plan)
{
    build_sliced(o, fmt, inst_off, gofs, candidate, max_vec, max_slices, sub_chunk, plan);
    tile_sliced(inst_off, o.rows, sub_chunk, group_nnz, plan);
}

}  // namespace scy
