// The pump loop of Algorithm 1 on a batch (scylla_batch_pump,
// scylla_batch_pump_ex): per round a batched warm-started solve, the device
// MIP-feasibility test of the iterate, host fix-and-propagate rounding on a
// thread pool, cycle detection and perturbation, and the objective update
// on the device (L1 distance: blend; L2 distance: QP objective).
#include "batch.h"

namespace {

// Integer flags [N] of the MIP-feasibility check (NULL: all integer).
void set_mip_isint(scylla_batch *h, const uint8_t *is_int)
{
    const size_t N = (size_t)std::max(h->N, 1);
    if (h->mip_isint.bytes < N) h->mip_isint.alloc(N);
    if (h->mip_rbad.bytes < (size_t)std::max(h->M, 1)) h->mip_rbad.alloc((size_t)std::max(h->M, 1));
    if (h->mip_cbad.bytes < N) h->mip_cbad.alloc(N);
    if (h->mip_ok.bytes < (size_t)h->count) h->mip_ok.alloc((size_t)h->count);
    std::vector<uint8_t> ii(N, 1);
    if (is_int)
        for (int32_t j = 0; j < h->N; ++j) ii[j] = is_int[j] ? 1 : 0;
    HIPC(hipMemcpyAsync(h->mip_isint.p, ii.data(), N, hipMemcpyHostToDevice, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
}

// MIP-feasibility of every instance's current x, on the device (integer
// flags from set_mip_isint); ok: [count] 1 / 0.
void mip_check(scylla_batch *h, double tol, uint8_t *ok)
{
    const OrientRT &o = h->orow;
    if (h->vbytes == 4)
        launch_mip_check<float>(o.mat, h->fmt, h->M, h->N, h->count, h->info.as<InstInfo>(), h->x.as<float>(),
                                h->b64.as<double>(), h->sense.as<uint8_t>(), h->l64.as<double>(),
                                h->u64.as<double>(), h->mip_isint.as<uint8_t>(), tol, h->mip_rbad.as<uint8_t>(),
                                h->mip_cbad.as<uint8_t>(), h->mip_ok.as<uint8_t>(), h->stream);
    else
        launch_mip_check<double>(o.mat, h->fmt, h->M, h->N, h->count, h->info.as<InstInfo>(), h->x.as<double>(),
                                 h->b64.as<double>(), h->sense.as<uint8_t>(), h->l64.as<double>(),
                                 h->u64.as<double>(), h->mip_isint.as<uint8_t>(), tol, h->mip_rbad.as<uint8_t>(),
                                 h->mip_cbad.as<uint8_t>(), h->mip_ok.as<uint8_t>(), h->stream);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(ok, h->mip_ok.p, (size_t)h->count, hipMemcpyDeviceToHost, h->stream));
    HIPC(hipStreamSynchronize(h->stream));
}

void build_locals(scylla_batch *h)
{
    if (!h->local.empty()) return;
    h->local.resize(h->count);
    const OrientRT &o = h->orow;
    for (int32_t q = 0; q < h->count; ++q) {
        auto &L = h->local[q];
        const int32_t r0 = h->row_off[q], r1 = h->row_off[q + 1], c0 = h->col_off[q];
        const int32_t e0 = o.host.ptr[r0];
        L.ptr.resize(r1 - r0 + 1);
        for (int32_t i = r0; i <= r1; ++i) L.ptr[i - r0] = o.host.ptr[i] - e0;
        const int32_t nnz = o.host.ptr[r1] - e0;
        L.col.resize(nnz);
        for (int32_t e = 0; e < nnz; ++e) {
            const uint32_t w = o.host.ent[e0 + e];
            L.col[e] = (int32_t)(h->fmt == FMT_PACKED ? (w & o.host.mask) : w) - c0;
        }
        FPProblem &P = L.P;
        P.m = r1 - r0;
        P.n = h->col_off[q + 1] - c0;
        P.ptr = L.ptr.data();
        P.col = L.col.data();
        P.val = h->hval.data() + e0;
        P.b = h->hb.data() + r0;
        P.sense = h->hsense.data() + r0;
        P.l = h->hl.data() + c0;
        P.u = h->hu.data() + c0;
        build_incidence(P, L.cptr, L.crow, L.cval);
    }
}

template <class F>
void parallel_for(int32_t count, int32_t threads, F &&f)
{
    int32_t nt = threads > 0 ? threads : (int32_t)std::max(1u, std::thread::hardware_concurrency());
    nt = std::max(1, std::min(nt, count));
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
        for (int32_t q = next++; q < count; q = next++) f(q);
    };
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

void reset_objective(scylla_batch *h)
{
    if (h->has_q) {
        HIPC(hipMemsetAsync(h->q64.p, 0, h->q64.bytes, h->stream));
        HIPC(hipMemsetAsync(h->qv.p, 0, h->qv.bytes, h->stream));
    }
    HIPC(hipMemcpyAsync(h->c64.p, h->corig64.p, sizeof(double) * h->N, hipMemcpyDeviceToDevice, h->stream));
    if (h->vbytes == 4) launch_cast<float>(h->c64.as<double>(), h->cv.as<float>(), h->N, h->stream);
    else launch_cast<double>(h->c64.as<double>(), h->cv.as<double>(), h->N, h->stream);
    launch_inst_norms(h->info.as<InstInfo>(), h->count, h->b64.as<double>(), h->c64.as<double>(),
                      h->dr64.as<double>(), h->dc64.as<double>(), h->st.as<InstState>(), h->stream);
    HIPC(hipGetLastError());
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a counter-based
// generator: the output function applied to the state seed + (counter + 1) *
// the golden-ratio increment.
uint64_t splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Number of binaries the K-th perturbation of instance q flips, in [10, 30].
int32_t perturb_count(uint64_t seed, int32_t q, int32_t K)
{
    return 10 + (int32_t)(splitmix64(seed, (uint64_t)q * 1048576ull + (uint64_t)K) % 21ull);
}

// Per-instance history of roundings for cycle detection: value hashes first,
// then exact comparison (0.0 and -0.0 compare equal).
struct RoundingHistory {
    std::vector<uint64_t> hash;
    std::vector<std::vector<double>> pts;

    static uint64_t digest(const double *x, int32_t n)
    {
        uint64_t hsh = 1469598103934665603ull;
        for (int32_t j = 0; j < n; ++j) {
            double v = x[j] + 0.0;
            uint64_t w;
            memcpy(&w, &v, 8);
            hsh = (hsh ^ w) * 1099511628211ull;
        }
        return hsh;
    }
    bool seen(const double *x, int32_t n) const
    {
        const uint64_t d = digest(x, n);
        for (size_t k = 0; k < pts.size(); ++k) {
            if (hash[k] != d) continue;
            bool eq = true;
            for (int32_t j = 0; j < n && eq; ++j) eq = pts[k][j] == x[j];
            if (eq) return true;
        }
        return false;
    }
    void add(const double *x, int32_t n)
    {
        hash.push_back(digest(x, n));
        pts.emplace_back(x, x + n);
    }
};

struct PumpOpts {
    int32_t rounds;
    bool eps_sched;
    double eps1, beta, eps_floor, alpha;
    int64_t total_iter_limit;
    bool early_exit, perturb;
    uint64_t seed;
    int32_t threads;
    int32_t distance;  // 1: L1 (linear objective), 2: L2 (QP objective)
    bool pipeline;     // two instance groups: host rounding overlaps device solves
    int32_t fp_batch = 0;        // 0: sequential rounding on the host; K: batched on the device
    int32_t fp_max_rounds = 1000;
};

// Algorithm 1 outer loop.  legacy_best: also keep, per instance, the first
// feasible rounding else the last one (scylla_batch_pump's output).
int pump_impl(scylla_batch *h, const scylla_params *p, const uint8_t *is_int, const PumpOpts &o,
              scylla_pump_record *rec, scylla_pump_outcome *outc, double *x_out, bool legacy_best)
{
    if (!h) throw_err(-EINVAL, "handle is NULL");
    if (o.rounds < 1) throw_err(-EINVAL, "rounds must be >= 1");
    if (!(o.alpha >= 0.0 && o.alpha < 1.0)) throw_err(-EINVAL, "alpha must be in [0, 1)");
    if (o.eps_sched && !(o.eps1 > 0.0 && o.beta > 0.0 && o.beta <= 1.0 && o.eps_floor > 0.0))
        throw_err(-EINVAL, "eps schedule needs eps1 > 0, 0 < beta <= 1, eps_floor > 0");
    if (o.total_iter_limit < 0) throw_err(-EINVAL, "total_iter_limit must be >= 0");
    if (o.distance != 1 && o.distance != 2) throw_err(-EINVAL, "distance must be 1 (L1) or 2 (L2)");
    if (o.fp_batch < 0) throw_err(-EINVAL, "fp_batch must be >= 0");
    if (o.fp_batch > 0 && o.fp_max_rounds < 1) throw_err(-EINVAL, "fp_max_rounds must be >= 1");
    if (o.fp_batch > 0 && o.pipeline) throw_err(-EINVAL, "device rounding (fp_batch > 0) needs pipeline = 0");
    validate_params(p);
    build_locals(h);
    const bool l2 = o.distance == 2;
    if (l2) ensure_q(h);
    const int32_t N = h->N, count = h->count;
    std::vector<uint8_t> isint(N, 1);
    if (is_int)
        for (int32_t j = 0; j < N; ++j) isint[j] = is_int[j] ? 1 : 0;
    // kappa_q = sqrt(|I_q|) / ||c_q|| (0 when c = 0: the term is dropped)
    std::vector<double> kappa(count, 0.0);
    std::vector<size_t> boff(count + 1, 0);
    for (int32_t q = 0; q < count; ++q) {
        double cn = 0.0;
        int64_t nI = 0;
        for (int32_t j = h->col_off[q]; j < h->col_off[q + 1]; ++j) {
            cn += h->hc[j] * h->hc[j];
            nI += isint[j];
        }
        kappa[q] = cn > 0.0 ? sqrt((double)nI) / sqrt(cn) : 0.0;
        boff[q + 1] = boff[q] + (size_t)(h->col_off[q + 1] - h->col_off[q] + 7) / 8;
    }
    std::vector<uint8_t> xbits(boff[count]), ibits(boff[count]);
    for (int32_t q = 0; q < count; ++q)
        for (int32_t j = h->col_off[q]; j < h->col_off[q + 1]; ++j) {
            const int32_t k = j - h->col_off[q];
            if (isint[j]) ibits[boff[q] + k / 8] |= (uint8_t)(1u << (k % 8));
        }
    if (h->bits_tmp.bytes < boff[count]) h->bits_tmp.alloc(boff[count]);
    if (h->ibits_tmp.bytes < boff[count]) h->ibits_tmp.alloc(boff[count]);
    HIPC(hipMemcpyAsync(h->ibits_tmp.p, ibits.data(), boff[count], hipMemcpyHostToDevice, h->stream));
    set_mip_isint(h, isint.data());
    reset_objective(h);
    HIPC(hipStreamSynchronize(h->stream));

    std::vector<double> xhat(N), xres(N, 0.0);
    std::vector<double> dev_xhat(o.fp_batch > 0 ? N : 0);  // device roundings of a round
    std::vector<int32_t> dev_info(o.fp_batch > 0 ? 2 * (size_t)count : 0);
    std::vector<double> chat, qhat;  // L2: next objective and Hessian
    if (l2) {
        chat = h->hc;
        qhat.assign(N, 0.0);
    }
    if (legacy_best) h->pump_best.assign(N, 0.0);
    std::vector<uint8_t> found_best(count, 0), active(count, 1);
    std::vector<scylla_pump_outcome> out(count);
    memset(out.data(), 0, sizeof(scylla_pump_outcome) * count);
    std::vector<RoundingHistory> hist(o.perturb ? count : 0);
    std::vector<FPPrep> prep(count);  // per-instance rounding state, built on first use
    if (rec) memset(rec, 0, sizeof(scylla_pump_record) * (size_t)o.rounds * count);
    std::vector<double> eps_k(o.rounds + 1, o.eps1);  // tolerance of round K (schedule)
    for (int32_t K = 2; K <= o.rounds; ++K) eps_k[K] = std::max(o.beta * eps_k[K - 1], o.eps_floor);

    // Instances run in one group, or in two groups of contiguous instances
    // (split at half the nonzeros) whose rounds alternate on the device: the
    // host rounds one group while the device solves the other.  Every
    // instance sees the same sequence of solves, roundings and objective
    // updates either way (a batched solve equals solves of its instances).
    struct Group {
        int32_t q0 = 0, q1 = 0, K = 1;
        std::vector<double> x;                // iterate copied out after the solve
        std::vector<uint8_t> ok;              // device MIP-feasibility flags
        std::vector<scylla_result> res;
        std::vector<int64_t> limits;
        double solve_s = 0.0, rounding_s = 0.0;
    };
    const int ng = (o.pipeline && count >= 2) ? 2 : 1;
    Group G[2];
    {
        int32_t mid = count;
        if (ng == 2) {
            const int64_t total = h->orow.host.ptr[h->M];
            mid = 1;
            while (mid < count - 1 && (int64_t)h->orow.host.ptr[h->row_off[mid]] * 2 < total) ++mid;
        }
        G[0].q0 = 0;
        G[0].q1 = mid;
        G[1].q0 = mid;
        G[1].q1 = count;
        for (int g = 0; g < ng; ++g) {
            G[g].x.assign(N, 0.0);
            G[g].ok.assign(count, 0);
            G[g].res.resize(count);
            G[g].limits.assign(count, 0);
        }
    }

    // Solves round G.K of a group; false when it has nothing left to solve.
    auto solve_group = [&](Group &g) -> bool {
        if (g.K > o.rounds) return false;
        int32_t n_active = 0;
        for (int32_t q = 0; q < count; ++q) g.limits[q] = 0;
        for (int32_t q = g.q0; q < g.q1; ++q) {
            int64_t lim = p->iter_limit;
            if (o.total_iter_limit > 0) lim = std::min(lim, o.total_iter_limit - out[q].iterations);
            if (active[q] && lim <= 0) active[q] = 0;
            g.limits[q] = active[q] ? lim : 0;
            n_active += active[q];
        }
        if (n_active == 0) return false;
        const double t0 = now_s();
        scylla_params pk = *p;
        if (o.eps_sched) pk.tol = eps_k[g.K];
        batch_solve_impl(h, &pk, g.K > 1 ? 1 : 0, g.res.data(), g.limits.data(), g.q0, g.q1);
        mip_check(h, 1e-6, g.ok.data());
        if (h->vbytes == 4) get_range<float>(h, h->x, 0, N, g.x.data());
        else get_range<double>(h, h->x, 0, N, g.x.data());
        g.solve_s = now_s() - t0;
        return true;
    };

    // Host rounding of round G.K of a group (Algorithm 1 after the solve).
    auto round_group = [&](Group &g) {
        const int32_t K = g.K;
        std::atomic<int> bad{0}, nonbinary{0};
        const double tr0 = now_s();
        if (o.fp_batch > 0) {  // all roundings of the group at once on the device
            std::vector<uint8_t> want(count, 0);
            for (int32_t q = g.q0; q < g.q1; ++q) want[q] = active[q] && g.res[q].status != SCYLLA_NUMERICAL_ERROR;
            fp_batched(h, isint.data(), nullptr, o.fp_batch, o.fp_max_rounds, want.data(), dev_xhat.data(),
                       dev_info.data(), nullptr);
        }
        parallel_for(g.q1 - g.q0, o.threads, [&](int32_t qi) {
            const int32_t q = g.q0 + qi;
            if (!active[q]) return;
            const auto &P = h->local[q].P;
            const int32_t c0 = h->col_off[q];
            const uint8_t *ii = isint.data() + c0;
            const double *xq = g.x.data() + c0;
            double *xh = xhat.data() + c0;
            scylla_pump_outcome &oc = out[q];
            oc.rounds_run = K;
            oc.iterations += g.res[q].iterations;
            scylla_pump_record rtmp;
            scylla_pump_record &r = rec ? rec[(size_t)(K - 1) * count + q] : rtmp;
            memset(&r, 0, sizeof(r));
            r.round = K;
            r.group = (int32_t)(&g - G);
            r.status = g.res[q].status;
            r.iterations = g.res[q].iterations;
            r.rel_kkt = g.res[q].rel_kkt;
            r.solve_seconds = g.res[q].solve_seconds;
            r.tune_seconds = g.res[q].tune_seconds;
            if (g.res[q].status == SCYLLA_NUMERICAL_ERROR) {
                // no usable iterate: the instance leaves the loop unrounded
                active[q] = 0;
                return;
            }
            r.lp_feasible = g.ok[q];
            if (r.lp_feasible && !oc.found_kind) {
                oc.found_kind = 1;
                oc.found_round = K;
                memcpy(xres.data() + c0, xq, sizeof(double) * P.n);
                if (o.early_exit) {
                    active[q] = 0;
                    return;
                }
            }
            if (o.fp_batch > 0) {
                memcpy(xh, dev_xhat.data() + c0, sizeof(double) * P.n);
                r.xhat_feasible = dev_info[2 * q];
                r.ignored_rows = dev_info[2 * q + 1];
            } else {
                if (!prep[q].ready) fp_prepare(P, ii, prep[q]);
                fix_and_propagate(P, ii, prep[q], xq, xh, &r.xhat_feasible, &r.ignored_rows);
            }
            double obj = 0.0;
            for (int32_t j = 0; j < P.n; ++j) obj += h->hc[c0 + j] * xh[j];
            r.xhat_obj = obj;
            if (legacy_best && !found_best[q]) {
                memcpy(h->pump_best.data() + c0, xh, sizeof(double) * P.n);
                if (r.xhat_feasible) found_best[q] = 1;
            }
            if (!oc.found_kind) memcpy(xres.data() + c0, xh, sizeof(double) * P.n);
            if (r.xhat_feasible && !oc.found_kind) {
                oc.found_kind = 2;
                oc.found_round = K;
                if (o.early_exit) {
                    active[q] = 0;
                    return;
                }
            }
            if (o.perturb) {
                if (hist[q].seen(xh, P.n)) {
                    // flip the T binaries farthest from the PDHG iterate
                    std::vector<int32_t> idx;
                    for (int32_t j = 0; j < P.n; ++j)
                        if (ii[j]) {
                            if (P.u[j] - P.l[j] != 1.0) nonbinary = 1;
                            idx.push_back(j);
                        }
                    if (!nonbinary) {
                        const size_t T = std::min<size_t>((size_t)perturb_count(o.seed, q, K), idx.size());
                        std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
                            return fabs(xq[a] - xh[a]) > fabs(xq[b] - xh[b]);
                        });
                        for (size_t t = 0; t < T; ++t) {
                            const int32_t j = idx[t];
                            xh[j] = xh[j] == P.l[j] ? P.u[j] : P.l[j];
                        }
                        r.perturbed = 1;
                        ++oc.perturbations;
                    }
                }
                hist[q].add(xh, P.n);
            }
            if (l2) {
                // L2 distance (Section 5): QP objective a kappa c - 2 (1 - a) x_hat
                // and Hessian 2 (1 - a) on the integer variables
                const double a = pow(o.alpha, (double)K);
                for (int32_t j = 0; j < P.n; ++j) {
                    chat[c0 + j] = a * kappa[q] * h->hc[c0 + j] - (ii[j] ? 2.0 * (1.0 - a) * xh[j] : 0.0);
                    qhat[c0 + j] = ii[j] ? 2.0 * (1.0 - a) : 0.0;
                }
                return;
            }
            // L1-distance gradient needs every integer at a bound
            uint8_t *xb = xbits.data() + boff[q];
            memset(xb, 0, boff[q + 1] - boff[q]);
            for (int32_t j = 0; j < P.n; ++j) {
                if (!ii[j]) continue;
                if (xh[j] == P.u[j] && xh[j] != P.l[j]) xb[j / 8] |= (uint8_t)(1u << (j % 8));
                else if (xh[j] != P.l[j]) bad = 1;
            }
        });
        g.rounding_s = now_s() - tr0;
        if (nonbinary) throw_err(-EINVAL, "cycle perturbation needs binary integer variables");
        if (bad) throw_err(-EINVAL, "an integer variable is rounded strictly inside its bounds: the L1 distance "
                                    "of general integers needs auxiliary variables");
    };

    // Next objective of the group's active instances on the device, then the
    // group's round is complete.
    auto finish_group = [&](Group &g) {
        const double tb = now_s();
        bool any = false;
        for (int32_t q = g.q0; q < g.q1; ++q) any = any || active[q];
        const int32_t c0 = h->col_off[g.q0], c1 = h->col_off[g.q1];
        if (g.K < o.rounds && any && l2) {
            HIPC(hipMemcpyAsync(h->c64.as<double>() + c0, chat.data() + c0, sizeof(double) * (c1 - c0),
                                hipMemcpyHostToDevice, h->stream));
            HIPC(hipMemcpyAsync(h->q64.as<double>() + c0, qhat.data() + c0, sizeof(double) * (c1 - c0),
                                hipMemcpyHostToDevice, h->stream));
            if (h->vbytes == 4) launch_cast<float>(h->c64.as<double>() + c0, h->cv.as<float>() + c0, c1 - c0, h->stream);
            else launch_cast<double>(h->c64.as<double>() + c0, h->cv.as<double>() + c0, c1 - c0, h->stream);
            cast_q(h);
        } else if (g.K < o.rounds && any) {
            const double a = pow(o.alpha, (double)g.K);
            const size_t b0 = boff[g.q0], b1 = boff[g.q1];
            HIPC(hipMemcpyAsync(h->bits_tmp.as<uint8_t>() + b0, xbits.data() + b0, b1 - b0, hipMemcpyHostToDevice,
                                h->stream));
            for (int32_t q = g.q0; q < g.q1; ++q) {
                if (!active[q]) continue;
                const int lo = h->col_off[q], hi = h->col_off[q + 1];
                const uint8_t *xb = h->bits_tmp.as<uint8_t>() + boff[q];
                const uint8_t *ib = h->ibits_tmp.as<uint8_t>() + boff[q];
                if (h->vbytes == 4)
                    launch_blend<float>(h->corig64.as<double>(), xb, ib, a, kappa[q], h->c64.as<double>(),
                                        h->cv.as<float>(), lo, hi, h->stream);
                else
                    launch_blend<double>(h->corig64.as<double>(), xb, ib, a, kappa[q], h->c64.as<double>(),
                                         h->cv.as<double>(), lo, hi, h->stream);
            }
        }
        if (g.K < o.rounds && any) {
            launch_inst_norms(h->info.as<InstInfo>(), h->count, h->b64.as<double>(), h->c64.as<double>(),
                              h->dr64.as<double>(), h->dc64.as<double>(), h->st.as<InstState>(), h->stream);
            HIPC(hipGetLastError());
            HIPC(hipStreamSynchronize(h->stream));
        }
        const double dt = g.solve_s + g.rounding_s + (now_s() - tb);
        if (rec)
            for (int32_t q = g.q0; q < g.q1; ++q) {
                scylla_pump_record &r = rec[(size_t)(g.K - 1) * count + q];
                if (r.round) {
                    r.round_seconds = dt;
                    r.rounding_seconds = g.rounding_s;
                }
            }
        ++g.K;
    };

    if (ng == 1) {
        while (solve_group(G[0])) {
            round_group(G[0]);
            finish_group(G[0]);
        }
    } else {
        // pending: the group whose solve awaits its rounding
        bool has[2] = {solve_group(G[0]), false};
        int r = 0;
        for (;;) {
            const int sg = 1 - r;
            std::exception_ptr err;
            std::thread worker;
            if (has[r])
                worker = std::thread([&]() {
                    try {
                        round_group(G[r]);
                    } catch (...) {
                        err = std::current_exception();
                    }
                });
            try {
                has[sg] = solve_group(G[sg]);
            } catch (...) {
                if (worker.joinable()) worker.join();
                throw;
            }
            if (worker.joinable()) worker.join();
            if (err) std::rethrow_exception(err);
            if (has[r]) finish_group(G[r]);
            if (!has[r] && !has[sg]) break;
            has[r] = false;
            r = sg;
        }
    }
    for (int32_t q = 0; q < count; ++q) {
        double obj = 0.0;
        for (int32_t j = h->col_off[q]; j < h->col_off[q + 1]; ++j) obj += h->hc[j] * xres[j];
        out[q].obj = obj;
    }
    if (outc) memcpy(outc, out.data(), sizeof(scylla_pump_outcome) * count);
    if (x_out) memcpy(x_out, xres.data(), sizeof(double) * N);
    return 0;
}

// ------------------------------------------------ allocation-free MIP test
// Device scratch of scylla_batch_mip_feasible_static: integer flags [N], row
// flags [M], column flags [N] and instance flags [count], each region at a
// 256-byte aligned offset.  Each GPU holds its own copy for the life of the
// process; every call on a GPU reuses it (each call overwrites every flag it
// reads, so nothing has to start at zero), so calls that overlap on one GPU
// race.
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_dev[kMaxDevices] = {};

// Device address of the current GPU's scratch, looked up once per device
// with that device current (in host code `scratch` names a host-side
// stand-in, not device memory).
uint8_t *static_scratch()
{
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw_err(-ENODEV, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        HIPC(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw_err(-EIO, "no device address for the static scratch");
        g_scratch_dev[dev] = static_cast<uint8_t *>(ptr);
    }
    return g_scratch_dev[dev];
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The MIP-feasibility test of mip_check with its flags in `scr` (layout
// above); ok goes to the first count bytes of `out`.
template <class V>
void mip_check_into(scylla_batch *h, const uint8_t *isint, double tol, uint8_t *rbad, uint8_t *cbad, uint8_t *ok)
{
    launch_mip_check<V>(h->orow.mat, h->fmt, h->M, h->N, h->count, h->info.as<InstInfo>(), h->x.as<V>(),
                        h->b64.as<double>(), h->sense.as<uint8_t>(), h->l64.as<double>(), h->u64.as<double>(),
                        isint, tol, rbad, cbad, ok, h->stream);
    HIPC(hipGetLastError());
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int scylla_fix_propagate(const scylla_lp *lp, const uint8_t *is_int, const double *x_ref, double *x_hat,
                         int32_t *info)
{
    return guarded([&]() {
        std::string err;
        int rc = validate_lp(lp, err);
        if (rc) throw_err(rc, err);
        if (!x_ref || !x_hat || !info) throw_err(-EINVAL, "NULL argument");
        const scylla_csr &A = lp->A;
        for (int32_t j = 0; j < A.n; ++j)
            if (!isfinite(x_ref[j])) throw_err(-EINVAL, "non-finite reference value");
        std::vector<int32_t> ptr(A.m + 1), cptr, crow;
        std::vector<double> cval;
        for (int32_t i = 0; i <= A.m; ++i) ptr[i] = (int32_t)A.row_ptr[i];
        FPProblem P;
        P.m = A.m;
        P.n = A.n;
        P.ptr = ptr.data();
        P.col = A.col_idx;
        P.val = A.val;
        P.b = lp->b;
        P.sense = lp->senses;
        P.l = lp->l;
        P.u = lp->u;
        build_incidence(P, cptr, crow, cval);
        std::vector<uint8_t> ii(A.n, 1);
        if (is_int)
            for (int32_t j = 0; j < A.n; ++j) ii[j] = is_int[j] ? 1 : 0;
        FPPrep prep;
        fp_prepare(P, ii.data(), prep);
        fix_and_propagate(P, ii.data(), prep, x_ref, x_hat, &info[0], &info[1]);
        return 0;
    });
}

int scylla_batch_mip_feasible(scylla_batch *h, const uint8_t *is_int, double tol, int32_t *feasible)
{
    return guarded([&]() {
        if (!h || !feasible) throw_err(-EINVAL, "handle or feasible is NULL");
        if (!(tol > 0.0) || !isfinite(tol)) throw_err(-EINVAL, "tol must be finite and > 0");
        set_mip_isint(h, is_int);
        std::vector<uint8_t> ok(h->count);
        mip_check(h, tol, ok.data());
        for (int32_t q = 0; q < h->count; ++q) feasible[q] = ok[q];
        return 0;
    });
}

int scylla_batch_mip_feasible_static(scylla_batch *h, const uint8_t *is_int, double tol, int32_t *feasible)
{
    return guarded([&]() {
        if (!h || !feasible) throw_err(-EINVAL, "handle or feasible is NULL");
        if (!(tol > 0.0) || !isfinite(tol)) throw_err(-EINVAL, "tol must be finite and > 0");
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t N = (size_t)std::max(h->N, 1), M = (size_t)std::max(h->M, 1);
        const size_t o_rbad = al(N), o_cbad = o_rbad + al(M), o_ok = o_cbad + al(N);
        const size_t need = o_ok + al((size_t)std::max(h->count, 1));
        if (need > kStaticScratchBytes)
            throw_err(-EINVAL, "the batch needs " + std::to_string(need) + " bytes of flags, more than the " +
                                   std::to_string(kStaticScratchBytes) + "-byte static scratch");
        uint8_t *s = static_scratch();
        uint8_t *isint = s, *rbad = s + o_rbad, *cbad = s + o_cbad, *ok = s + o_ok;
        if (h->N > 0) {
            if (is_int)  // nonzero = integer, as the kernel reads it
                HIPC(hipMemcpyAsync(isint, is_int, (size_t)h->N, hipMemcpyHostToDevice, h->stream));
            else
                hipLaunchKernelGGL(k_fill_u8, dim3((h->N + 255) / 256), dim3(256), 0, h->stream, isint,
                                   (uint8_t)1, h->N);
        }
        if (h->vbytes == 4) mip_check_into<float>(h, isint, tol, rbad, cbad, ok);
        else mip_check_into<double>(h, isint, tol, rbad, cbad, ok);
        // the flags land in the first count bytes of the caller's int32
        // array and are widened in place from the last one down (byte q
        // sits at or below int q, so nothing unread is overwritten)
        if (h->count > 0)
            HIPC(hipMemcpyAsync(feasible, ok, (size_t)h->count, hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
        const uint8_t *bytes = reinterpret_cast<const uint8_t *>(feasible);
        for (int32_t q = h->count - 1; q >= 0; --q) feasible[q] = bytes[q];
        return 0;
    });
}

int scylla_batch_pump(scylla_batch *h, const scylla_params *p, const uint8_t *is_int, int32_t rounds,
                      double alpha, int32_t threads, scylla_pump_record *records, double *xhat_out)
{
    return guarded([&]() {
        PumpOpts o{rounds, false, 0.0, 0.0, 0.0, alpha, 0, false, false, 0, threads, 1, false};
        pump_impl(h, p, is_int, o, records, nullptr, nullptr, true);
        if (xhat_out) memcpy(xhat_out, h->pump_best.data(), sizeof(double) * h->N);
        return 0;
    });
}

int scylla_pump_params_default(scylla_pump_params *o)
{
    if (!o) {
        g_err = "pump params is NULL";
        return -EINVAL;
    }
    memset(o, 0, sizeof(*o));
    o->rounds = 20;
    o->eps_schedule = 1;
    o->eps1 = 0.01;
    o->beta = 0.98;
    o->eps_floor = 1e-8;
    o->alpha = 0.9;
    o->total_iter_limit = 0;
    o->early_exit = 1;
    o->perturb = 1;
    o->seed = 0;
    o->threads = 0;
    o->distance = 1;
    o->pipeline = 0;
    o->fp_batch = 0;
    o->fp_max_rounds = 1000;
    return 0;
}

int scylla_batch_pump_ex(scylla_batch *h, const scylla_params *params, const uint8_t *is_int,
                         const scylla_pump_params *opt, scylla_pump_record *records,
                         scylla_pump_outcome *outcome, double *x_out)
{
    return guarded([&]() {
        if (!opt) throw_err(-EINVAL, "pump params is NULL");
        PumpOpts o{opt->rounds,    opt->eps_schedule != 0, opt->eps1,         opt->beta,
                   opt->eps_floor, opt->alpha,             opt->total_iter_limit, opt->early_exit != 0,
                   opt->perturb != 0, opt->seed, opt->threads, opt->distance, opt->pipeline != 0,
                   opt->fp_batch, opt->fp_max_rounds};
        return pump_impl(h, params, is_int, o, records, outcome, x_out, false);
    });
}

}  // extern "C"
