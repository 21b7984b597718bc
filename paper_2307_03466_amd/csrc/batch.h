// The library's handle (struct scylla_batch: a device-resident batch of LPs)
// and what the solver runtime (runtime.hip) and the pump loop (pump.hip)
// share: error plumbing, owned device memory, the matrix orientations, and
// the functions one file exports to the other.
#pragma once
#include <errno.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include <atomic>
#include <cstdlib>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>
#include <thread>

#include "fixprop.h"
#include "kernels.h"
#include "scylla_internal.h"

namespace scy {

extern thread_local std::string g_err;

struct Err {
    int code;
    std::string msg;
};

[[noreturn]] inline void throw_err(int code, const std::string &msg) { throw Err{code, msg}; }

inline void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        const int code = (e == hipErrorOutOfMemory) ? -ENOMEM : -EIO;
        throw_err(code, std::string(what) + ": " + hipGetErrorString(e));
    }
}
#define HIPC(x) hip_check((x), #x)

inline double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Owned device allocation.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b)
    {
        release();
        bytes = b;
        HIPC(hipMalloc(&p, b > 0 ? b : 16));
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

template <class T>
void upload(DevMem &d, const std::vector<T> &h, hipStream_t s)
{
    d.alloc(h.size() * sizeof(T));
    if (!h.empty()) HIPC(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

}  // namespace scy

using namespace scy;

// One orientation of the matrix on the device: the CSR (row pass, dual
// step) or the CSC copy (column pass, primal step), in its normal layout or
// its gather-blocked layout, with the tile plan in use and its buffers.
struct OrientRT {
    bool row = true;
    int32_t rows = 0, gather = 0;
    bool cached = false;  // iteration passes read the matrix with plain loads
    HostOrient host;  // normal layout (host copy kept for re-planning)
    DevMem ptr, ent, val;
    MatView mat{};
    TilePlan plan;
    int32_t ept = 8;
    // gather-blocked layout (when chosen)
    bool blocked = false;
    BlockedHost bh;  // host copy of the block pointers (entries dropped after upload)
    DevMem bptr, bent, bval;
    MatView bmat{};
    BlockedPlan bplan;
    DevMem P, P64, ctiles;
    // LDS-staged layout (when chosen): staged tiles for instances whose
    // gathered vector fits in LDS, normal tiles for the rest
    bool staged = false;
    StagedPlan splan;
    DevMem stiles, subtiles, gofs, rtiles, rlongs, rseg;
    size_t shmem = 0;
    int32_t staged_nnz = 0;
    int32_t svariant = 0;
    // LDS-sliced instances of the staged layout (when enabled): the regrouped
    // entries are kept for the (max_vec, sub-tile) they were built for
    bool sliced = false;
    bool shalf = false;   // half-LDS budget per workgroup
    int32_t nstiles = 0;  // staged + sliced tiles
    SlicedPlan xplan;
    int32_t x_max_vec = -1, x_sub = -1;
    DevMem xptr, xent, xval, xsub, xctiles, xP, xsq;
    std::vector<int32_t> stiles_h;  // host copy of stiles
    // direct staged layout (when chosen): the whole gathered vector of each
    // qualifying instance in LDS, rows reduced in registers; normal tiles
    // (splan.rest) for the other instances
    bool direct = false;
    std::vector<uint8_t> dinst;
    std::vector<int32_t> dtiles_h;
    DevMem dtiles;
    int32_t dnnz = 0, dlanes = 1;
    size_t dshmem = 0;
    // plan buffers
    DevMem tiles, longs, seg, seg64, part, lpart;
    DevMem part2, lpart2;  // check partials of the running average
    // adaptive-step partials: 2 doubles per epilogue slot; slot spaces of the
    // launches of the active layout start at these offsets
    DevMem ipart;
    int32_t ipo_long = 0, ipo_comb = 0, ipo_rest = 0, ipo_rlong = 0, ip_slots = 0;
    // compacted tile lists of the iteration launches (the tiles of running
    // instances only, in the original order; the check launches keep the
    // full lists) and the epilogue slot offsets that go with them
    bool cmp = false;
    DevMem c_tiles, c_stiles, c_xctiles, c_rtiles, c_dtiles;
    std::vector<int32_t> c_tiles_h, c_stiles_h, c_xctiles_h, c_rtiles_h, c_dtiles_h;
    int32_t cipo_long = 0, cipo_comb = 0, cipo_rest = 0, cipo_rlong = 0;
    int32_t ntiles() const { return (int32_t)((blocked ? bplan.tiles.size() : plan.tiles.size()) / 4); }
    int32_t nlong() const { return (int32_t)((blocked ? bplan.longs.size() : plan.longs.size()) / 4); }
};

// Device copy of the problem and work arrays of the batched
// fix-and-propagate (built on its first call).
struct FPDev {
    bool ready = false;
    DevMem rptr, col, val, cptr, crow, rowoff, coloff;  // FP64 CSR + column incidence
    DevMem nint, isint, want, xbar, key, key2, ord0, ord, tmp;
    DevMem L, U, cL, cU, vst, rst, ign, bad, act, nxt, chg, xhat, info;
    size_t tmp_bytes = 0;
};

struct scylla_batch {
    int32_t count = 0, precision = SCYLLA_FP32, fmt = FMT_PACKED;
    int32_t vbytes = 4;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap = nullptr;  // private stream used for graph capture
    hipStream_t side = nullptr; // second branch (staged and normal tiles overlap)
    hipEvent_t fork = nullptr, join = nullptr;
    int32_t M = 0, N = 0;
    int64_t NNZ = 0;
    std::vector<int32_t> row_off, col_off;
    OrientRT orow, ocol;
    // vectors in the path precision
    DevMem x, xbar, xr, y, yr, cv, lv, uv, dc2, b_v, dr2;
    DevMem sense;
    // FP64 data
    DevMem c64, corig64, l64, u64, b64, dr64, dc64;
    DevMem st, info;
    DevMem ax;              // running A x of the row pass (adaptive steps)
    DevMem ibnd;            // [2 * count] (l, u) shared by all columns of an
                            // instance, NaN where they differ
    DevMem start_flag;      // validation flag of a device warm start
    DevMem q64, qv;         // diagonal Hessian (QP objectives), once set
    DevMem xp, yp, axp, atyp;  // previous check's point and products
    bool has_q = false;
    bool adaptive = false;  // adaptive step sizes in the current graph
    bool avg_on = false;    // restart to the average in the current graph
    DevMem xavg, yavg, axavg;  // running means of x, y (and A x, adaptive)
    DevMem bits_tmp, ibits_tmp;
    DevMem mip_isint, mip_rbad, mip_cbad, mip_ok;  // MIP-feasibility check
    // graph
    hipGraphExec_t gexec = nullptr;
    // window graph over the compacted tile lists, and earlier ones of the
    // same solve (destroyed once the stream has drained)
    hipGraphExec_t cexec = nullptr;
    std::vector<hipGraphExec_t> retired;
    int64_t graph_tiles = 0;          // tiles of the current graph's iteration launches
    std::vector<InstInfo> hinfo_c;    // instance info with the compacted slot ranges
    void *cstage = nullptr;           // pinned staging of the cut lists
    size_t cstage_bytes = 0;
    int32_t graph_R = 0;
    bool tuned = false;
    int32_t lds_max = 65536;  // dynamic LDS bytes a workgroup may use
    bool tiny_ok = false;     // every instance fits the fused window
    size_t tiny_shmem = 0;
    bool graph_tiny = false;
    bool graph_adapt = false;
    bool graph_avg = false;
    // host copy of the problem (for the pump's rounding on the host)
    std::vector<double> hval, hb, hl, hu, hc;
    std::vector<char> hsense;
    struct LocalLP {
        std::vector<int32_t> ptr, col, cptr, crow;
        std::vector<double> cval;
        FPProblem P;
    };
    std::vector<LocalLP> local;  // built on the first pump call
    std::vector<double> pump_best;
    FPDev fpd;  // batched fix-and-propagate on the device
    // host mirrors
    std::vector<InstInfo> hinfo;
    InstState *pinned = nullptr;  // 2 * count states
    hipEvent_t ev[2] = {nullptr, nullptr};
    double setup_seconds = 0.0;

    ~scylla_batch()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cexec) (void)hipGraphExecDestroy(cexec);
        for (hipGraphExec_t g : retired) (void)hipGraphExecDestroy(g);
        if (pinned) (void)hipHostFree(pinned);
        if (cstage) (void)hipHostFree(cstage);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        if (side) (void)hipStreamDestroy(side);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace scy {

// ---- defined in runtime.hip
int fail_code(const Err &e);

// Runs f and turns an exception into a negative errno-style return code
// (message in g_err); every C entry point goes through it.
template <class F>
int guarded(F &&f)
{
    try {
        g_err.clear();
        return f();
    } catch (const Err &e) {
        return fail_code(e);
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return -ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return -EIO;
    } catch (...) {
        g_err = "unknown error";
        return -EIO;
    }
}

int validate_params(const scylla_params *p);
// k_limits (optional, [count]): per-instance iteration limit of this solve;
// an instance with a limit <= 0 takes no part (its state is left as it is).
// Only instances [q0, q1) (q1 < 0: all) have their start points projected
// (and zeroed on a cold start); the others must have limits <= 0.
int batch_solve_impl(scylla_batch *h, const scylla_params *p, int32_t warm, scylla_result *results,
                     const int64_t *k_limits = nullptr, int32_t q0 = 0, int32_t q1 = -1);
void ensure_q(scylla_batch *h);
void cast_q(scylla_batch *h);

// ---- defined in fixprop_dev.hip
// Batched fix-and-propagate of every wanted instance on the device.
// is_int: [N] 0/1 (host); xbar: [N] host reference values, or NULL for the
// handle's current primal iterate; want: [count] 0/1 or NULL (all);
// xhat: [N], info: [2 count] (feasible, ignored rows), ignored: [M] or NULL
// (host outputs, written for the wanted instances only).
void fp_batched(scylla_batch *h, const uint8_t *is_int, const double *xbar, int32_t K, int32_t max_rounds,
                const uint8_t *want, double *xhat, int32_t *info, uint8_t *ignored);

// Device range [lo, lo + len) of a vector in the path precision to / from
// FP64 host values.
template <class V>
void get_range(scylla_batch *h, const DevMem &d, int32_t lo, int32_t len, double *out)
{
    if (len <= 0 || !out) return;
    if (sizeof(V) == 8) {
        HIPC(hipMemcpyAsync(out, d.as<char>() + (size_t)lo * 8, (size_t)len * 8, hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
    } else {
        std::vector<float> tmp(len);
        HIPC(hipMemcpyAsync(tmp.data(), d.as<char>() + (size_t)lo * 4, (size_t)len * 4, hipMemcpyDeviceToHost, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
        for (int32_t i = 0; i < len; ++i) out[i] = (double)tmp[i];
    }
}

template <class V>
void put_range(scylla_batch *h, DevMem &d, int32_t lo, int32_t len, const double *in)
{
    if (len <= 0) return;
    if (sizeof(V) == 8) {
        HIPC(hipMemcpyAsync(d.as<char>() + (size_t)lo * 8, in, (size_t)len * 8, hipMemcpyHostToDevice, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
    } else {
        std::vector<float> tmp(len);
        for (int32_t i = 0; i < len; ++i) tmp[i] = (float)in[i];
        HIPC(hipMemcpyAsync(d.as<char>() + (size_t)lo * 4, tmp.data(), (size_t)len * 4, hipMemcpyHostToDevice, h->stream));
        HIPC(hipStreamSynchronize(h->stream));
    }
}

}  // namespace scy

