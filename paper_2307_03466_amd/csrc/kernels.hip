// Device kernels of the PDHG library (gfx950, wave64).
//
// One PDHG iteration (Algorithm 1 inner loop, diagonal steps from the
// preconditioner) is two bandwidth-bound passes:
//   column pass over the CSC copy:  g = c_hat - A^T y,
//       x+ = proj_[l,u](x - t D_c^2 g),  x_bar = 2 x+ - x     (primal step)
//   row pass over the CSR:          y+ = proj_Y(y + s D_r^2 (b - A x_bar))
//                                                             (dual step)
// Both passes use the same tile kernel: a workgroup streams a contiguous
// run of nonzeros (coalesced, non-temporal so the gathered vector keeps the
// L2), multiplies by the gathered vector into LDS, then reduces each row
// with a power-of-two group of lanes sized to the tile's row count and
// applies the fused projection epilogue.  Rows longer than a tile are cut
// into segments whose partial sums a small combine kernel adds in a fixed
// order, so no floating-point atomics are used anywhere and every result is
// bitwise reproducible.
//
// Every R iterations a check (FP64 accumulation) evaluates the relative KKT
// errors of Section 2.2 and the restart quantities; a one-workgroup-per-
// instance decision kernel reduces them in a fixed order and sets status,
// restart and step sizes in FP64 on the device.  With restarts to the
// average the epilogues also fold every iterate into running means, a
// second check evaluates the means, and the decision takes the better of
// the two points.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "scylla_internal.h"
#include "kernels.h"

namespace scy {

// ------------------------------------------------------------------ utils
// The hardware hands consecutive workgroups to the 8 XCDs in turn; map them
// so every XCD works on one contiguous range of tiles (neighbouring tiles
// share cache lines of the row-side vectors in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int xcd = b & 7, local = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    const int base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
    return base + local;
}

template <class V>
__device__ __forceinline__ V wave_sum_width(V v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

// Fixed-order block sum (result valid in thread 0).
template <class V, int NT>
__device__ __forceinline__ V block_sum(V v, V *red)
{
    v = wave_sum_width(v, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    V s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) s += red[q];
    }
    return s;
}

// Fixed-order block sum of two values (results valid in thread 0); red
// holds 2 * NT / 64 doubles.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red)
{
    a = wave_sum_width(a, 64);
    b = wave_sum_width(b, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) {
            sa += red[2 * q];
            sb += red[2 * q + 1];
        }
        a = sa;
        b = sb;
    }
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// Loads of the streamed matrix words / values (read once per pass).
template <int FMT>
struct Entry {
    uint32_t w;
    float f;
    double d;
};

// A matrix entry load: non-temporal (streamed past the caches), or with
// FMT_CACHED in the format a plain load, which the device's last-level
// (Infinity) cache keeps across iterations when an iteration's data fits.
template <int FMT, class T>
__device__ __forceinline__ T mat_load(const T *p)
{
    if constexpr ((FMT & FMT_CACHED) != 0) return *p;
    else return __builtin_nontemporal_load(p);
}

template <int FMT, class A>
__device__ __forceinline__ void load_entry(const MatView &M, int e, uint32_t &w, A &a)
{
    constexpr int F = FMT & ~FMT_CACHED;
    w = mat_load<FMT>(M.ent + e);
    if constexpr (F == FMT_BF16) {
        a = (A)bf16_to_f32(mat_load<FMT>((const uint16_t *)M.val + e));
    } else if constexpr (F == FMT_F32) {
        a = (A)mat_load<FMT>((const float *)M.val + e);
    } else if constexpr (F == FMT_F64) {
        a = (A)mat_load<FMT>((const double *)M.val + e);
    } else {
        a = (A)0;
    }
}

template <int FMT, class A>
__device__ __forceinline__ int decode_entry(const MatView &M, uint32_t w, A &a)
{
    if constexpr ((FMT & ~FMT_CACHED) == FMT_PACKED) {
        a = (A)((int32_t)w >> M.shift);
        return (int)(w & M.mask);
    } else {
        return (int)w;
    }
}

// Stage prod[e - e0] = a_e * vec[idx_e] for e in [e0, e1), e1 - e0 <= NT*EPT.
template <class A, class GV, int FMT, int NT, int EPT>
__device__ __forceinline__ void stage_products(const MatView &M, const GV *__restrict__ vec, int e0,
                                               int e1, A *prod)
{
    const int tid = threadIdx.x;
    uint32_t w[EPT];
    A a[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = e0 + q * NT + tid;
        w[q] = 0;
        a[q] = (A)0;
        if (e < e1) load_entry<FMT, A>(M, e, w[q], a[q]);
    }
    A g[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = e0 + q * NT + tid;
        g[q] = (A)0;
        if (e < e1) {
            const int idx = decode_entry<FMT, A>(M, w[q], a[q]);
            g[q] = (A)vec[idx];
        }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = e0 + q * NT + tid;
        if (e < e1) prod[e - e0] = a[q] * g[q];
    }
}

// ------------------------------------------------------------ epilogues
// Operands of one row's epilogue, loaded before the LDS barrier so their
// latency overlaps the matrix stream.
template <class V>
struct RowOps {
    V own, rhs, diag2, lo, hi, q;
    double ax;  // running A x (adaptive steps)
    uint8_t sense;
};

// Bounds shared by every column of an instance (binary problems, say): the
// column pass reads them once per workgroup instead of twice per column.
template <class V>
struct InstBounds {
    bool uni;
    V lo, hi;
};

template <class V, int DIR>
__device__ __forceinline__ InstBounds<V> inst_bounds(const PassArgs<V> &p, int inst)
{
    InstBounds<V> b{false, (V)0, (V)0};
    if (DIR == DIR_COL && p.ibnd) {
        b.lo = p.ibnd[2 * inst];
        b.hi = p.ibnd[2 * inst + 1];
        b.uni = b.lo == b.lo;
    }
    return b;
}

template <class V, int DIR>
__device__ __forceinline__ void load_ops(const PassArgs<V> &p, int i, RowOps<V> &o, const InstBounds<V> &ib)
{
    o.own = p.own[i];
    o.rhs = p.rhs[i];
    o.diag2 = p.diag2[i];
    if (DIR == DIR_COL) {
        if (ib.uni) {
            o.lo = ib.lo;
            o.hi = ib.hi;
        } else {
            o.lo = p.lo[i];
            o.hi = p.hi[i];
        }
        if (p.q) o.q = p.q[i];
    } else {
        o.sense = p.sense[i];
        if (p.adapt) o.ax = p.ax[i];
    }
}

// The fused epilogue: primal step (column pass) or dual step (row pass) of
// Algorithm 1 for row i given its sum; with adaptive steps it also adds
// this row's terms of the step-size estimate to ip.  Adaptive steps change
// what the row pass gathers: the column pass stores dx = x+ - x in `bar`,
// the row pass's sum is then (A dx)_i, and (A x_bar)_i = (A x)_i + 2 (A dx)_i
// with the running FP64 (A x)_i.
// Iterates in the running average of restart-to-average once this
// iteration's is folded in (the iterates produced since the last restart),
// or 0 without an average.
template <class V>
__device__ __forceinline__ V avg_count(const PassArgs<V> &p, const InstState &S, int jw)
{
    return p.avg ? (V)(S.k + jw + 1 - S.kr) : (V)0;
}

// Folds the new iterate value v of entry i into the running mean (the first
// iterate after a restart starts it).
template <class V>
__device__ __forceinline__ void fold_avg(const PassArgs<V> &p, int i, V v, V acnt)
{
    if (acnt > (V)0) p.avg[i] = acnt == (V)1 ? v : p.avg[i] + (v - p.avg[i]) / acnt;
}

template <class V, int DIR>
__device__ __forceinline__ void apply_ops(const PassArgs<V> &p, int i, V sum, V step, bool copy_ref,
                                          const RowOps<V> &o, double (&ip)[2], V acnt)
{
    if (DIR == DIR_COL) {
        V xn = o.own + step * o.diag2 * (sum - o.rhs);
        if (p.q) xn /= (V)1 + step * o.diag2 * o.q;  // exact prox of q x^2 / 2
        xn = xn < o.lo ? o.lo : xn;
        xn = xn > o.hi ? o.hi : xn;
        if (copy_ref) p.own_ref[i] = o.own;
        p.bar[i] = p.adapt ? xn - o.own : (V)2 * xn - o.own;
        p.own[i] = xn;
        fold_avg(p, i, xn, acnt);
        if (p.adapt) {
            const double d = (double)xn - (double)o.own;
            ip[0] += d * d / (double)o.diag2;
        }
    } else {
        // residual b_i - (A x_bar)_i; with adaptive steps sum = (A dx)_i
        const V res = p.adapt ? (V)((double)o.rhs - (o.ax + 2.0 * (double)sum)) : o.rhs - sum;
        V v = o.own + step * o.diag2 * res;
        if (o.sense == 'G') v = v > (V)0 ? v : (V)0;
        else if (o.sense == 'L') v = v < (V)0 ? v : (V)0;
        if (copy_ref) p.own_ref[i] = o.own;
        p.own[i] = v;
        fold_avg(p, i, v, acnt);
        if (p.adapt) {
            const double dy = (double)v - (double)o.own;
            ip[0] += dy * dy / (double)o.diag2;
            ip[1] += dy * (double)sum;
            p.ax[i] = o.ax + (double)sum;
        }
    }
}

// Lanes per row for a tile of `nrows` rows: the largest power of two (<= 64)
// with nrows * L <= NT.
template <int NT>
__device__ __forceinline__ int lanes_per_row(int nrows)
{
    int L = 1;
    while (L < 64 && nrows * (L << 1) <= NT) L <<= 1;
    return L;
}

// ------------------------------------------------------- iteration pass
template <class V, int FMT, int DIR, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_pass(const PassArgs<V> p, const int jw)
{
    constexpr int CH = NT * EPT;
    __shared__ V prod[CH];
    __shared__ V red[NT / 64];
    __shared__ double red2[2 * NT / 64];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int4 T = p.tiles[t];
    const InstState &S = p.st[T.z];
    if (S.status != ST_RUN || jw >= S.nrun) return;
    const bool copy_ref = (jw == 0) && (S.restart_now != 0);
    const V step = DIR == DIR_COL ? (V)S.t : (V)S.s;
    const V acnt = avg_count(p, S, jw);
    const int tid = threadIdx.x;
    const InstBounds<V> ib = inst_bounds<V, DIR>(p, T.z);
    if (T.w >= 0) {  // one segment of a long row: partial sum only
        stage_products<V, V, FMT, NT, EPT>(p.M, p.gvec, T.x, T.y, prod);
        __syncthreads();
        V s = 0;
        for (int q = tid; q < T.y - T.x; q += NT) s += prod[q];
        s = block_sum<V, NT>(s, red);
        if (tid == 0) {
            p.seg[T.w] = s;
            if (p.adapt) p.ipart[2 * t] = p.ipart[2 * t + 1] = 0.0;
        }
        return;
    }
    double ip[2] = {0.0, 0.0};
    const int r0 = T.x, nrows = T.y - T.x;
    const int e0 = p.M.ptr[r0], e1 = p.M.ptr[T.y];
    const int L = lanes_per_row<NT>(nrows);
    const int groups = NT / L, lane = tid & (L - 1);
    // first row of this lane group: bounds and epilogue operands up front
    int r = tid / L;
    int rb = 0, re = 0;
    RowOps<V> ops;
    if (r < nrows) {
        rb = p.M.ptr[r0 + r] - e0;
        re = p.M.ptr[r0 + r + 1] - e0;
        if (lane == 0) load_ops<V, DIR>(p, r0 + r, ops, ib);
    }
    stage_products<V, V, FMT, NT, EPT>(p.M, p.gvec, e0, e1, prod);
    __syncthreads();
    for (; r < nrows; r += groups) {
        V s = 0;
        for (int q = rb + lane; q < re; q += L) s += prod[q];
        if (L > 1) s = wave_sum_width(s, L);
        if (lane == 0) apply_ops<V, DIR>(p, r0 + r, s, step, copy_ref, ops, ip, acnt);
        const int rn = r + groups;
        if (rn < nrows) {
            rb = p.M.ptr[r0 + rn] - e0;
            re = p.M.ptr[r0 + rn + 1] - e0;
            if (lane == 0) load_ops<V, DIR>(p, r0 + rn, ops, ib);
        }
    }
    if (p.adapt) {
        block_sum2<NT>(ip[0], ip[1], red2);
        if (tid == 0) {
            p.ipart[2 * t] = ip[0];
            p.ipart[2 * t + 1] = ip[1];
        }
    }
}

// ------------------------------------------- gather-blocked pass (partials)
// Tile of block b (bits 24.. of T.z) of a gather-blocked orientation: row
// sums over the block's nonzeros go to P[b * rows + i] (A = V for the
// iteration, double for the check); long sub-rows go to segment slots.
template <class V, class A, int FMT, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_bpart(const PassArgs<V> p, const int jw, const int check)
{
    constexpr int CH = NT * EPT;
    __shared__ A prod[CH];
    __shared__ A red[NT / 64];
    const int4 T = p.tiles[blockIdx.x];
    const int inst = T.z & 0xffffff, b = T.z >> 24;
    const InstState &S = p.st[inst];
    if (S.status != ST_RUN || (!check && jw >= S.nrun)) return;
    const int tid = threadIdx.x;
    A *P = (A *)(check ? (void *)p.P64 : (void *)p.P);
    if (T.w >= 0) {
        stage_products<A, V, FMT, NT, EPT>(p.M, p.gvec, T.x, T.y, prod);
        __syncthreads();
        A s = 0;
        for (int q = tid; q < T.y - T.x; q += NT) s += prod[q];
        s = block_sum<A, NT>(s, red);
        A *seg = (A *)(check ? (void *)p.seg64 : (void *)p.seg);
        if (tid == 0) seg[T.w] = s;
        return;
    }
    const int32_t *ptr = p.bptr + (size_t)b * (p.rows + 1);
    const int r0 = T.x, nrows = T.y - T.x;
    const int e0 = ptr[r0], e1 = ptr[T.y];
    const int L = lanes_per_row<NT>(nrows);
    const int groups = NT / L, lane = tid & (L - 1);
    int r = tid / L;
    int rb = 0, re = 0;
    if (r < nrows) {
        rb = ptr[r0 + r] - e0;
        re = ptr[r0 + r + 1] - e0;
    }
    stage_products<A, V, FMT, NT, EPT>(p.M, p.gvec, e0, e1, prod);
    __syncthreads();
    A *Pb = P + (size_t)b * p.rows;
    for (; r < nrows; r += groups) {
        A s = 0;
        for (int q = rb + lane; q < re; q += L) s += prod[q];
        if (L > 1) s = wave_sum_width(s, L);
        if (lane == 0) Pb[r0 + r] = s;
        const int rn = r + groups;
        if (rn < nrows) {
            rb = ptr[r0 + rn] - e0;
            re = ptr[r0 + rn + 1] - e0;
        }
    }
}

// Long sub-rows of a blocked orientation: P[b][row] = sum of its segments.
template <class V, class A>
__global__ __launch_bounds__(256) void k_bseg(const PassArgs<V> p, const int jw, const int check)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.nlong) return;
    const int4 L = p.longs[q];
    const int inst = L.w & 0xffffff, b = L.w >> 24;
    const InstState &S = p.st[inst];
    if (S.status != ST_RUN || (!check && jw >= S.nrun)) return;
    const A *seg = (const A *)(check ? (const void *)p.seg64 : (const void *)p.seg);
    A s = 0;
    for (int k = 0; k < L.z; ++k) s += seg[L.y + k];
    A *P = (A *)(check ? (void *)p.P64 : (void *)p.P);
    P[(size_t)b * p.rows + L.x] = s;
}

// Combine of a blocked orientation (one thread per row, 256 rows of one
// instance per workgroup): sum the B block partials in block order, then the
// fused epilogue.
template <class V, int DIR>
__global__ __launch_bounds__(256) void k_bcombine(const PassArgs<V> p, const int jw)
{
    __shared__ double red2[8];
    const int4 T = p.ctiles[blockIdx.x];
    const InstState &S = p.st[T.z];
    if (S.status != ST_RUN || jw >= S.nrun) return;
    const int i = T.x + threadIdx.x;
    const InstBounds<V> ib = inst_bounds<V, DIR>(p, T.z);
    double ip[2] = {0.0, 0.0};
    if (i < T.y) {
        const bool copy_ref = (jw == 0) && (S.restart_now != 0);
        RowOps<V> ops;
        load_ops<V, DIR>(p, i, ops, ib);
        V s = 0;
        const int nb = p.bq ? p.bq[T.z] : p.B;
        for (int b = 0; b < nb; ++b) s += p.P[(size_t)b * p.rows + i];
        apply_ops<V, DIR>(p, i, s, DIR == DIR_COL ? (V)S.t : (V)S.s, copy_ref, ops, ip, avg_count(p, S, jw));
    }
    if (p.adapt) {
        block_sum2<256>(ip[0], ip[1], red2);
        if (threadIdx.x == 0) {
            p.ipart[2 * blockIdx.x] = ip[0];
            p.ipart[2 * blockIdx.x + 1] = ip[1];
        }
    }
}

// ------------------------------------------- LDS-staged pass (small instances)
// When an instance's whole gathered vector fits in LDS, one workgroup copies
// it there once and then walks a run of sub-tiles of that instance (whole
// rows, <= NT*EPT nonzeros each): every gather is an LDS read.  The loop is
// software-pipelined: the coalesced loads of sub-tile t+1's nonzeros are in
// flight while sub-tile t's rows are reduced and updated.
// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (__syncthreads also waits for them, which would
// serialise the prefetch of the next sub-tile with the current one).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Copies src[0, n) into LDS by NT threads in 16-byte words, U in flight per
// thread (a plain strided loop would wait for each load before its LDS
// store).  The copy starts at `base` (16-byte aligned LDS) shifted by the
// source's misalignment, so that every word is aligned on both sides, and
// the copied vector begins at the returned pointer (dst[k] = src[k], k < n;
// base needs n values + LDS_COPY_SLACK bytes).
// The words may start up to 12 bytes before src, inside the same buffer
// (device buffers are 256-byte aligned); the tail is copied value by value.
template <int NT, int U, class V>
__device__ __forceinline__ V *copy_to_lds_vec(V *base, const V *__restrict__ src, int n)
{
    constexpr int W = 16 / sizeof(V);
    typedef V VW __attribute__((ext_vector_type(W)));
    const int mis = (int)(((uintptr_t)src & 15) / sizeof(V));
    const V *asrc = src - mis;
    const int words = (mis + n) / W;
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < words; k0 += NT * U) {
        VW t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * NT + tid;
            if (k < words) t[u] = reinterpret_cast<const VW *>(asrc)[k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * NT + tid;
            if (k < words) reinterpret_cast<VW *>(base)[k] = t[u];
        }
    }
    for (int k = words * W + tid; k < mis + n; k += NT) base[k] = asrc[k];
    return base + mis;
}

template <class V, int FMT, int NT, int EPT>
__device__ __forceinline__ void spass_load(const MatView &M, int e0, int e1, uint32_t (&w)[EPT], V (&a)[EPT])
{
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = e0 + q * NT + (int)threadIdx.x;
        w[q] = 0;
        a[q] = (V)0;
        if (e < e1) load_entry<FMT, V>(M, e, w[q], a[q]);
    }
}

template <class V, int FMT, int DIR, int NT, int EPT, bool PF>
__global__ __launch_bounds__(NT) void k_spass(const PassArgs<V> p, const int jw)
{
    constexpr int CH = NT * EPT;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *prod = reinterpret_cast<V *>(lds_raw);  // [CH]
    V *sv = prod + CH;                         // [gathered length]
    const int4 T = p.tiles[xcd_tile(blockIdx.x, gridDim.x)];  // {sub0, sub1, inst | slice << 24, kind}
    // kind -1: a whole instance's gathered vector in LDS, fused epilogue;
    // kind -2: one slice of it, partial sums to xP (added by the combine)
    const bool part = T.w == -2;
    const int inst = T.z & 0xffffff, sl = T.z >> 24;
    const InstState &S = p.st[inst];
    if (S.status != ST_RUN || jw >= S.nrun) return;
    const bool copy_ref = (jw == 0) && (S.restart_now != 0);
    const V step = DIR == DIR_COL ? (V)S.t : (V)S.s;
    const V acnt = avg_count(p, S, jw);
    const int tid = threadIdx.x;
    const InstBounds<V> ib = inst_bounds<V, DIR>(p, inst);
    MatView M = p.M;
    const int4 *sub = p.sub;
    int g0 = p.gofs[inst], glen = p.gofs[inst + 1] - g0;
    V *Ps = nullptr;
    if (part) {
        M = p.X;
        M.ptr = p.X.ptr + (size_t)sl * (p.rows + 1);
        sub = p.xsub;
        const int Sq = p.xSq[inst];
        const int lo = (int)(((int64_t)glen * sl) / Sq), hi = (int)(((int64_t)glen * (sl + 1)) / Sq);
        g0 += lo;
        glen = hi - lo;
        Ps = p.xP + (size_t)sl * p.rows;
    }
    double ip[2] = {0.0, 0.0};
    // Descriptors of the first SPASS_DMAX sub-tiles (first row, end row,
    // first and end nonzero) go to LDS with the vector, so that starting
    // the next sub-tile's loads needs no dependent global reads.
    __shared__ int sdesc[4][SPASS_DMAX];
    for (int u = tid; u < T.y - T.x && u < SPASS_DMAX; u += NT) {
        const int4 d = sub[T.x + u];
        sdesc[0][u] = d.x;
        sdesc[1][u] = d.y;
        sdesc[2][u] = M.ptr[d.x];
        sdesc[3][u] = M.ptr[d.y];
    }
    // sub-tile state (nonzeros in registers one sub-tile ahead; with PF also
    // this thread's first row bounds and epilogue operands)
    int4 D = sub[T.x];
    int e0 = M.ptr[D.x], e1 = M.ptr[D.y];
    uint32_t w[EPT];
    V a[EPT];
    spass_load<V, FMT, NT, EPT>(M, e0, e1, w, a);
    int L = 1, r = 0, rb = 0, re = 0;
    RowOps<V> ops;
    if (PF) {
        L = lanes_per_row<NT>(D.y - D.x);
        r = tid / L;
        if (r < D.y - D.x) {
            rb = M.ptr[D.x + r] - e0;
            re = M.ptr[D.x + r + 1] - e0;
            if (!part && (tid & (L - 1)) == 0) load_ops<V, DIR>(p, D.x + r, ops, ib);
        }
    }
    sv = copy_to_lds_vec<NT, 8>(sv, p.gvec + g0, glen);
    lds_barrier();
    for (int t = T.x; t < T.y; ++t) {
        // products of sub-tile t from the registers
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            const int e = e0 + q * NT + tid;
            if (e < e1) {
                const int idx = decode_entry<FMT, V>(M, w[q], a[q]);
                prod[e - e0] = a[q] * sv[idx - g0];
            }
        }
        const int r0c = D.x, nrows = D.y - D.x, e0c = e0;
        int Lc, rc, rbc, rec;
        RowOps<V> opc;
        if (PF) {
            Lc = L;
            rc = r;
            rbc = rb;
            rec = re;
            opc = ops;
        } else {
            Lc = lanes_per_row<NT>(nrows);
            rc = tid / Lc;
            rbc = rec = 0;
            if (rc < nrows) {
                rbc = M.ptr[r0c + rc] - e0c;
                rec = M.ptr[r0c + rc + 1] - e0c;
                if (!part && (tid & (Lc - 1)) == 0) load_ops<V, DIR>(p, r0c + rc, opc, ib);
            }
        }
        lds_barrier();
        // sub-tile t+1's nonzeros (and with PF its row bounds and operands)
        // are in flight during this reduction
        if (t + 1 < T.y) {
            const int u = t + 1 - T.x;
            if (u < SPASS_DMAX) {
                D.x = sdesc[0][u];
                D.y = sdesc[1][u];
                e0 = sdesc[2][u];
                e1 = sdesc[3][u];
            } else {
                D = sub[t + 1];
                e0 = M.ptr[D.x];
                e1 = M.ptr[D.y];
            }
            spass_load<V, FMT, NT, EPT>(M, e0, e1, w, a);
            if (PF) {
                L = lanes_per_row<NT>(D.y - D.x);
                r = tid / L;
                if (r < D.y - D.x) {
                    rb = M.ptr[D.x + r] - e0;
                    re = M.ptr[D.x + r + 1] - e0;
                    if (!part && (tid & (L - 1)) == 0) load_ops<V, DIR>(p, D.x + r, ops, ib);
                }
            }
        }
        const int groups = NT / Lc, lane = tid & (Lc - 1);
        for (; rc < nrows; rc += groups) {
            V sum = 0;
            for (int q = rbc + lane; q < rec; q += Lc) sum += prod[q];
            if (Lc > 1) sum = wave_sum_width(sum, Lc);
            if (lane == 0) {
                if (part) Ps[r0c + rc] = sum;
                else apply_ops<V, DIR>(p, r0c + rc, sum, step, copy_ref, opc, ip, acnt);
            }
            const int rn = rc + groups;
            if (rn < nrows) {
                rbc = M.ptr[r0c + rn] - e0c;
                rec = M.ptr[r0c + rn + 1] - e0c;
                if (!part && lane == 0) load_ops<V, DIR>(p, r0c + rn, opc, ib);
            }
        }
        lds_barrier();
    }
    if (p.adapt && !part) {
        // the product buffer is free after the last barrier
        block_sum2<NT>(ip[0], ip[1], reinterpret_cast<double *>(lds_raw));
        if (tid == 0) {
            const int t = xcd_tile(blockIdx.x, gridDim.x);
            p.ipart[2 * t] = ip[0];
            p.ipart[2 * t + 1] = ip[1];
        }
    }
}

// ------------------------------------------ direct LDS-staged pass
// For instances whose whole gathered vector fits in LDS with nothing beside
// it: a workgroup copies the instance's vector to LDS once, then each group
// of L lanes reduces whole rows straight from their nonzeros (streamed from
// global memory, gathered from LDS), DPASS_R rows at a time, combines its
// lanes with shuffles and applies the fused epilogue; each lane takes K
// nonzeros of a row per round (K = 16 / L for the plan's lanes per row L,
// between 2 and 8, so a row of up to 16 nonzeros is one round).  The row bounds of
// the next DPASS_R rows load while the current ones are reduced, so each
// step waits for one round trip (the nonzeros).  Without a product buffer
// the vector may fill the LDS.  Tile {r0, r1, inst, L}; within a row each
// lane adds its nonzeros in order and the lanes combine in a fixed tree, so
// the result is reproducible for a given plan.
constexpr int DPASS_R = 4;

template <class V, int FMT, int K>
__device__ __forceinline__ V direct_row_chunk(const MatView &M, const V *sv, int g0, int e, int e1, int L)
{
    uint32_t w[K];
    V a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int ee = e + k * L;
        w[k] = 0;
        a[k] = (V)0;
        if (ee < e1) load_entry<FMT, V>(M, ee, w[k], a[k]);
    }
    V s = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (e + k * L < e1) {
            const int idx = decode_entry<FMT, V>(M, w[k], a[k]);
            s += a[k] * sv[idx - g0];
        }
    }
    return s;
}

template <class V, int FMT, int DIR, int NT, int K>
__global__ __launch_bounds__(NT) void k_dpass(const PassArgs<V> p, const int jw)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red2[2 * NT / 64];
    V *sv = reinterpret_cast<V *>(lds_raw);
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int4 T = p.dtiles[t];
    const InstState &S = p.st[T.z];
    if (S.status != ST_RUN || jw >= S.nrun) return;
    const bool copy_ref = (jw == 0) && (S.restart_now != 0);
    const V step = DIR == DIR_COL ? (V)S.t : (V)S.s;
    const V acnt = avg_count(p, S, jw);
    const InstBounds<V> ib = inst_bounds<V, DIR>(p, T.z);
    const int tid = threadIdx.x, L = T.w, lane = tid & (L - 1), groups = NT / L;
    const int g0 = p.gofs[T.z], glen = p.gofs[T.z + 1] - g0;
    // bounds of this lane group's first DPASS_R rows, then the vector copy
    int nb0[DPASS_R], nb1[DPASS_R];
    const int first = T.x + tid / L;
#pragma unroll
    for (int u = 0; u < DPASS_R; ++u) {
        const int r = first + u * groups;
        nb0[u] = nb1[u] = 0;
        if (r < T.y) {
            nb0[u] = p.M.ptr[r];
            nb1[u] = p.M.ptr[r + 1];
        }
    }
    sv = copy_to_lds_vec<NT, 8>(sv, p.gvec + g0, glen);
    lds_barrier();
    double ip[2] = {0.0, 0.0};
    for (int base = first; base < T.y; base += DPASS_R * groups) {
        int b0[DPASS_R], b1[DPASS_R];
#pragma unroll
        for (int u = 0; u < DPASS_R; ++u) {
            b0[u] = nb0[u];
            b1[u] = nb1[u];
        }
        // nonzeros of the current rows (first K per lane of each)
        uint32_t w[DPASS_R][K];
        V a[DPASS_R][K];
#pragma unroll
        for (int u = 0; u < DPASS_R; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int e = b0[u] + lane + k * L;
                w[u][k] = 0;
                a[u][k] = (V)0;
                if (e < b1[u]) load_entry<FMT, V>(p.M, e, w[u][k], a[u][k]);
            }
        RowOps<V> ops[DPASS_R];
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < DPASS_R; ++u)
                if (base + u * groups < T.y) load_ops<V, DIR>(p, base + u * groups, ops[u], ib);
        }
        // bounds of the next rows load meanwhile
#pragma unroll
        for (int u = 0; u < DPASS_R; ++u) {
            const int r = base + (DPASS_R + u) * groups;
            nb0[u] = nb1[u] = 0;
            if (r < T.y) {
                nb0[u] = p.M.ptr[r];
                nb1[u] = p.M.ptr[r + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < DPASS_R; ++u) {
            V sum = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (b0[u] + lane + k * L < b1[u]) {
                    const int idx = decode_entry<FMT, V>(p.M, w[u][k], a[u][k]);
                    sum += a[u][k] * sv[idx - g0];
                }
            }
            // rows longer than K per lane: further rounds
            for (int c = lane + K * L; b0[u] + c < b1[u]; c += K * L)
                sum += direct_row_chunk<V, FMT, K>(p.M, sv, g0, b0[u] + c, b1[u], L);
            if (L > 1) sum = wave_sum_width(sum, L);
            const int r = base + u * groups;
            if (lane == 0 && r < T.y) apply_ops<V, DIR>(p, r, sum, step, copy_ref, ops[u], ip, acnt);
        }
    }
    if (p.adapt) {
        block_sum2<NT>(ip[0], ip[1], red2);
        if (tid == 0) {
            p.ipart[2 * t] = ip[0];
            p.ipart[2 * t + 1] = ip[1];
        }
    }
}

// Long rows: add the segment partials in segment order, then the epilogue.
template <class V, int DIR>
__global__ __launch_bounds__(256) void k_combine(const PassArgs<V> p, const int jw)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= p.nlong) return;
    const int4 L = p.longs[q];
    const InstState &S = p.st[L.w];
    if (S.status != ST_RUN || jw >= S.nrun) return;
    const bool copy_ref = (jw == 0) && (S.restart_now != 0);
    const InstBounds<V> ib = inst_bounds<V, DIR>(p, L.w);
    V s = 0;
    for (int k = 0; k < L.z; ++k) s += p.seg[L.y + k];
    RowOps<V> ops;
    load_ops<V, DIR>(p, L.x, ops, ib);
    double ip[2] = {0.0, 0.0};
    apply_ops<V, DIR>(p, L.x, s, DIR == DIR_COL ? (V)S.t : (V)S.s, copy_ref, ops, ip, avg_count(p, S, jw));
    if (p.adapt) {
        p.iplong[2 * q] = ip[0];
        p.iplong[2 * q + 1] = ip[1];
    }
}

// ------------------------------------------------------------ KKT check
// Per-row / per-column FP64 contributions (Section 2.2, original problem).
//   row i : q0 = r_p,i^2, q1 = b_i y_i, q2 = ((y_i - yr_i) / d_r,i)^2
//   col j : q0 = r_d,j^2, q1 = c_j x_j, q2 = l_j max(lam_j,0) + u_j min(lam_j,0),
//           q3 = ((x_j - xr_j) / d_c,j)^2
template <class V>
__device__ __forceinline__ void row_terms(const PassArgs<V> &p, int i, double ax, double q[CHK])
{
    const double b = p.rhs64[i];
    const uint8_t sn = p.sense[i];
    double r;
    if (sn == 'G') r = fmax(b - ax, 0.0);
    else if (sn == 'L') r = fmax(ax - b, 0.0);
    else r = b - ax;
    const double y = (double)p.own[i];
    const double dy = (y - (double)p.own_ref[i]) / p.d64[i];
    q[0] += r * r;
    q[1] += b * y;
    q[2] += dy * dy;
    // moves since the previous check: v = y - y_prev, A d = A x - (A x)_prev
    // (the check of the running average has none)
    if (!p.own_prev) return;
    const double v = y - (double)p.own_prev[i];
    const double vp = sn == 'G' ? fmax(v, 0.0) : (sn == 'L' ? fmin(v, 0.0) : v);
    const double ad = ax - p.prod_prev[i];
    const double viol = sn == 'G' ? fmax(-ad, 0.0) : (sn == 'L' ? fmax(ad, 0.0) : ad);
    q[4] += b * v;
    q[5] += (v - vp) * (v - vp);
    q[6] += viol * viol;
    p.own_prev[i] = p.own[i];
    p.prod_prev[i] = ax;
}

template <class V>
__device__ __forceinline__ void col_terms(const PassArgs<V> &p, int j, double aty, double q[CHK])
{
    // with a diagonal Hessian: reduced cost c + Q x - A^T y, primal objective
    // + x^T Q x / 2, dual objective - x^T Q x / 2 (kept with the bound terms)
    const double x = (double)p.own[j];
    const double qx = p.q64 ? p.q64[j] * x : 0.0;
    const double g = p.rhs64[j] + qx - aty;
    const double l = p.lo64[j], u = p.hi64[j];
    const bool lf = isfinite(l), uf = isfinite(u);
    double lam;
    if (lf && uf) lam = g;
    else if (lf) lam = fmax(g, 0.0);
    else if (uf) lam = fmin(g, 0.0);
    else lam = 0.0;
    const double rd = g - lam;
    const double dx = (x - (double)p.own_ref[j]) / p.d64[j];
    q[0] += rd * rd;
    q[1] += p.rhs64[j] * x + 0.5 * qx * x;
    if (lf && lam > 0.0) q[2] += l * lam;
    if (uf && lam < 0.0) q[2] += u * lam;
    q[2] -= 0.5 * qx * x;
    q[3] += dx * dx;
    // moves since the previous check: A^T v = A^T y - (A^T y)_prev, d = x - x_prev
    // (the check of the running average has none)
    if (!p.own_prev) return;
    const double w = aty - p.prod_prev[j];
    double rl;
    if (lf && uf) rl = -w;
    else if (lf) rl = fmax(-w, 0.0);
    else if (uf) rl = fmin(-w, 0.0);
    else rl = 0.0;
    q[4] += (w + rl) * (w + rl);
    if (lf && rl > 0.0) q[5] += l * rl;
    if (uf && rl < 0.0) q[5] += u * rl;
    const double d = x - (double)p.own_prev[j];
    q[6] += p.rhs64[j] * d;
    double bv;
    if (lf && uf) bv = d;
    else if (lf) bv = fmin(d, 0.0);
    else if (uf) bv = fmax(d, 0.0);
    else bv = 0.0;
    q[7] += bv * bv;
    if (p.q64) q[7] += (p.q64[j] * d) * (p.q64[j] * d);
    p.own_prev[j] = p.own[j];
    p.prod_prev[j] = aty;
}

template <class V, int FMT, int DIR, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_check(const PassArgs<V> p)
{
    constexpr int CH = NT * EPT;
    __shared__ double prod[CH];
    __shared__ double red[NT / 64];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int4 T = p.tiles[t];
    const InstState &S = p.st[T.z];
    if (S.status != ST_RUN) return;
    int e0, e1;
    if (T.w >= 0) {
        e0 = T.x;
        e1 = T.y;
    } else {
        e0 = p.M.ptr[T.x];
        e1 = p.M.ptr[T.y];
    }
    // row check gathers x (not x_bar), column check gathers y
    stage_products<double, V, FMT, NT, EPT>(p.M, p.gvec, e0, e1, prod);
    __syncthreads();
    const int tid = threadIdx.x;
    if (T.w >= 0) {
        // a segment's row terms are added once by the combine kernel; its own
        // tile slot contributes nothing
        double s = 0;
        for (int q = tid; q < e1 - e0; q += NT) s += prod[q];
        s = block_sum<double, NT>(s, red);
        if (tid == 0) {
            p.seg64[T.w] = s;
            for (int k = 0; k < CHK; ++k) p.part[CHK * t + k] = 0.0;
        }
        return;
    }
    const int r0 = T.x, nrows = T.y - T.x;
    int L = 1;
    while (L < 64 && nrows * (L << 1) <= NT) L <<= 1;
    const int groups = NT / L, lane = tid & (L - 1);
    double q[CHK] = {};
    for (int r = tid / L; r < nrows; r += groups) {
        const int rb = p.M.ptr[r0 + r] - e0, re = p.M.ptr[r0 + r + 1] - e0;
        double s = 0;
        for (int k = rb + lane; k < re; k += L) s += prod[k];
        if (L > 1) s = wave_sum_width(s, L);
        if (lane == 0) {
            if (DIR == DIR_COL) {
                col_terms(p, r0 + r, s, q);
            } else {
                row_terms(p, r0 + r, s, q);
                if (p.adapt) p.ax[r0 + r] = s;  // A x of the current point (FP64)
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CHK; ++k) {
        __syncthreads();
        const double v = block_sum<double, NT>(q[k], red);
        if (tid == 0) p.part[CHK * t + k] = v;
    }
}

template <class V, int DIR>
__global__ __launch_bounds__(256) void k_combine_check(const PassArgs<V> p)
{
    const int qi = blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= p.nlong) return;
    const int4 L = p.longs[qi];
    const InstState &S = p.st[L.w];
    if (S.status != ST_RUN) return;
    double s = 0;
    for (int k = 0; k < L.z; ++k) s += p.seg64[L.y + k];
    double q[CHK] = {};
    if (DIR == DIR_COL) {
        col_terms(p, L.x, s, q);
    } else {
        row_terms(p, L.x, s, q);
        if (p.adapt) p.ax[L.x] = s;
    }
    for (int k = 0; k < CHK; ++k) p.lpart[CHK * qi + k] = q[k];
}

// Check combine of a blocked orientation: FP64 row sums from the block
// partials, row / column KKT terms, fixed-order sum per combine tile.
template <class V, int DIR>
__global__ __launch_bounds__(256) void k_bcombine_check(const PassArgs<V> p)
{
    __shared__ double red[4];
    const int ct = blockIdx.x;
    const int4 T = p.ctiles[ct];
    const InstState &S = p.st[T.z];
    if (S.status != ST_RUN) return;
    const int i = T.x + threadIdx.x;
    double q[CHK] = {};
    if (i < T.y) {
        double s = 0;
        for (int b = 0; b < p.B; ++b) s += p.P64[(size_t)b * p.rows + i];
        if (DIR == DIR_COL) {
            col_terms(p, i, s, q);
        } else {
            row_terms(p, i, s, q);
            if (p.adapt) p.ax[i] = s;
        }
    }
#pragma unroll
    for (int k = 0; k < CHK; ++k) {
        __syncthreads();
        const double v = block_sum<double, 256>(q[k], red);
        if (threadIdx.x == 0) p.part[CHK * ct + k] = v;
    }
}

// ------------------------------------------------------------- decision
// Termination test (Section 2.2), infeasibility certificates, restart rule
// and primal-weight update in FP64 for one instance, from the check window's
// reduced sums tot = {||r_p||^2, b^T y, ||dy~||^2, ||r_d||^2, c^T x, bound
// terms, ||dx~||^2, b^T v, |v - proj_Y v|^2, |row violation of A d|^2,
// |A^T v + lam|^2, ray bound terms, c^T d, |bound violation of d|^2}.
constexpr int NTOT = 14;

// Relative KKT error of a check's totals (Section 2.2): rho_p, rho_d,
// rho_g, P, D and E = max of the three (NaN when one is not finite).
struct Kkt {
    double rho_p, rho_d, rho_g, P, D, E;
};

__device__ __forceinline__ Kkt kkt_of(const InstState &S, const double tot[NTOT])
{
    Kkt r;
    r.rho_p = sqrt(tot[0]) / (1.0 + S.bnorm);
    r.rho_d = sqrt(tot[3]) / (1.0 + S.cnorm);
    r.P = tot[4];
    r.D = tot[1] + tot[5];
    r.rho_g = fabs(r.P - r.D) / (1.0 + fabs(r.P) + fabs(r.D));
    r.E = fmax(r.rho_p, fmax(r.rho_d, r.rho_g));
    if (!isfinite(r.rho_p) || !isfinite(r.rho_d) || !isfinite(r.rho_g)) r.E = NAN;
    return r;
}

// The decision at a check.  totA: the totals of the running average
// (restart to the average), or null.  The candidate is the average when
// its error is below the current iterate's; its error drives termination,
// the restart rule and E_prev, a restart or an OPTIMAL / iteration-limit
// stop takes it (take_avg), and infeasibility and stalling look at the
// current iterate.
__device__ void decide_state(InstState &S, const double tot[NTOT], const double *totA, int R)
{
    const int64_t k = S.k + S.nrun;
    S.k = k;
    S.nrun = 0;
    S.restart_now = 0;
    S.take_avg = 0;
    const Kkt cur = kkt_of(S, tot);
    if (!isfinite(cur.E)) {
        S.rho_p = cur.rho_p;
        S.rho_d = cur.rho_d;
        S.rho_g = cur.rho_g;
        S.pobj = cur.P;
        S.dobj = cur.D;
        S.rel = cur.E;
        S.status = ST_NUM;
        return;
    }
    // the average exists once an iterate was produced since the last restart
    bool use_avg = false;
    Kkt avg = cur;
    if (totA && S.avg_on && k > S.kr) {
        avg = kkt_of(S, totA);
        use_avg = avg.E < cur.E;
    }
    const Kkt &c = use_avg ? avg : cur;
    const double E = c.E;
    S.rho_p = c.rho_p;
    S.rho_d = c.rho_d;
    S.rho_g = c.rho_g;
    S.pobj = c.P;
    S.dobj = c.D;
    S.rel = E;
    if (E <= S.tol) {
        S.take_avg = use_avg;
        S.status = ST_OPT;
        return;
    }
    if (S.infeas_tol > 0.0 && k > 0) {
        // a dual ray certifies primal infeasibility, a primal ray dual
        // infeasibility (moves since the previous check)
        const double rho = tot[7] + tot[11], rres = sqrt(tot[8] + tot[10]);
        if (rho > 0.0 && rres <= S.infeas_tol * rho) { S.status = ST_PINF; return; }
        const double cd = tot[12], pviol = sqrt(tot[9] + tot[13]);
        if (cd < 0.0 && pviol <= -S.infeas_tol * cd) { S.status = ST_DINF; return; }
    }
    if (S.stall_tol > 0.0) {
        // bounds stalling (Algorithm 1's inner-loop exit): neither objective
        // bound of the current iterate moved by more than stall_tol
        // (1 + |value|) since the previous check, stall_checks times in a row
        if (k > 0) {
            const bool moved = fabs(cur.P - S.pprev) > S.stall_tol * (1.0 + fabs(cur.P)) ||
                               fabs(cur.D - S.dprev) > S.stall_tol * (1.0 + fabs(cur.D));
            S.nstall = moved ? 0 : S.nstall + 1;
            if (S.nstall >= S.stall_checks) { S.status = ST_STALL; return; }
        }
        S.pprev = cur.P;
        S.dprev = cur.D;
    }
    if (k >= S.k_limit) {
        S.take_avg = use_avg;
        S.status = ST_ITER;
        return;
    }
    if (S.force_stop) { S.status = ST_TIME; return; }
    if (k == 0) {
        S.Er = E;
        S.kr = 0;
        S.restart_now = 1;
    } else if (S.restart_on) {
        const bool fire = (E <= 0.2 * S.Er) || (E <= 0.8 * S.Er && E > S.Ep) ||
                          ((double)(k - S.kr) >= 0.36 * (double)k);
        if (fire) {
            // distances of the candidate to the last restart point
            const double *tc = use_avg ? totA : tot;
            const double dx = sqrt(tc[6]), dy = sqrt(tc[2]);
            if (dx > 1e-10 && dy > 1e-10) {
                S.omega = exp(0.5 * log(dy / dx) + 0.5 * log(S.omega));
                S.t = S.eta / S.omega;
                S.s = S.eta * S.omega;
            }
            S.Er = E;
            S.kr = k;
            S.restarts += 1;
            S.restart_now = 1;
            S.take_avg = use_avg;
        }
    }
    S.Ep = E;
    const int64_t left = S.k_limit - k;
    S.nrun = (int32_t)(left < (int64_t)R ? left : (int64_t)R);
}


// One workgroup per instance: fixed-order FP64 reduction of the check
// partials, then termination (Section 2.2), restart and primal-weight
// update, all in FP64.
__global__ __launch_bounds__(256) void k_decide(const DecideArgs d)
{
    const int inst = blockIdx.x;
    InstState &S = d.st[inst];
    if (S.status != ST_RUN) return;
    const InstInfo I = d.info[inst];
    __shared__ double red[4];
    // tot layout as in decide_state: rows {0, 1, 2} and {7, 8, 9}, columns
    // {3, 4, 5, 6} and {10, 11, 12, 13}
    double acc[NTOT] = {};
    auto row_add = [&](const double *q) {
        for (int k = 0; k < 3; ++k) acc[k] += q[k];
        for (int k = 0; k < 3; ++k) acc[7 + k] += q[4 + k];
    };
    auto col_add = [&](const double *q) {
        for (int k = 0; k < 4; ++k) acc[3 + k] += q[k];
        for (int k = 0; k < 4; ++k) acc[10 + k] += q[4 + k];
    };
    for (int t = I.rt0 + threadIdx.x; t < I.rt1; t += 256) row_add(d.rpart + CHK * t);
    for (int t = I.lr0 + threadIdx.x; t < I.lr1; t += 256) row_add(d.lrpart + CHK * t);
    for (int t = I.ct0 + threadIdx.x; t < I.ct1; t += 256) col_add(d.cpart + CHK * t);
    for (int t = I.lc0 + threadIdx.x; t < I.lc1; t += 256) col_add(d.lcpart + CHK * t);
    double tot[NTOT], tot2[NTOT];
    for (int k = 0; k < NTOT; ++k) {
        __syncthreads();
        tot[k] = block_sum<double, 256>(acc[k], red);
    }
    if (d.rpart2) {
        // the same reduction over the running average's check
        for (int k = 0; k < NTOT; ++k) acc[k] = 0.0;
        for (int t = I.rt0 + threadIdx.x; t < I.rt1; t += 256) row_add(d.rpart2 + CHK * t);
        for (int t = I.lr0 + threadIdx.x; t < I.lr1; t += 256) row_add(d.lrpart2 + CHK * t);
        for (int t = I.ct0 + threadIdx.x; t < I.ct1; t += 256) col_add(d.cpart2 + CHK * t);
        for (int t = I.lc0 + threadIdx.x; t < I.lc1; t += 256) col_add(d.lcpart2 + CHK * t);
        for (int k = 0; k < NTOT; ++k) {
            __syncthreads();
            tot2[k] = block_sum<double, 256>(acc[k], red);
        }
    }
    if (threadIdx.x != 0) return;
    decide_state(S, tot, d.rpart2 ? tot2 : nullptr, d.R);
}

// ------------------------------------------------------- adaptive steps
// Step-size rule after the k-th iteration (k counted from 1 over the call),
// in FP64 (Algorithm 1's step-size update, read as PDLP's adaptive rule
// without retries): eta_bar = (omega |dx~|^2 + |dy~|^2 / omega) / (2 |dy^T A dx|),
// eta <- min((1 - (k+1)^-0.3) eta_bar, (1 + (k+1)^-0.6) eta); eta_bar is
// infinite when the interaction is 0, and eta is kept when the move is 0.
__device__ __forceinline__ void adapt_step(InstState &S, double nx, double ny, double inter, int64_t k)
{
    if (!(nx + ny > 0.0)) return;
    const double grow = (1.0 + pow((double)k + 1.0, -0.6)) * S.eta;
    double eta = grow;
    if (inter != 0.0) {
        const double ebar = (S.omega * nx + ny / S.omega) / (2.0 * fabs(inter));
        const double shrink = (1.0 - pow((double)k + 1.0, -0.3)) * ebar;
        eta = shrink < grow ? shrink : grow;
    }
    S.eta = eta;
    S.t = eta / S.omega;
    S.s = eta * S.omega;
}

// One workgroup per instance: fixed-order FP64 sums of the iteration
// partials of both passes (slot ranges in InstInfo::ir), then the rule.
// Each thread issues its loads in groups of STEP_U before adding them, so
// an instance with thousands of tiles is not bound by load latency.
constexpr int STEP_NT = 1024, STEP_U = 8;

__device__ __forceinline__ void step_sum(const double *ip, int lo, int hi, int comp, double &acc)
{
    for (int q0 = lo + (int)threadIdx.x; q0 < hi; q0 += STEP_NT * STEP_U) {
        double v[STEP_U];
#pragma unroll
        for (int u = 0; u < STEP_U; ++u) {
            const int q = q0 + u * STEP_NT;
            v[u] = q < hi ? ip[2 * q + comp] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < STEP_U; ++u) acc += v[u];
    }
}

__global__ __launch_bounds__(STEP_NT) void k_step(const StepArgs a)
{
    __shared__ double red2[2 * STEP_NT / 64];
    const int inst = blockIdx.x;
    InstState &S = a.st[inst];
    if (S.status != ST_RUN || a.jw >= S.nrun) return;
    const InstInfo I = a.info[inst];
    double nx = 0.0, ny = 0.0, inter = 0.0;
    for (int r = 0; r < 3; ++r) {
        step_sum(a.cip, I.ir[1][r][0], I.ir[1][r][1], 0, nx);
        step_sum(a.rip, I.ir[0][r][0], I.ir[0][r][1], 0, ny);
        step_sum(a.rip, I.ir[0][r][0], I.ir[0][r][1], 1, inter);
    }
    double zero = 0.0;
    block_sum2<STEP_NT>(nx, zero, red2);
    block_sum2<STEP_NT>(ny, inter, red2);
    if (threadIdx.x == 0) adapt_step(S, nx, ny, inter, S.k + a.jw + 1);
}

// --------------------------------------------- fused window (tiny instances)
// One workgroup per instance runs a whole check window -- FP64 KKT check,
// decision, then up to R iterations -- with the instance's matrix (both
// orientations, decoded to local index + value) and vectors held in LDS and
// workgroup barriers between the passes.  Used when every instance of the
// handle fits in LDS; it removes the per-pass launch latency that dominates
// such instances.  No workgroup ever waits for another.
template <class V>
struct TinyLds {
    int *rptr, *cptr, *rcol, *ccol;
    V *rval, *cval, *x, *xb, *xr, *c, *l, *u, *dc2, *q, *y, *yr, *b, *dr2;
    double *ax;
    uint8_t *sense;
};

template <class V>
__device__ __forceinline__ TinyLds<V> tiny_carve(unsigned char *base, int m, int n, int rnnz, int cnnz)
{
    TinyLds<V> t;
    unsigned char *q = base;
    auto take = [&](size_t bytes) {
        unsigned char *p = q;
        q += (bytes + 15) & ~(size_t)15;
        return p;
    };
    t.rptr = (int *)take(4 * (size_t)(m + 1));
    t.cptr = (int *)take(4 * (size_t)(n + 1));
    t.rcol = (int *)take(4 * (size_t)rnnz);
    t.ccol = (int *)take(4 * (size_t)cnnz);
    t.rval = (V *)take(sizeof(V) * (size_t)rnnz);
    t.cval = (V *)take(sizeof(V) * (size_t)cnnz);
    t.x = (V *)take(sizeof(V) * (size_t)n);
    t.xb = (V *)take(sizeof(V) * (size_t)n);
    t.xr = (V *)take(sizeof(V) * (size_t)n);
    t.c = (V *)take(sizeof(V) * (size_t)n);
    t.l = (V *)take(sizeof(V) * (size_t)n);
    t.u = (V *)take(sizeof(V) * (size_t)n);
    t.dc2 = (V *)take(sizeof(V) * (size_t)n);
    t.q = (V *)take(sizeof(V) * (size_t)n);
    t.y = (V *)take(sizeof(V) * (size_t)m);
    t.yr = (V *)take(sizeof(V) * (size_t)m);
    t.b = (V *)take(sizeof(V) * (size_t)m);
    t.dr2 = (V *)take(sizeof(V) * (size_t)m);
    t.ax = (double *)take(8 * (size_t)m);
    t.sense = (uint8_t *)take((size_t)m);
    return t;
}

template <class V, int FMT>
__global__ __launch_bounds__(1024) void k_tiny(const TinyArgs<V> a, const int R)
{
    constexpr int NT = 1024;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red[NT / 64];
    __shared__ double red2[2 * NT / 64];
    __shared__ int sh_nrun, sh_restart;
    __shared__ V sh_t, sh_s;
    const int inst = blockIdx.x, tid = threadIdx.x;
    InstState &S = a.st[inst];
    if (S.status != ST_RUN) return;
    const InstInfo I = a.info[inst];
    const int m = I.row1 - I.row0, n = I.col1 - I.col0;
    const int re0 = a.R.ptr[I.row0], rnnz = a.R.ptr[I.row1] - re0;
    const int ce0 = a.C.ptr[I.col0], cnnz = a.C.ptr[I.col1] - ce0;
    const TinyLds<V> L = tiny_carve<V>(lds_raw, m, n, rnnz, cnnz);
    // ---- load the instance into LDS
    for (int i = tid; i <= m; i += NT) L.rptr[i] = a.R.ptr[I.row0 + i] - re0;
    for (int j = tid; j <= n; j += NT) L.cptr[j] = a.C.ptr[I.col0 + j] - ce0;
    for (int e = tid; e < rnnz; e += NT) {
        uint32_t w;
        V v;
        load_entry<FMT, V>(a.R, re0 + e, w, v);
        L.rcol[e] = decode_entry<FMT, V>(a.R, w, v) - I.col0;
        L.rval[e] = v;
    }
    for (int e = tid; e < cnnz; e += NT) {
        uint32_t w;
        V v;
        load_entry<FMT, V>(a.C, ce0 + e, w, v);
        L.ccol[e] = decode_entry<FMT, V>(a.C, w, v) - I.row0;
        L.cval[e] = v;
    }
    for (int j = tid; j < n; j += NT) {
        const int g = I.col0 + j;
        L.x[j] = a.x[g];
        L.xb[j] = a.xbar[g];
        L.xr[j] = a.xr[g];
        L.c[j] = a.c[g];
        L.l[j] = a.l[g];
        L.u[j] = a.u[g];
        L.dc2[j] = a.dc2[g];
        L.q[j] = a.q ? a.q[g] : (V)0;
    }
    for (int i = tid; i < m; i += NT) {
        const int g = I.row0 + i;
        L.y[i] = a.y[g];
        L.yr[i] = a.yr[g];
        L.b[i] = a.b[g];
        L.dr2[i] = a.dr2[g];
        L.sense[i] = a.sense[g];
    }
    __syncthreads();
    // ---- FP64 KKT check of the current point (Section 2.2)
    double acc[NTOT] = {};
    for (int i = tid; i < m; i += NT) {
        double ax = 0.0;
        for (int e = L.rptr[i]; e < L.rptr[i + 1]; ++e) ax += (double)L.rval[e] * (double)L.x[L.rcol[e]];
        const double bb = a.b64[I.row0 + i];
        const uint8_t sn = L.sense[i];
        double r;
        if (sn == 'G') r = fmax(bb - ax, 0.0);
        else if (sn == 'L') r = fmax(ax - bb, 0.0);
        else r = bb - ax;
        const double yy = (double)L.y[i];
        const double dy = (yy - (double)L.yr[i]) / a.dr64[I.row0 + i];
        L.ax[i] = ax;  // A x of the current point in FP64 (adaptive steps)
        acc[0] += r * r;
        acc[1] += bb * yy;
        acc[2] += dy * dy;
        // moves since the previous check (infeasibility certificates)
        const int gi = I.row0 + i;
        const double v = yy - (double)a.yp[gi];
        const double vp = sn == 'G' ? fmax(v, 0.0) : (sn == 'L' ? fmin(v, 0.0) : v);
        const double ad = ax - a.axp[gi];
        const double viol = sn == 'G' ? fmax(-ad, 0.0) : (sn == 'L' ? fmax(ad, 0.0) : ad);
        acc[7] += bb * v;
        acc[8] += (v - vp) * (v - vp);
        acc[9] += viol * viol;
        a.yp[gi] = L.y[i];
        a.axp[gi] = ax;
    }
    for (int j = tid; j < n; j += NT) {
        double aty = 0.0;
        for (int e = L.cptr[j]; e < L.cptr[j + 1]; ++e) aty += (double)L.cval[e] * (double)L.y[L.ccol[e]];
        const int g = I.col0 + j;
        const double cc = a.c64[g], lo = a.l64[g], hi = a.u64[g];
        const double xq = (double)L.x[j];
        const double qx = a.q64 ? a.q64[g] * xq : 0.0;
        const double gr = cc + qx - aty;
        const bool lf = isfinite(lo), uf = isfinite(hi);
        double lam;
        if (lf && uf) lam = gr;
        else if (lf) lam = fmax(gr, 0.0);
        else if (uf) lam = fmin(gr, 0.0);
        else lam = 0.0;
        const double rd = gr - lam;
        const double dx = (xq - (double)L.xr[j]) / a.dc64[g];
        acc[3] += rd * rd;
        acc[4] += cc * xq + 0.5 * qx * xq;
        if (lf && lam > 0.0) acc[5] += lo * lam;
        if (uf && lam < 0.0) acc[5] += hi * lam;
        acc[5] -= 0.5 * qx * xq;
        acc[6] += dx * dx;
        const double w = aty - a.atyp[g];
        double rl;
        if (lf && uf) rl = -w;
        else if (lf) rl = fmax(-w, 0.0);
        else if (uf) rl = fmin(-w, 0.0);
        else rl = 0.0;
        acc[10] += (w + rl) * (w + rl);
        if (lf && rl > 0.0) acc[11] += lo * rl;
        if (uf && rl < 0.0) acc[11] += hi * rl;
        const double d = xq - (double)a.xp[g];
        acc[12] += cc * d;
        double bv;
        if (lf && uf) bv = d;
        else if (lf) bv = fmin(d, 0.0);
        else if (uf) bv = fmax(d, 0.0);
        else bv = 0.0;
        acc[13] += bv * bv;
        if (a.q64) acc[13] += (a.q64[g] * d) * (a.q64[g] * d);
        a.xp[g] = L.x[j];
        a.atyp[g] = aty;
    }
    double tot[NTOT];
    for (int k = 0; k < NTOT; ++k) {
        __syncthreads();
        tot[k] = block_sum<double, NT>(acc[k], red);
    }
    if (tid == 0) {
        decide_state(S, tot, nullptr, R);
        sh_nrun = S.status == ST_RUN ? S.nrun : 0;
        sh_restart = S.restart_now;
        sh_t = (V)S.t;
        sh_s = (V)S.s;
    }
    __syncthreads();
    const int nrun = sh_nrun;
    if (nrun == 0) return;
    V t = sh_t, sd = sh_s;
    // lane groups: a power of two of lanes per column / row, as many as fit
    const int Lc = lanes_per_row<NT>(n), Lr = lanes_per_row<NT>(m);
    const int lc = tid & (Lc - 1), lr = tid & (Lr - 1);
    // ---- nrun PDHG iterations (Algorithm 1): column pass, barrier, row pass
    for (int it = 0; it < nrun; ++it) {
        const bool copy_ref = it == 0 && sh_restart != 0;
        double nx = 0.0, ny = 0.0, inter = 0.0;
        for (int j = tid / Lc; j < n; j += NT / Lc) {
            V aty = 0;
            for (int e = L.cptr[j] + lc; e < L.cptr[j + 1]; e += Lc) aty += L.cval[e] * L.y[L.ccol[e]];
            if (Lc > 1) aty = wave_sum_width(aty, Lc);
            if (lc == 0) {
                const V xj = L.x[j];
                V xn = xj + t * L.dc2[j] * (aty - L.c[j]);
                if (a.q) xn /= (V)1 + t * L.dc2[j] * L.q[j];
                xn = xn < L.l[j] ? L.l[j] : xn;
                xn = xn > L.u[j] ? L.u[j] : xn;
                if (copy_ref) L.xr[j] = xj;
                L.xb[j] = a.adapt ? xn - xj : (V)2 * xn - xj;  // adaptive: the move dx
                L.x[j] = xn;
                if (a.adapt) {
                    const double d = (double)xn - (double)xj;
                    nx += d * d / (double)L.dc2[j];
                }
            }
        }
        __syncthreads();
        for (int i = tid / Lr; i < m; i += NT / Lr) {
            V axb = 0;
            for (int e = L.rptr[i] + lr; e < L.rptr[i + 1]; e += Lr) axb += L.rval[e] * L.xb[L.rcol[e]];
            if (Lr > 1) axb = wave_sum_width(axb, Lr);
            if (lr == 0) {
                const V yi = L.y[i];
                // adaptive: axb = (A dx)_i and (A x_bar)_i = (A x)_i + 2 (A dx)_i
                const V res = a.adapt ? (V)((double)L.b[i] - (L.ax[i] + 2.0 * (double)axb)) : L.b[i] - axb;
                V v = yi + sd * L.dr2[i] * res;
                const uint8_t sn = L.sense[i];
                if (sn == 'G') v = v > (V)0 ? v : (V)0;
                else if (sn == 'L') v = v < (V)0 ? v : (V)0;
                if (copy_ref) L.yr[i] = yi;
                L.y[i] = v;
                if (a.adapt) {
                    const double dy = (double)v - (double)yi;
                    ny += dy * dy / (double)L.dr2[i];
                    inter += dy * (double)axb;
                    L.ax[i] += (double)axb;
                }
            }
        }
        __syncthreads();
        if (a.adapt) {
            double zero = 0.0;
            block_sum2<NT>(nx, zero, red2);
            block_sum2<NT>(ny, inter, red2);
            if (tid == 0) {
                adapt_step(S, nx, ny, inter, S.k + it + 1);
                sh_t = (V)S.t;
                sh_s = (V)S.s;
            }
            __syncthreads();
            t = sh_t;
            sd = sh_s;
        }
    }
    // ---- write the iterates back
    for (int j = tid; j < n; j += NT) {
        const int g = I.col0 + j;
        a.x[g] = L.x[j];
        a.xbar[g] = L.xb[j];
        a.xr[g] = L.xr[j];
    }
    for (int i = tid; i < m; i += NT) {
        const int g = I.row0 + i;
        a.y[g] = L.y[i];
        a.yr[g] = L.yr[i];
    }
}

template <class V>
void launch_tiny(const TinyArgs<V> &a, int fmt, int count, int R, size_t shmem, hipStream_t s, bool prepare)
{
    auto run = [&](auto fn) {
        if (prepare) (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)shmem);
        else hipLaunchKernelGGL(fn, dim3(count), dim3(1024), shmem, s, a, R);
    };
    if constexpr (sizeof(V) == 8) {
        run(k_tiny<V, FMT_F64>);
    } else {
        if (fmt == FMT_PACKED) run(k_tiny<V, FMT_PACKED>);
        else if (fmt == FMT_BF16) run(k_tiny<V, FMT_BF16>);
        else run(k_tiny<V, FMT_F32>);
    }
}

// Restart to the average: one workgroup per instance copies the running
// mean over the iterate where the decision took it (restart, OPTIMAL or
// iteration-limit stop), then clears the flag.  The restart reference is
// copied from the new iterate by the next iteration, as for any restart.
template <class V>
__global__ __launch_bounds__(256) void k_take_avg(InstState *st, const InstInfo *info, V *x, V *y, const V *xa,
                                                  const V *ya, double *ax, const double *axa)
{
    const int inst = blockIdx.x;
    if (!st[inst].take_avg) return;
    const InstInfo I = info[inst];
    for (int j = I.col0 + threadIdx.x; j < I.col1; j += 256) x[j] = xa[j];
    for (int i = I.row0 + threadIdx.x; i < I.row1; i += 256) {
        y[i] = ya[i];
        if (ax) ax[i] = axa[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) st[inst].take_avg = 0;
}

__global__ void k_force_stop(InstState *st, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && st[i].status == ST_RUN) st[i].force_stop = 1;
}

// ---------------------------------------------------------------- setup
// Preconditioner reductions over one orientation (one wave per row):
// mode 0: r_i = max_j |d_r,i a_ij d_c,j|;  mode 1: r_i = sum_j |...|.
// `drow` scales the rows of this orientation, `dcol` the columns.
template <int FMT>
__global__ __launch_bounds__(256) void k_scale_reduce(const MatView M, int rows, const double *drow,
                                                      const double *dcol, double *out, int mode)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const int e0 = M.ptr[row], e1 = M.ptr[row + 1];
    double acc = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
        uint32_t w;
        double a;
        load_entry<FMT, double>(M, e, w, a);
        const int idx = decode_entry<FMT, double>(M, w, a);
        const double v = fabs(drow[row] * a * dcol[idx]);
        acc = mode == 0 ? fmax(acc, v) : acc + v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(acc, off, 64);
        acc = mode == 0 ? fmax(acc, o) : acc + o;
    }
    if (lane == 0) out[row] = acc;
}

__global__ void k_scale_apply(double *d, const double *r, int len)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len && r[i] > 0.0) d[i] /= sqrt(r[i]);
}

// Per-instance norms of the current objective c_hat and of b: ||b||,
// ||c_hat||, and the cold-start primal weight ||D_c c_hat|| / ||D_r b|| (or 1).
__global__ __launch_bounds__(256) void k_inst_norms(const InstInfo *info, const double *b,
                                                    const double *c, const double *dr,
                                                    const double *dc, InstState *st)
{
    const int inst = blockIdx.x;
    const InstInfo I = info[inst];
    __shared__ double red[4];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int i = I.row0 + threadIdx.x; i < I.row1; i += 256) {
        a0 += b[i] * b[i];
        const double v = dr[i] * b[i];
        a1 += v * v;
    }
    for (int j = I.col0 + threadIdx.x; j < I.col1; j += 256) {
        a2 += c[j] * c[j];
        const double v = dc[j] * c[j];
        a3 += v * v;
    }
    const double s0 = block_sum<double, 256>(a0, red);
    __syncthreads();
    const double s1 = block_sum<double, 256>(a1, red);
    __syncthreads();
    const double s2 = block_sum<double, 256>(a2, red);
    __syncthreads();
    const double s3 = block_sum<double, 256>(a3, red);
    if (threadIdx.x == 0) {
        InstState &S = st[inst];
        S.cnorm = sqrt(s2);
        S.bnorm = sqrt(s0);
        const double bs = sqrt(s1), cs = sqrt(s3);
        S.omega0 = (cs > 0.0 && bs > 0.0) ? cs / bs : 1.0;
    }
}

template <class V>
__global__ void k_finish_diag(const double *d, V *d2, int len)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) d2[i] = (V)(d[i] * d[i]);
}

template <class V>
__global__ void k_cast(const double *src, V *dst, int len)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) dst[i] = (V)src[i];
}

// Start point: x = proj_[l,u](x), y = proj_Y(y) on [lo, hi) ranges; zero
// first when `zero` is set.
template <class V>
__global__ void k_project_primal(V *x, const V *l, const V *u, int lo, int hi, int zero)
{
    const int j = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= hi) return;
    V v = zero ? (V)0 : x[j];
    v = v < l[j] ? l[j] : v;
    v = v > u[j] ? u[j] : v;
    x[j] = v;
}

// flag |= 1 if some x[j] is NaN, |= 2 if some y[i] is not finite (a warm
// start read from device memory is checked before anything is written).
__global__ void k_start_check(const double *x, int n, const double *y, int m, int *flag)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    int bad = 0;
    if (x && k < n && isnan(x[k])) bad |= 1;
    if (y && k < m && !isfinite(y[k])) bad |= 2;
    if (bad) atomicOr(flag, bad);
}

void launch_start_check(const double *x, int n, const double *y, int m, int *flag, hipStream_t s)
{
    const int nx = x ? n : 0, ny = y ? m : 0, len = nx > ny ? nx : ny;
    if (len > 0) hipLaunchKernelGGL(k_start_check, dim3((len + 255) / 256), dim3(256), 0, s, x, n, y, m, flag);
}

template <class V>
__global__ void k_project_dual(V *y, const uint8_t *sense, int lo, int hi, int zero)
{
    const int i = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= hi) return;
    V v = zero ? (V)0 : y[i];
    const uint8_t sn = sense[i];
    if (sn == 'G') v = v > (V)0 ? v : (V)0;
    else if (sn == 'L') v = v < (V)0 ? v : (V)0;
    y[i] = v;
}

// Pump objective (Algorithm 1, objective update) on columns [lo, hi):
// c_hat_j = a kappa c_j + (1 - a) g_j, g_j = +1 / -1 from the rounding bit,
// 0 for continuous columns.
template <class V>
__global__ void k_blend(const double *c_orig, const uint8_t *xbits, const uint8_t *ibits, double a,
                        double kappa, double *c64, V *cv, int lo, int hi)
{
    const int j = lo + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= hi) return;
    const int q = j - lo;
    const bool integer = ibits ? ((ibits[q >> 3] >> (q & 7)) & 1) : true;
    const bool up = (xbits[q >> 3] >> (q & 7)) & 1;
    const double g = integer ? (up ? -1.0 : 1.0) : 0.0;
    const double v = a * kappa * c_orig[j] + (1.0 - a) * g;
    c64[j] = v;
    cv[j] = (V)v;
}

// ------------------------------------------------ MIP feasibility
// Algorithm 1 tests the PDHG point itself before rounding it: x is
// MIP-feasible when every row holds within tol (1 + |b_i|), every x_j lies
// within tol of [l_j, u_j] and every integer x_j within tol of an integer.
// Row activities are FP64 sums of a_ij x_j (16 lanes per row); a
// non-finite value counts as a violation.  Flags: 1 = violated.
template <class V, int FMT>
__global__ __launch_bounds__(256) void k_mip_rows(const MatView M, int rows, const V *__restrict__ x,
                                                  const double *__restrict__ b, const uint8_t *__restrict__ sense,
                                                  double tol, uint8_t *__restrict__ bad)
{
    const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
    const int lane = threadIdx.x & 15;
    // whole 16-lane groups leave together, so the shuffles below only
    // involve lanes that are still running
    if (row >= rows) return;
    const int e1 = M.ptr[row + 1];
    double acc = 0.0;
    for (int e = M.ptr[row] + lane; e < e1; e += 16) {
        uint32_t w;
        double a;
        load_entry<FMT, double>(M, e, w, a);
        const int j = decode_entry<FMT, double>(M, w, a);
        acc += a * (double)x[j];
    }
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (lane == 0) {
        const double bi = b[row], t = tol * (1.0 + fabs(bi));
        const uint8_t sn = sense[row];
        bool ok = isfinite(acc);
        if (sn != 'L') ok = ok && acc >= bi - t;
        if (sn != 'G') ok = ok && acc <= bi + t;
        bad[row] = ok ? 0 : 1;
    }
}

template <class V>
__global__ void k_mip_cols(const V *__restrict__ x, const double *__restrict__ l, const double *__restrict__ u,
                           const uint8_t *__restrict__ is_int, double tol, int n, uint8_t *__restrict__ bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double v = (double)x[j];
    bool ok = v >= l[j] - tol && v <= u[j] + tol;
    if (is_int[j]) ok = ok && fabs(v - rint(v)) <= tol;
    bad[j] = ok ? 0 : 1;
}

// One workgroup per instance: feasible[inst] = no violated row or column.
__global__ __launch_bounds__(256) void k_mip_reduce(const InstInfo *__restrict__ info, const uint8_t *__restrict__ rbad,
                                                    const uint8_t *__restrict__ cbad, uint8_t *__restrict__ feasible)
{
    const InstInfo I = info[blockIdx.x];
    int any = 0;
    for (int i = I.row0 + threadIdx.x; i < I.row1; i += 256) any |= rbad[i];
    for (int j = I.col0 + threadIdx.x; j < I.col1; j += 256) any |= cbad[j];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) feasible[blockIdx.x] = any ? 0 : 1;
}

// ------------------------------------------------------ host launchers
template <class V, int FMT, int DIR, int NT, int EPT>
static void launch_pass_t(const PassArgs<V> &p, int jw, hipStream_t s)
{
    hipLaunchKernelGGL((k_pass<V, FMT, DIR, NT, EPT>), dim3(p.ntiles), dim3(NT), 0, s, p, jw);
}

template <class V, int FMT, int DIR, int NT, int EPT>
static void launch_check_t(const PassArgs<V> &p, hipStream_t s)
{
    hipLaunchKernelGGL((k_check<V, FMT, DIR, NT, EPT>), dim3(p.ntiles), dim3(NT), 0, s, p);
}

// ept: nonzeros per thread of 256-thread tile workgroups (tiles of 256 ept
// nonzeros); -8 / -16: the tiles of ept 8 / 16 run by 1024-thread
// workgroups, 2 / 4 nonzeros per thread (a thread then has at most one row
// of a tile).
template <class V, int FMT, int DIR>
static void dispatch_pass(const PassArgs<V> &p, int ept, int jw, bool check, hipStream_t s)
{
    switch (ept) {
    case -8:
        check ? launch_check_t<V, FMT, DIR, 1024, 2>(p, s) : launch_pass_t<V, FMT, DIR, 1024, 2>(p, jw, s);
        break;
    case -16:
        check ? launch_check_t<V, FMT, DIR, 1024, 4>(p, s) : launch_pass_t<V, FMT, DIR, 1024, 4>(p, jw, s);
        break;
    case 2:
        check ? launch_check_t<V, FMT, DIR, 256, 2>(p, s) : launch_pass_t<V, FMT, DIR, 256, 2>(p, jw, s);
        break;
    case 4:
        check ? launch_check_t<V, FMT, DIR, 256, 4>(p, s) : launch_pass_t<V, FMT, DIR, 256, 4>(p, jw, s);
        break;
    case 8:
        check ? launch_check_t<V, FMT, DIR, 256, 8>(p, s) : launch_pass_t<V, FMT, DIR, 256, 8>(p, jw, s);
        break;
    default:
        check ? launch_check_t<V, FMT, DIR, 256, 16>(p, s) : launch_pass_t<V, FMT, DIR, 256, 16>(p, jw, s);
        break;
    }
}

template <class V, class A, int FMT>
static void dispatch_bpart(const PassArgs<V> &p, int ept, int jw, int check, hipStream_t s)
{
    const dim3 g(p.ntiles), b(256);
    switch (ept) {
    case -8: hipLaunchKernelGGL((k_bpart<V, A, FMT, 1024, 2>), g, dim3(1024), 0, s, p, jw, check); break;
    case -16: hipLaunchKernelGGL((k_bpart<V, A, FMT, 1024, 4>), g, dim3(1024), 0, s, p, jw, check); break;
    case 2: hipLaunchKernelGGL((k_bpart<V, A, FMT, 256, 2>), g, b, 0, s, p, jw, check); break;
    case 4: hipLaunchKernelGGL((k_bpart<V, A, FMT, 256, 4>), g, b, 0, s, p, jw, check); break;
    case 8: hipLaunchKernelGGL((k_bpart<V, A, FMT, 256, 8>), g, b, 0, s, p, jw, check); break;
    default: hipLaunchKernelGGL((k_bpart<V, A, FMT, 256, 16>), g, b, 0, s, p, jw, check); break;
    }
}

// Calls f(std::integral_constant<int, F>{}) with F the FP32 storage format
// fmt, with or without the FMT_CACHED flag.
template <class Fn>
static void fp32_format(int fmt, Fn &&f)
{
    const bool c = (fmt & FMT_CACHED) != 0;
    switch (fmt & ~FMT_CACHED) {
    case FMT_PACKED:
        if (c) f(std::integral_constant<int, FMT_PACKED | FMT_CACHED>{});
        else f(std::integral_constant<int, FMT_PACKED>{});
        break;
    case FMT_BF16:
        if (c) f(std::integral_constant<int, FMT_BF16 | FMT_CACHED>{});
        else f(std::integral_constant<int, FMT_BF16>{});
        break;
    default:
        if (c) f(std::integral_constant<int, FMT_F32 | FMT_CACHED>{});
        else f(std::integral_constant<int, FMT_F32>{});
        break;
    }
}

template <class V, class A>
static void bpart_fmt(const PassArgs<V> &p, int fmt, int ept, int jw, int check, hipStream_t s)
{
    if constexpr (sizeof(V) == 8) {
        dispatch_bpart<V, A, FMT_F64>(p, ept, jw, check, s);
    } else {
        fp32_format(fmt, [&](auto fc) { dispatch_bpart<V, A, decltype(fc)::value>(p, ept, jw, check, s); });
    }
}

template <class V>
void launch_pass(const PassArgs<V> &p, int fmt, int dir, int ept, int jw, bool check, bool blocked, hipStream_t s)
{
    if (blocked) {
        if (p.ntiles > 0) {
            if (check) bpart_fmt<V, double>(p, fmt, ept, jw, 1, s);
            else bpart_fmt<V, V>(p, fmt, ept, jw, 0, s);
        }
        if (p.nlong > 0) {
            const int nb = (p.nlong + 255) / 256;
            if (check) hipLaunchKernelGGL((k_bseg<V, double>), dim3(nb), dim3(256), 0, s, p, jw, 1);
            else hipLaunchKernelGGL((k_bseg<V, V>), dim3(nb), dim3(256), 0, s, p, jw, 0);
        }
        if (p.nctiles > 0) {
            const dim3 g(p.nctiles), b(256);
            if (check) {
                if (dir == DIR_COL) hipLaunchKernelGGL((k_bcombine_check<V, DIR_COL>), g, b, 0, s, p);
                else hipLaunchKernelGGL((k_bcombine_check<V, DIR_ROW>), g, b, 0, s, p);
            } else {
                if (dir == DIR_COL) hipLaunchKernelGGL((k_bcombine<V, DIR_COL>), g, b, 0, s, p, jw);
                else hipLaunchKernelGGL((k_bcombine<V, DIR_ROW>), g, b, 0, s, p, jw);
            }
        }
        return;
    }
    if (p.ntiles > 0) {
        if constexpr (sizeof(V) == 8) {
            if (dir == DIR_COL) dispatch_pass<V, FMT_F64, DIR_COL>(p, ept, jw, check, s);
            else dispatch_pass<V, FMT_F64, DIR_ROW>(p, ept, jw, check, s);
        } else {
            fp32_format(fmt, [&](auto fc) {
                constexpr int F = decltype(fc)::value;
                if (dir == DIR_COL) dispatch_pass<V, F, DIR_COL>(p, ept, jw, check, s);
                else dispatch_pass<V, F, DIR_ROW>(p, ept, jw, check, s);
            });
        }
    }
    if (p.nlong > 0) {
        const int nb = (p.nlong + 255) / 256;
        if (check) {
            if (dir == DIR_COL) hipLaunchKernelGGL((k_combine_check<V, DIR_COL>), dim3(nb), dim3(256), 0, s, p);
            else hipLaunchKernelGGL((k_combine_check<V, DIR_ROW>), dim3(nb), dim3(256), 0, s, p);
        } else {
            if (dir == DIR_COL) hipLaunchKernelGGL((k_combine<V, DIR_COL>), dim3(nb), dim3(256), 0, s, p, jw);
            else hipLaunchKernelGGL((k_combine<V, DIR_ROW>), dim3(nb), dim3(256), 0, s, p, jw);
        }
    }
}

template <class V, int FMT, int DIR, int EPT, bool PF>
static void staged_v(const PassArgs<V> &p, int jw, size_t shmem, hipStream_t s, bool prepare)
{
    auto fn = k_spass<V, FMT, DIR, SPASS_NT, EPT, PF>;
    if (prepare) {
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        return;
    }
    hipLaunchKernelGGL(fn, dim3(p.ntiles), dim3(SPASS_NT), shmem, s, p, jw);
}

template <class V, int FMT, int DIR>
static void staged_t(const PassArgs<V> &p, int variant, int jw, size_t shmem, hipStream_t s, bool prepare)
{
    // variant bits: 1 = prefetch row bounds and operands, 2 = 8 nonzeros per
    // thread (else 4)
    switch (variant & 3) {
    case 0: staged_v<V, FMT, DIR, 4, false>(p, jw, shmem, s, prepare); break;
    case 1: staged_v<V, FMT, DIR, 4, true>(p, jw, shmem, s, prepare); break;
    case 2: staged_v<V, FMT, DIR, 8, false>(p, jw, shmem, s, prepare); break;
    default: staged_v<V, FMT, DIR, 8, true>(p, jw, shmem, s, prepare); break;
    }
}

template <class V>
void launch_staged(const PassArgs<V> &p, int fmt, int dir, int variant, int jw, size_t shmem, hipStream_t s,
                   bool prepare)
{
    if (!prepare && p.ntiles <= 0) return;
    if constexpr (sizeof(V) == 8) {
        if (dir == DIR_COL) staged_t<V, FMT_F64, DIR_COL>(p, variant, jw, shmem, s, prepare);
        else staged_t<V, FMT_F64, DIR_ROW>(p, variant, jw, shmem, s, prepare);
    } else {
        fp32_format(fmt, [&](auto fc) {
            constexpr int F = decltype(fc)::value;
            if (dir == DIR_COL) staged_t<V, F, DIR_COL>(p, variant, jw, shmem, s, prepare);
            else staged_t<V, F, DIR_ROW>(p, variant, jw, shmem, s, prepare);
        });
    }
}

template <class V, int FMT, int DIR, int K>
void direct_k(const PassArgs<V> &p, int jw, size_t shmem, hipStream_t s, bool prepare)
{
    auto fn = k_dpass<V, FMT, DIR, DPASS_NT, K>;
    if (prepare) {
        (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        return;
    }
    hipLaunchKernelGGL(fn, dim3(p.ndtiles), dim3(DPASS_NT), shmem, s, p, jw);
}

template <class V, int FMT, int DIR>
void direct_t(const PassArgs<V> &p, int k, int jw, size_t shmem, hipStream_t s, bool prepare)
{
    if (k <= 2) direct_k<V, FMT, DIR, 2>(p, jw, shmem, s, prepare);
    else if (k <= 4) direct_k<V, FMT, DIR, 4>(p, jw, shmem, s, prepare);
    else direct_k<V, FMT, DIR, 8>(p, jw, shmem, s, prepare);
}

template <class V>
void launch_direct(const PassArgs<V> &p, int fmt, int dir, int k, int jw, size_t shmem, hipStream_t s,
                   bool prepare)
{
    if (!prepare && p.ndtiles <= 0) return;
    if constexpr (sizeof(V) == 8) {
        if (dir == DIR_COL) direct_t<V, FMT_F64, DIR_COL>(p, k, jw, shmem, s, prepare);
        else direct_t<V, FMT_F64, DIR_ROW>(p, k, jw, shmem, s, prepare);
    } else {
        fp32_format(fmt, [&](auto fc) {
            constexpr int F = decltype(fc)::value;
            if (dir == DIR_COL) direct_t<V, F, DIR_COL>(p, k, jw, shmem, s, prepare);
            else direct_t<V, F, DIR_ROW>(p, k, jw, shmem, s, prepare);
        });
    }
}

template <class V>
void launch_combine(const PassArgs<V> &p, int dir, int jw, hipStream_t s)
{
    if (p.nctiles <= 0) return;
    const dim3 g(p.nctiles), b(256);
    if (dir == DIR_COL) hipLaunchKernelGGL((k_bcombine<V, DIR_COL>), g, b, 0, s, p, jw);
    else hipLaunchKernelGGL((k_bcombine<V, DIR_ROW>), g, b, 0, s, p, jw);
}

void launch_step(const StepArgs &a, int count, hipStream_t s)
{
    if (count > 0) hipLaunchKernelGGL(k_step, dim3(count), dim3(STEP_NT), 0, s, a);
}

void launch_decide(const DecideArgs &d, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_decide, dim3(count), dim3(256), 0, s, d);
}

template <class V>
void launch_take_avg(InstState *st, const InstInfo *info, V *x, V *y, const V *xa, const V *ya, double *ax,
                     const double *axa, int count, hipStream_t s)
{
    if (count > 0) hipLaunchKernelGGL(k_take_avg<V>, dim3(count), dim3(256), 0, s, st, info, x, y, xa, ya, ax, axa);
}

void launch_force_stop(InstState *st, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_force_stop, dim3((count + 255) / 256), dim3(256), 0, s, st, count);
}

void launch_scale_reduce(const MatView &M, int fmt, int rows, const double *drow, const double *dcol,
                         double *out, int mode, hipStream_t s)
{
    if (rows <= 0) return;
    dim3 g((rows + 3) / 4), b(256);
    switch (fmt) {
    case FMT_PACKED: hipLaunchKernelGGL(k_scale_reduce<FMT_PACKED>, g, b, 0, s, M, rows, drow, dcol, out, mode); break;
    case FMT_BF16: hipLaunchKernelGGL(k_scale_reduce<FMT_BF16>, g, b, 0, s, M, rows, drow, dcol, out, mode); break;
    case FMT_F32: hipLaunchKernelGGL(k_scale_reduce<FMT_F32>, g, b, 0, s, M, rows, drow, dcol, out, mode); break;
    default: hipLaunchKernelGGL(k_scale_reduce<FMT_F64>, g, b, 0, s, M, rows, drow, dcol, out, mode); break;
    }
}

void launch_scale_apply(double *d, const double *r, int len, hipStream_t s)
{
    if (len > 0) hipLaunchKernelGGL(k_scale_apply, dim3((len + 255) / 256), dim3(256), 0, s, d, r, len);
}

void launch_inst_norms(const InstInfo *info, int count, const double *b, const double *c,
                       const double *dr, const double *dc, InstState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_inst_norms, dim3(count), dim3(256), 0, s, info, b, c, dr, dc, st);
}

template <class V>
void launch_finish_diag(const double *d, V *d2, int len, hipStream_t s)
{
    if (len > 0) hipLaunchKernelGGL(k_finish_diag<V>, dim3((len + 255) / 256), dim3(256), 0, s, d, d2, len);
}

template <class V>
void launch_cast(const double *src, V *dst, int len, hipStream_t s)
{
    if (len > 0) hipLaunchKernelGGL(k_cast<V>, dim3((len + 255) / 256), dim3(256), 0, s, src, dst, len);
}

template <class V>
void launch_project(V *x, const V *l, const V *u, int clo, int chi, V *y, const uint8_t *sense, int rlo,
                    int rhi, int zero, hipStream_t s)
{
    if (chi > clo)
        hipLaunchKernelGGL(k_project_primal<V>, dim3((chi - clo + 255) / 256), dim3(256), 0, s, x, l, u, clo, chi, zero);
    if (rhi > rlo)
        hipLaunchKernelGGL(k_project_dual<V>, dim3((rhi - rlo + 255) / 256), dim3(256), 0, s, y, sense, rlo, rhi, zero);
}

template <class V>
void launch_blend(const double *c_orig, const uint8_t *xbits, const uint8_t *ibits, double a, double kappa,
                  double *c64, V *cv, int lo, int hi, hipStream_t s)
{
    if (hi > lo)
        hipLaunchKernelGGL(k_blend<V>, dim3((hi - lo + 255) / 256), dim3(256), 0, s, c_orig, xbits, ibits, a,
                           kappa, c64, cv, lo, hi);
}

template <class V>
void launch_mip_check(const MatView &M, int fmt, int m, int n, int count, const InstInfo *info, const V *x,
                      const double *b, const uint8_t *sense, const double *l, const double *u,
                      const uint8_t *is_int, double tol, uint8_t *rbad, uint8_t *cbad, uint8_t *feasible,
                      hipStream_t s)
{
    if (m > 0) {
        dim3 g((m + 15) / 16), bl(256);
        if constexpr (sizeof(V) == 8) {
            hipLaunchKernelGGL((k_mip_rows<V, FMT_F64>), g, bl, 0, s, M, m, x, b, sense, tol, rbad);
        } else {
            switch (fmt) {
            case FMT_PACKED: hipLaunchKernelGGL((k_mip_rows<V, FMT_PACKED>), g, bl, 0, s, M, m, x, b, sense, tol, rbad); break;
            case FMT_BF16: hipLaunchKernelGGL((k_mip_rows<V, FMT_BF16>), g, bl, 0, s, M, m, x, b, sense, tol, rbad); break;
            default: hipLaunchKernelGGL((k_mip_rows<V, FMT_F32>), g, bl, 0, s, M, m, x, b, sense, tol, rbad); break;
            }
        }
    }
    if (n > 0)
        hipLaunchKernelGGL(k_mip_cols<V>, dim3((n + 255) / 256), dim3(256), 0, s, x, l, u, is_int, tol, n, cbad);
    if (count > 0) hipLaunchKernelGGL(k_mip_reduce, dim3(count), dim3(256), 0, s, info, rbad, cbad, feasible);
}

#define SCY_INST(V)                                                                                    \
    template void launch_tiny<V>(const TinyArgs<V> &, int, int, int, size_t, hipStream_t, bool);       \
    template void launch_staged<V>(const PassArgs<V> &, int, int, int, int, size_t, hipStream_t, bool); \
    template void launch_pass<V>(const PassArgs<V> &, int, int, int, int, bool, bool, hipStream_t);    \
    template void launch_combine<V>(const PassArgs<V> &, int, int, hipStream_t);                       \
    template void launch_direct<V>(const PassArgs<V> &, int, int, int, int, size_t, hipStream_t, bool); \
    template void launch_finish_diag<V>(const double *, V *, int, hipStream_t);                        \
    template void launch_take_avg<V>(InstState *, const InstInfo *, V *, V *, const V *, const V *,      \
                                     double *, const double *, int, hipStream_t);                       \
    template void launch_cast<V>(const double *, V *, int, hipStream_t);                               \
    template void launch_project<V>(V *, const V *, const V *, int, int, V *, const uint8_t *, int, int, \
                                    int, hipStream_t);                                                 \
    template void launch_blend<V>(const double *, const uint8_t *, const uint8_t *, double, double,    \
                                  double *, V *, int, int, hipStream_t);                               \
    template void launch_mip_check<V>(const MatView &, int, int, int, int, const InstInfo *, const V *, \
                                      const double *, const uint8_t *, const double *, const double *, \
                                      const uint8_t *, double, uint8_t *, uint8_t *, uint8_t *, hipStream_t);
SCY_INST(float)
SCY_INST(double)

}  // namespace scy
