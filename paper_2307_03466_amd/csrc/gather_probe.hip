// Random-gather probe (gfx950), built as its own library for the benchmark
// and the profiles; the solver library does not contain it.
//
// Every nonzero of a PDHG pass gathers one 4-byte element of the other
// vector at a data-dependent position, so the device's rate of random
// 4-byte gathers bounds both passes.  gather_probe_ms runs `gathers` such
// gathers at hashed positions of a float vector of `vec_bytes` bytes with
// 8, 16 and 32 gathers per thread and reports the average launch time of
// the fastest of the three, in milliseconds (HIP events, 10 launches after
// a warm-up launch, on a stream of its own).
//
//   int gather_probe_ms(int64_t vec_bytes, int64_t gathers, double *ms);
//   4 <= vec_bytes <= 1 GiB, 1 <= gathers <= 2^31; returns 0, -22 (bad
//   argument) or -5 (a HIP call failed).  Allocates and frees its buffers.
#include <errno.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// Indices are a fixed hash of the position taken modulo the vector length,
// so every gather is in range.
__global__ void k_probe_init(uint32_t *idx, int64_t n, uint32_t len, float *vec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (int64_t)len) vec[i] = (float)(i & 1023) * 0.001f;
    if (i >= n) return;
    uint32_t x = (uint32_t)i * 2654435761u ^ 0x9e3779b9u;
    x ^= x >> 13;
    x *= 0x5bd1e995u;
    x ^= x >> 15;
    x *= 0x27d4eb2du;
    x ^= x >> 16;
    idx[i] = x % len;
}

// K gathers per thread: the index loads stream (non-temporal), then the K
// gathers are in flight together.
template <int K>
__global__ __launch_bounds__(256) void k_probe_gather(const uint32_t *__restrict__ idx,
                                                     const float *__restrict__ vec, float *__restrict__ out,
                                                     int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * 256 * K + threadIdx.x;
    uint32_t w[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t e = base + (int64_t)k * 256;
        w[k] = e < n ? __builtin_nontemporal_load(idx + e) : 0u;
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t e = base + (int64_t)k * 256;
        if (e < n) s += vec[w[k]];
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

void launch_gather(const uint32_t *idx, const float *vec, float *out, int64_t n, int k, hipStream_t s)
{
    const auto grid = [&](int per) { return dim3((unsigned)((n + 256 * per - 1) / (256 * per))); };
    switch (k) {
    case 32: hipLaunchKernelGGL(k_probe_gather<32>, grid(32), dim3(256), 0, s, idx, vec, out, n); break;
    case 16: hipLaunchKernelGGL(k_probe_gather<16>, grid(16), dim3(256), 0, s, idx, vec, out, n); break;
    default: hipLaunchKernelGGL(k_probe_gather<8>, grid(8), dim3(256), 0, s, idx, vec, out, n); break;
    }
}

}  // namespace

extern "C" int gather_probe_ms(int64_t vec_bytes, int64_t gathers, double *ms)
{
    if (!ms || vec_bytes < 4 || vec_bytes > ((int64_t)1 << 30) || gathers < 1 || gathers > ((int64_t)1 << 31))
        return -EINVAL;
    const uint32_t len = (uint32_t)(vec_bytes / 4);
    uint32_t *idx = nullptr;
    float *vec = nullptr, *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -EIO;
    double best = 1e30;
    // out: one float per thread of the 8-per-thread grid, the largest
    const size_t out_elems = (size_t)((gathers + 2047) / 2048) * 256;
    if (hipMalloc((void **)&idx, (size_t)gathers * 4) != hipSuccess) goto done;
    if (hipMalloc((void **)&vec, (size_t)len * 4) != hipSuccess) goto done;
    if (hipMalloc((void **)&out, out_elems * 4) != hipSuccess) goto done;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) goto done;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
    {
        const int64_t m = gathers > (int64_t)len ? gathers : (int64_t)len;
        hipLaunchKernelGGL(k_probe_init, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, idx, gathers, len,
                           vec);
    }
    for (int k : {8, 16, 32}) {
        launch_gather(idx, vec, out, gathers, k, s);
        if (hipEventRecord(e0, s) != hipSuccess) goto done;
        for (int r = 0; r < 10; ++r) launch_gather(idx, vec, out, gathers, k, s);
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
        if (hipGetLastError() != hipSuccess) goto done;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) goto done;
        if ((double)t / 10.0 < best) best = (double)t / 10.0;
    }
    *ms = best;
    rc = 0;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (idx) (void)hipFree(idx);
    if (vec) (void)hipFree(vec);
    if (out) (void)hipFree(out);
    (void)hipGetLastError();
    return rc;
}
