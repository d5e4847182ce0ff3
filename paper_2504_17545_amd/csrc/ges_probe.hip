// Device peak probes for the measurement script: a plain copy (HBM
// bandwidth) and global atomic adds spread over a counter array (the rate the
// binning passes' count kernels are bound by).  Declared in
// include/ges_probe.h; nothing on the render path calls them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ges_probe.h"

namespace {

// Four 16-byte loads per thread in flight before the stores; the grid walks
// the buffer in chunks of 4 * 256 vectors per block.
__global__ void __launch_bounds__(256) k_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                int64_t n) {
    const int64_t chunk = 4 * 256;
    for (int64_t c = (int64_t)blockIdx.x * chunk; c < n; c += (int64_t)gridDim.x * chunk) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = c + u * 256 + threadIdx.x;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = c + u * 256 + threadIdx.x;
            if (i < n) dst[i] = v[u];
        }
    }
}

__device__ inline uint32_t mix32(uint32_t x) {  // integer hash (xorshift-multiply)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(256) k_atomics(uint32_t *cnt, int64_t n, uint32_t counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd(cnt + (int64_t)(mix32((uint32_t)i) % counters) * 32, 1u);
}

// Best time of `reps` runs of launch(), each after prep() outside the timed span.
template <class Prep, class Launch>
hipError_t best_ms(int reps, Prep prep, Launch launch, float *best) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    *best = 1e30f;
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = prep();
        if (e == hipSuccess) e = hipEventRecord(a, 0);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, 0);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && ms < *best) *best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

}  // namespace

extern "C" int ges_probe_copy(int device, size_t bytes, int reps, double *out_gbs) {
    if (!out_gbs || reps < 1 || bytes < 16) return (int)hipErrorInvalidValue;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return (int)e;
    const int64_t n = (int64_t)(bytes / 16);
    float4 *src = nullptr, *dst = nullptr;
    if ((e = hipMalloc(&src, n * 16)) != hipSuccess) return (int)e;
    if ((e = hipMalloc(&dst, n * 16)) != hipSuccess) {
        (void)hipFree(src);
        return (int)e;
    }
    e = hipMemset(src, 0, n * 16);
    float ms = 0.f;
    if (e == hipSuccess)
        e = best_ms(reps, [] { return hipSuccess; }, [&] {
            const int64_t blocks = (n + 1023) / 1024;
            hipLaunchKernelGGL(k_copy16, dim3((unsigned)(blocks < 256 * 64 ? blocks : 256 * 64)), dim3(256), 0, 0,
                               src, dst, n);
            return hipGetLastError();
        }, &ms);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (e != hipSuccess) return (int)e;
    *out_gbs = 2.0 * (double)n * 16 / (ms * 1e-3) / 1e9;
    return 0;
}

extern "C" int ges_probe_atomics(int device, int64_t atomics, int32_t counters, int reps, double *out_gops) {
    if (!out_gops || reps < 1 || atomics < 1 || counters < 1) return (int)hipErrorInvalidValue;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return (int)e;
    uint32_t *cnt = nullptr;
    const size_t bytes = (size_t)counters * 32 * sizeof(uint32_t);
    if ((e = hipMalloc(&cnt, bytes)) != hipSuccess) return (int)e;
    float ms = 0.f;
    e = best_ms(reps, [&] { return hipMemsetAsync(cnt, 0, bytes, 0); }, [&] {
        hipLaunchKernelGGL(k_atomics, dim3((unsigned)((atomics + 255) / 256)), dim3(256), 0, 0, cnt, atomics,
                           (uint32_t)counters);
        return hipGetLastError();
    }, &ms);
    (void)hipFree(cnt);
    if (e != hipSuccess) return (int)e;
    *out_gops = (double)atomics / (ms * 1e-3) / 1e9;
    return 0;
}
