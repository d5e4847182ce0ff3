// Device primitives: fills and an exclusive scan of u32 counts.  A chunk is
// 2048 dense counts (8 per thread) or 256 strided ones (1 per thread: each
// strided count is a cache line of its own, so one per thread spreads the
// line fetches over 8x more blocks).  One chunk: one launch.  More: per-block sums, then a per-block scan
// plus carry where each block adds up the preceding block sums itself (two
// launches); very large counts scan the block sums in one block in between
// (three launches).  No block ever waits on another.  Used to turn per-tile
// and per-primitive counts into list offsets.  The input may be strided (tile
// counters live one per cache line) and the output dense; in place when
// in == out and the stride is 1 (each thread reads its items before writing
// them).
#include "ges_internal.h"

namespace ges {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;  // per thread, dense input
constexpr int64_t kScanSelfCarryBlocks = 2048;  // up to here each apply block sums the block sums itself

// blockIdx.y picks the region
__global__ void k_fill_set(FillSet f) {
    const int r = blockIdx.y;
    uint32_t *p = f.p[r];
    const int64_t count = f.n[r];
    const uint32_t val = f.val[r];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += stride) p[k] = val;
}

// The frame's status as ges_run_status (one thread): the header's counts,
// the spread box-pixel and visible-surfel sums, and the overflow flags a
// count above its capacity implies.
__global__ void k_status(const WsHeader *h, int64_t s_cap, int64_t g_cap, int splatted, ges_run_status *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    ges_run_status r;
    r.flags = h->flags;
    r.reserved = 0;
    r.surfel_pairs = (int64_t)h->s_pairs;
    r.gauss_pairs = (int64_t)h->g_pairs;
    r.surfel_slots = (int64_t)h->s_slots;
    r.gauss_slots = (int64_t)h->g_slots;
    r.surfel_box_pixels = r.gauss_box_pixels = r.visible_surfels = 0;
    for (int k = 0; k < kAreaSlots; ++k) {
        r.surfel_box_pixels += (int64_t)h->s_area[k * 16];
        r.gauss_box_pixels += (int64_t)h->g_area[k * 16];
        r.visible_surfels += (int64_t)h->s_visible[k * 16];
    }
    r.active_gaussians = (int64_t)h->g_active;
    if (r.surfel_pairs > s_cap || r.surfel_slots > s_cap) r.flags |= kFlagSurfelOverflow;
    if (splatted && (r.gauss_pairs > g_cap || r.gauss_slots > g_cap)) r.flags |= kFlagGaussOverflow;
    *out = r;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += stride) p[k] = value;
}

// Fill of mult * (*count) words (at most max), the count read on the device.
__global__ void k_fill_u32_counted(uint32_t *p, uint32_t value, const unsigned long long *count, int64_t mult,
                                   int64_t max) {
    int64_t n = (int64_t)*count * mult;
    if (n > max) n = max;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < n; k += stride) p[k] = value;
}

// Exclusive scan of one value per thread across a 256-thread block; returns
// the block total in *total.
__device__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *total) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = x;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t carry = 0, tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) carry += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return carry + inc - x;
}

// Sum of chunk `blk` of a scan's input into tmp[blk].
template <int IT>
__device__ void scan_reduce_block(const uint32_t *in, int64_t stride, int64_t count, uint32_t *tmp, int64_t blk) {
    const int64_t base = blk * (kScanThreads * IT) + threadIdx.x * IT;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k)
        if (base + k < count) s += in[(base + k) * stride];
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) tmp[blk] = tot;
}

template <int IT>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t *in, int64_t stride, int64_t count,
                                                              uint32_t *tmp) {
    scan_reduce_block<IT>(in, stride, count, tmp, blockIdx.x);
}

// Two scans' reduce phases in one launch: blocks below n0 belong to job 0.
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce2(ScanJob j0, ScanJob j1, int64_t n0) {
    const int64_t b = blockIdx.x;
    if (b < n0) scan_reduce_block<kScanItems>(j0.in, j0.stride, j0.count, j0.tmp, b);
    else scan_reduce_block<kScanItems>(j1.in, j1.stride, j1.count, j1.tmp, b - n0);
}

// One block: exclusive scan of the nb block sums in place; the 64-bit total
// goes to *total64 and to p[count].
__global__ void __launch_bounds__(kScanThreads) k_scan_top(uint32_t *tmp, int64_t nb, uint32_t *p, int64_t count,
                                                           unsigned long long *total64) {
    unsigned long long carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        const uint32_t x = i < nb ? tmp[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(x, &tot);
        if (i < nb) tmp[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) {
        p[count] = (uint32_t)carry;
        if (total64) *total64 = carry;
    }
}

// Sum of x over the block (every thread gets it).
__device__ unsigned long long block_sum_u64(unsigned long long x) {
    __shared__ unsigned long long wsum[kScanThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += wsum[w];
    __syncthreads();
    return t;
}

// Apply pass that finds its own carry: block b adds up the sums of blocks
// 0..b-1 (nb is small, so every block reads them all); the last block also
// writes the total.  Two launches, no block waits on another.
template <int IT>
__device__ void scan_apply_carry_block(const uint32_t *in, int64_t stride, uint32_t *p, int64_t count,
                                       const uint32_t *tmp, int64_t nb, unsigned long long *total64, int64_t b) {
    unsigned long long c = 0;
    for (int64_t i = threadIdx.x; i < b; i += kScanThreads) c += tmp[i];
    const unsigned long long carry = block_sum_u64(c);
    const int64_t base = b * (kScanThreads * IT) + threadIdx.x * IT;
    uint32_t v[IT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        v[k] = base + k < count ? in[(base + k) * stride] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot) + (uint32_t)carry;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (base + k < count) p[base + k] = run;
        run += v[k];
    }
    if (b == nb - 1 && threadIdx.x == 0) {
        p[count] = (uint32_t)(carry + tot);
        if (total64) *total64 = carry + tot;
    }
}

template <int IT>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply_carry(const uint32_t *in, int64_t stride, uint32_t *p,
                                                                   int64_t count, const uint32_t *tmp, int64_t nb,
                                                                   unsigned long long *total64) {
    scan_apply_carry_block<IT>(in, stride, p, count, tmp, nb, total64, blockIdx.x);
}

// Two scans' apply phases in one launch: blocks below nb0 belong to job 0.
__global__ void __launch_bounds__(kScanThreads) k_scan_apply_carry2(ScanJob j0, ScanJob j1, int64_t nb0, int64_t nb1) {
    const int64_t b = blockIdx.x;
    if (b < nb0) scan_apply_carry_block<kScanItems>(j0.in, j0.stride, j0.out, j0.count, j0.tmp, nb0, j0.total64, b);
    else scan_apply_carry_block<kScanItems>(j1.in, j1.stride, j1.out, j1.count, j1.tmp, nb1, j1.total64, b - nb0);
}

template <int IT>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t *in, int64_t stride, uint32_t *p,
                                                             int64_t count, const uint32_t *tmp) {
    const int64_t base = (int64_t)blockIdx.x * (kScanThreads * IT) + threadIdx.x * IT;
    uint32_t v[IT];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        v[k] = base + k < count ? in[(base + k) * stride] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot) + tmp[blockIdx.x];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        if (base + k < count) p[base + k] = run;
        run += v[k];
    }
}

}  // namespace

// block sums a scan of count values may need (the smaller, strided chunk)
int64_t scan_tmp_blocks(int64_t count) { return (count + kScanThreads - 1) / kScanThreads + 1; }

hipError_t launch_status(const WsHeader *h, int64_t s_cap, int64_t g_cap, int splatted, ges_run_status *out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, h, s_cap, g_cap, splatted, out);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_fill_u32_counted(uint32_t *p, uint32_t value, const unsigned long long *count, int64_t mult,
                                   int64_t max, hipStream_t s) {
    if (max <= 0) return hipSuccess;
    int64_t blocks = (max + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_fill_u32_counted, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count, mult, max);
    return hipGetLastError();
}

hipError_t launch_fill_set(const FillSet &f, hipStream_t s) {
    int64_t most = 0;
    for (int r = 0; r < f.count; ++r) most = f.n[r] > most ? f.n[r] : most;
    if (f.count <= 0 || most <= 0) return hipSuccess;
    int64_t blocks = (most + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fill_set, dim3((unsigned)blocks, (unsigned)f.count), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_scan2_u32(const ScanJob &j0, const ScanJob &j1, int64_t tmp_blocks, hipStream_t s) {
    constexpr int64_t C = kScanThreads * kScanItems;
    if (j0.stride != 1 || j1.stride != 1) return hipErrorInvalidValue;  // paired scans are dense
    const int64_t nb0 = (j0.count + C - 1) / C, nb1 = (j1.count + C - 1) / C;
    if (nb0 + 1 > tmp_blocks || nb1 + 1 > tmp_blocks) return hipErrorInvalidValue;
    if (nb0 > kScanSelfCarryBlocks || nb1 > kScanSelfCarryBlocks || nb0 < 1 || nb1 < 1) {
        hipError_t e = launch_scan_u32(j0.in, j0.stride, j0.out, j0.count, j0.tmp, tmp_blocks, j0.total64, s);
        return e == hipSuccess ? launch_scan_u32(j1.in, j1.stride, j1.out, j1.count, j1.tmp, tmp_blocks, j1.total64, s)
                               : e;
    }
    // a job of one chunk needs no reduce block (its carry is zero)
    const int64_t r0 = nb0 > 1 ? nb0 : 0, r1 = nb1 > 1 ? nb1 : 0;
    if (r0 + r1 > 0) {
        if (r0 > 0) hipLaunchKernelGGL(k_scan_reduce2, dim3((unsigned)(r0 + r1)), dim3(kScanThreads), 0, s, j0, j1, r0);
        else hipLaunchKernelGGL(k_scan_reduce2, dim3((unsigned)r1), dim3(kScanThreads), 0, s, j1, j1, (int64_t)0);
    }
    hipLaunchKernelGGL(k_scan_apply_carry2, dim3((unsigned)(nb0 + nb1)), dim3(kScanThreads), 0, s, j0, j1, nb0, nb1);
    return hipGetLastError();
}

namespace {

template <int IT>
hipError_t scan_u32(const uint32_t *in, int64_t in_stride, uint32_t *out, int64_t count, uint32_t *tmp,
                    int64_t tmp_blocks, unsigned long long *total64, hipStream_t s) {
    constexpr int64_t C = kScanThreads * IT;
    const int64_t nb = (count + C - 1) / C;
    if (nb + 1 > tmp_blocks) return hipErrorInvalidValue;
    if (nb <= 1) {  // one chunk: no carry to find
        hipLaunchKernelGGL(k_scan_apply_carry<IT>, dim3(1), dim3(kScanThreads), 0, s, in, in_stride, out, count, tmp,
                           (int64_t)1, total64);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce<IT>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, in_stride, count, tmp);
    if (nb <= kScanSelfCarryBlocks) {
        hipLaunchKernelGGL(k_scan_apply_carry<IT>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, in_stride, out,
                           count, tmp, nb, total64);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, tmp, nb, out, count, total64);
    hipLaunchKernelGGL(k_scan_apply<IT>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, in_stride, out, count, tmp);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_u32(const uint32_t *in, int64_t in_stride, uint32_t *out, int64_t count, uint32_t *tmp,
                           int64_t tmp_blocks, unsigned long long *total64, hipStream_t s) {
    return in_stride == 1 ? scan_u32<kScanItems>(in, in_stride, out, count, tmp, tmp_blocks, total64, s)
                          : scan_u32<1>(in, in_stride, out, count, tmp, tmp_blocks, total64, s);
}

}  // namespace ges
