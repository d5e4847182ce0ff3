// Pruning scores of a rendered frame (Sec. 4.1, surfel pruning; Sec. 4.2,
// Eq. 9, Gaussian pruning).
//
//   covering score  n_{i,j}: the number of pixels of view j whose frontmost
//                   surfel is i (the pixels of the id map equal to i); the
//                   score is n_i = max over views.  Per view: each raster
//                   tile groups its pixels by surfel id in an LDS hash table
//                   and counts them (LDS integer atomics), then adds one
//                   count per (tile, surfel it shows) into a per-surfel
//                   counter; a per-surfel pass folds the view's counts into
//                   the running maximum and clears the counters for the next
//                   view.  Integer sums and maxima: exact.
//   contribution    s_{i,j} = max over the pixels where Gaussian i counts
//   score           (alpha >= alpha_min and the depth test passes, the same
//                   decisions as pass 2) of c_{i,j} alpha / (W_s + W_G),
//                   c_{i,j} its largest colour channel in view j.  Per splat
//                   tile, 8 lanes take one list entry and walk its pixels in
//                   the tile; the largest value per entry is folded into the
//                   Gaussian's score with an integer atomic maximum of the
//                   non-negative float's bits (order-free, exact).
#include "ges_internal.h"

namespace ges {

namespace {

// Per raster tile of one view: pixels grouped by their surfel (open
// addressing over twice as many slots as pixels, so an insert always finds
// a free slot), then one global add per (tile, surfel) into cnt[id].
template <int T>
__global__ void __launch_bounds__(T * T) k_score_surfel_tiles(FrameArgs a, int v, int ntiles, const int32_t *sid,
                                                              uint32_t *cnt) {
    constexpr int NT = T * T;
    constexpr int HS = 2 * NT;
    __shared__ uint32_t h_id[HS];
    __shared__ uint32_t h_cnt[HS];
    const int tid = (int)threadIdx.x;
    const ViewDev &V = a.views[v];
    const int lt = xcd_tile((int)blockIdx.x, ntiles);
    const int tx = lt % V.rtx, ty = lt / V.rtx;
    const int px = tx * T + tid % T, py = ty * T + tid / T;
    for (int i = tid; i < HS; i += NT) {
        h_id[i] = 0xFFFFFFFFu;
        h_cnt[i] = 0u;
    }
    __syncthreads();
    int id = -1;
    if (px < V.W && py < V.H) id = sid[V.pix_off + (int64_t)py * V.W + px];
    if (id >= 0 && (int64_t)id < a.n) {
        uint32_t h = ((uint32_t)id * 2654435761u) & (HS - 1);
        for (;;) {  // ends: at most NT distinct ids in HS = 2 NT slots
            const uint32_t prev = atomicCAS(&h_id[h], 0xFFFFFFFFu, (uint32_t)id);
            if (prev == 0xFFFFFFFFu || prev == (uint32_t)id) break;
            h = (h + 1) & (HS - 1);
        }
        atomicAdd(&h_cnt[h], 1u);
    }
    __syncthreads();
    for (int i = tid; i < HS; i += NT) {
        const uint32_t s = h_id[i];
        if (s != 0xFFFFFFFFu) atomicAdd(&cnt[s], h_cnt[i]);
    }
}

// cover[i] <- max(cover[i], cnt[i]) (or cnt[i] for the first view of a
// call that does not accumulate); cnt[i] <- 0 for the next view.
__global__ void __launch_bounds__(256) k_score_fold(int64_t n, uint32_t *cnt, int32_t *cover, int first_overwrite) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cnt[i];
    cnt[i] = 0u;
    const int32_t cur = first_overwrite ? 0 : cover[i];
    cover[i] = (int32_t)c > cur ? (int32_t)c : cur;
}

// Per splat tile (all views in one launch): the largest c alpha / (W_s + W_G)
// of every list entry over its pixels in the tile, folded into best[gauss].
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_score_gauss_tiles(FrameArgs a, const float *depth, const float *accum,
                                                               uint32_t *best) {
    constexpr int NT = TW * TH;
    __shared__ float s_inv[NT];
    __shared__ float s_ds[NT];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_toff);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)toff[t], cap), b1 = umin64((uint64_t)toff[t + 1], cap);
    if (b0 >= b1) return;  // no Gaussian reaches this tile
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int tx0 = (lt % V.stx) * TW, ty0 = (lt / V.stx) * TH;
    {
        const int px = tx0 + (int)(threadIdx.x % TW), py = ty0 + (int)(threadIdx.x / TW);
        float inv = 0.f, ds = -__int_as_float(0x7f800000);  // outside the image: nothing passes
        if (px < V.W && py < V.H) {
            const int64_t lp = (int64_t)py * V.W + px;
            const int64_t P = (int64_t)V.W * V.H;
            inv = 1.f / (a.opt.w_s + accum[4 * V.pix_off + 3 * P + lp]);
            ds = depth[V.pix_off + lp];
        }
        s_inv[threadIdx.x] = inv;
        s_ds[threadIdx.x] = ds;
    }
    __syncthreads();
    const GEnt *ents = reinterpret_cast<const GEnt *>(a.ws + a.L.g_ents);
    const float amin = a.opt.alpha_min;
    constexpr int kSplit = 8;  // lanes per entry; lane `sub` walks rows y0 + sub, y0 + sub + 8, ...
    const int sub = (int)threadIdx.x % kSplit;
    for (uint64_t base = b0; base < b1; base += NT / kSplit) {
        const uint64_t pos = base + threadIdx.x / kSplit;
        const bool have = pos < b1;
        float mx = 0.f;
        uint32_t gi = 0;
        float cmax = 0.f;
        if (have) {
            const GEnt &e = ents[pos];
            const GRec g = e.g;
            gi = e.gauss;
            cmax = fmaxf(g.r, fmaxf(g.g, g.b)) * (float)kFixInv;
            const uint32_t lb = e.lbox;
            const int x0 = tx0 + (int)(lb & 15), x1 = tx0 + (int)((lb >> 4) & 15);
            const int y0 = ty0 + (int)((lb >> 8) & 15), y1 = ty0 + (int)((lb >> 12) & 15);
            for (int yy = y0 + sub; yy <= y1; yy += kSplit)
                for (int xx = x0; xx <= x1; ++xx) {
                    const int lp = (yy - ty0) * TW + (xx - tx0);
                    float dx, dy, q;
                    const float al = gauss_alpha(g, (float)xx + 0.5f, (float)yy + 0.5f, dx, dy, q);
                    if ((al >= amin) & (g.dme < s_ds[lp])) mx = fmaxf(mx, al * s_inv[lp]);
                }
        }
#pragma unroll
        for (int off = kSplit / 2; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if (have && sub == 0) {
            const float s = cmax * mx;
            if (s > 0.f && (int64_t)gi < a.m) atomicMax(&best[gi], __float_as_uint(s));
        }
    }
}

// keep flags from the final scores; either array may be absent.
__global__ void __launch_bounds__(256) k_score_masks(int64_t n, int64_t m, const int32_t *cover, const float *contrib,
                                                    int32_t cover_min, float contrib_min, uint8_t *keep_s,
                                                    uint8_t *keep_g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (keep_s && i < n) keep_s[i] = cover[i] >= cover_min ? 1 : 0;
    if (keep_g && i < m) keep_g[i] = contrib[i] >= contrib_min ? 1 : 0;
}

inline unsigned blocks_of(int64_t count) { return (unsigned)((count + 255) / 256); }

}  // namespace

hipError_t launch_score_surfel_view(const FrameArgs &a, int v, int ntiles, const int32_t *sid, uint32_t *cnt,
                                    int32_t *cover, int first_overwrite, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (ntiles > 0) {
        if (a.opt.raster_tile == 8)
            hipLaunchKernelGGL(k_score_surfel_tiles<8>, dim3((unsigned)ntiles), dim3(64), 0, s, a, v, ntiles, sid, cnt);
        else
            hipLaunchKernelGGL(k_score_surfel_tiles<16>, dim3((unsigned)ntiles), dim3(256), 0, s, a, v, ntiles, sid,
                               cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_score_fold, dim3(blocks_of(a.n)), dim3(256), 0, s, a.n, cnt, cover, first_overwrite);
    return hipGetLastError();
}

hipError_t launch_score_gauss(const FrameArgs &a, const float *depth, const float *accum, float *contrib,
                              hipStream_t s) {
    if (a.m <= 0 || a.L.stiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.L.stiles);
    uint32_t *best = reinterpret_cast<uint32_t *>(contrib);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_score_gauss_tiles<8, 8>), grid, dim3(64), 0, s, a, depth, accum, best);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_score_gauss_tiles<16, 8>), grid, dim3(128), 0, s, a, depth, accum, best);
    else
        hipLaunchKernelGGL((k_score_gauss_tiles<16, 16>), grid, dim3(256), 0, s, a, depth, accum, best);
    return hipGetLastError();
}

hipError_t launch_score_masks(int64_t n, int64_t m, const int32_t *cover, const float *contrib, int32_t cover_min,
                              float contrib_min, uint8_t *keep_s, uint8_t *keep_g, hipStream_t s) {
    const int64_t k = n > m ? n : m;
    if (k <= 0 || (!keep_s && !keep_g)) return hipSuccess;
    hipLaunchKernelGGL(k_score_masks, dim3(blocks_of(k)), dim3(256), 0, s, n, m, cover, contrib, cover_min,
                       contrib_min, keep_s, keep_g);
    return hipGetLastError();
}

}  // namespace ges
