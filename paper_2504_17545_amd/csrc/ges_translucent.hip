// Translucent surfels of the surfel optimisation stage (Sec. 4.1, Eq. 6-7):
// a surfel's opacity at the point (x, y) of its local plane is
// alpha = min(1, w G(x, y)), G = exp(-(x^2 + y^2) / 2), zero where
// min(alpha, G) < 1/255, and the surfels are alpha-blended front to back in
// the order of their centre depth, optionally with the pixel's nearest
// surfel first.  The lists are the surfel binning's (ges_project and the
// surfel fill, run in translucent mode: no occluders; each entry carries the
// centre depth, w and its slot index).
//
//   tblend      per raster tile: the tile's entries sorted by (centre depth,
//               surfel index) in LDS (a bitonic sort of 64-bit keys, at most
//               kSortCap entries per tile, else the frame is flagged), the
//               sorted order kept for the backward; with the order
//               adjustment, a first pass finds each pixel's nearest surfel
//               with alpha > 0; then the blend, one thread per pixel, in
//               batches of records staged in LDS, stopping once every pixel
//               of the tile is opaque (T = 0).  Per pixel it keeps, for the
//               backward, T before the last blended entry, that entry's
//               place in the sorted order and the front entry's place.
//   tblend_bwd  per raster tile, the blend in reverse: from the last blended
//               entry back, T before each entry is recovered by dividing by
//               (1 - alpha) (below the last entry every alpha is < 1, else
//               the blend would have stopped there) and the colour behind it
//               is carried along; each pixel's terms for the entry are
//               summed over the wave (a fixed reduction tree) and the waves'
//               sums in wave order: one partial per entry, 13 floats (dL/dU,
//               dL/dV, dL/dn of the record, dL/dw, dL/dc), stored at its slot.
//               The front entries' terms are added in a second pass.
//   tsurfels    per surfel: the partials of its slot run (views in order,
//               box tiles in row order), then the chain rule in FP64 to the
//               centre, rotation, scales, w and SH (colour and its view
//               direction).
#include "ges_internal.h"

namespace ges {

namespace {

constexpr int kSortCap = 2048;                // entries a tile's sort holds
constexpr float kLog2_255 = 7.99435343685885793f;
constexpr double kLn255 = 5.5412635451584258;
constexpr int kBwdBatch = 64;                 // entries per backward batch
constexpr int kTsBlock = 128;                 // surfels per chain-rule block

__device__ __forceinline__ void put_nt(float *p, float v) { __builtin_nontemporal_store(v, p); }

// Order-preserving unsigned key of a float (any sign).
__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// One list entry (SEnt): r0 = (Ux, Uy, Uz, Vx), r1 = (Vy, Vz, nx, ny),
// r2 = (nz, w, zmin, surfel index), r3 = (lbox, centre depth, w_mod, slot).
// Staged in LDS as 64 bytes: zmin (not needed here) gives way to w_mod, and
// the surfel's colour in this view fills the last word but one.
struct TRec {
    float4 r0, r1, r2;  // r2.z = w_mod
    float c0, c1, c2;   // colour in the blend passes; c0 = zmin in the front pass
    uint32_t lb;        // the disc's screen box inside the tile (pack_lbox)
};
static_assert(sizeof(TRec) == 64, "TRec is one 64-byte LDS record");

// Whether tile-local pixel (lx, ly) lies in an entry's box.  The box bounds
// every pixel whose ray passes the FP32 disc test (the opaque raster
// evaluates only these pixels too), so outside it alpha is 0.
__device__ __forceinline__ bool in_lbox(uint32_t lb, int lx, int ly) {
    return (lx >= (int)(lb & 15u)) & (lx <= (int)((lb >> 4) & 15u)) & (ly >= (int)((lb >> 8) & 15u)) &
           (ly <= (int)((lb >> 12) & 15u));
}

// A wave-list word: the entry's place in the staged batch | its box << 16.
// kMissWord pads a list to a multiple of 4: place 0 with an empty box.
constexpr uint32_t kMissWord = 15u << 16;

// LDS writes of the wave's lanes visible to its later reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The wave's own list of a staged batch: the places kk < nb, in order,
// whose box meets tile rows [r0, r1] (the wave's pixels), as list words,
// then four kMissWord (the list holds nb + 4 words, 16-byte aligned);
// returns their number.  The pixel loops then run over entries that can
// touch the wave, four words at a time, instead of testing every entry of
// the batch in every wave.
__device__ __forceinline__ int wave_compact(const uint32_t *lbs, int nb, int r0, int r1, uint32_t *list, int lane) {
    int cnt = 0;
    for (int i0 = 0; i0 < nb; i0 += 64) {
        const int e = i0 + lane;
        bool hit = false;
        uint32_t lb = 0;
        if (e < nb) {
            lb = lbs[e] & 0xffffu;
            hit = ((int)((lb >> 8) & 15u) <= r1) & ((int)((lb >> 12) & 15u) >= r0);
        }
        const unsigned long long m = __ballot((int)hit);
        if (hit) {
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            list[cnt + r] = (uint32_t)e | (lb << 16);
        }
        cnt += __popcll(m);
    }
    if (lane < 4) list[cnt + lane] = kMissWord;
    wave_lds_sync();
    return cnt;
}

// Four list words and their staged records (the LDS reads issued together).
__device__ __forceinline__ void read4(const uint32_t *list, int q, const TRec *recs, uint32_t (&le)[4], TRec (&e4)[4]) {
    const uint4 l4 = *reinterpret_cast<const uint4 *>(list + q);
    le[0] = l4.x;
    le[1] = l4.y;
    le[2] = l4.z;
    le[3] = l4.w;
#pragma unroll
    for (int u = 0; u < 4; ++u) e4[u] = recs[le[u] & 0xffffu];
}

// The ray (xr, yr, 1) against one record: its opacity (Eq. 6-7), with the
// disc test of the opaque raster for the G >= 1/255 half of the rule (the
// same FP32 decision), the hit depth and the quantities the backward needs.
struct THit {
    float alpha, z, G, au, bv, c;
    bool clamp;  // w G >= 1: alpha = 1, no gradient through it
};

__device__ __forceinline__ THit thit(const TRec &e, float xr, float yr, float zn) {
    THit h;
    h.c = fmaf(e.r1.z, xr, fmaf(e.r1.w, yr, e.r2.x));
    h.au = fmaf(e.r0.x, xr, fmaf(e.r0.y, yr, e.r0.z));
    h.bv = fmaf(e.r0.w, xr, fmaf(e.r1.x, yr, e.r1.y));
    const bool in = (h.c > 0.f) & (fmaf(h.au, h.au, h.bv * h.bv) <= h.c * h.c) & (e.r2.y >= zn * h.c);
    const float ic = __builtin_amdgcn_rcpf(h.c);  // the opaque raster's reciprocal (hit depth w / c alike)
    const float ua = h.au * ic, vb = h.bv * ic;
    const float rho2 = fmaf(ua, ua, vb * vb);           // (x^2 + y^2) / R^2, R^2 = 2 ln 255
    h.G = __builtin_amdgcn_exp2f(-kLog2_255 * rho2);    // exp(-(x^2 + y^2) / 2)
    const float wg = e.r2.z * h.G;
    h.clamp = wg >= 1.f;
    const float a = fminf(wg, 1.f);
    h.alpha = (in && a >= 1.f / 255.f) ? a : 0.f;
    h.z = e.r2.y * ic;
    return h;
}

__device__ __forceinline__ TRec load_trec(const float4 *ents, uint64_t pos) {
    TRec e;
    const float4 *p = ents + pos * 4;
    e.r0 = p[0];
    e.r1 = p[1];
    e.r2 = p[2];
    const float4 r3 = p[3];
    e.r2.z = r3.z;
    e.lb = __float_as_uint(r3.x);
    e.c0 = e.c1 = e.c2 = 0.f;
    return e;
}

template <int T>
__global__ void __launch_bounds__(T * T) k_tblend(FrameArgs a, float *color, float *alpha_out, float *depth_out,
                                                  int32_t *front_out) {
    constexpr int NT = T * T, NW = NT / 64, RW = 64 / T;  // RW: tile rows per wave
    // the sort's keys; once sorted, the same LDS holds the wave lists and boxes
    __shared__ __align__(16) unsigned long long keys[kSortCap];
    __shared__ uint16_t kpos[kSortCap];
    __shared__ TRec recs[NT];
    __shared__ int s_any;
    static_assert((NW * (NT + 4) + NT) * 4 <= kSortCap * 8, "wave lists fit in the key array");
    uint32_t *const lbs = reinterpret_cast<uint32_t *>(keys) + NW * (NT + 4);
    const TileOrd o = reinterpret_cast<const TileOrd *>(a.ws + a.L.s_ord)[blockIdx.x];
    const int t = (int)o.tile;
    const int v = view_of_rtile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.rt_off;
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lx = tid % T, ly = tid / T;
    const int px = (lt % V.rtx) * T + lx, py = (lt / V.rtx) * T + ly;
    const bool inside = px < V.W && py < V.H;
    const float xr = ((float)px + 0.5f - V.cx) / V.fx, yr = ((float)py + 0.5f - V.cy) / V.fy;
    const float zn = V.znear;
    uint32_t *const mylist = reinterpret_cast<uint32_t *>(keys) + wv * (NT + 4);
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);
    const int count = (int)(b1 - b0);
    const int ns = count < kSortCap ? count : kSortCap;
    if (count > kSortCap && tid == 0) atomicOr(&reinterpret_cast<WsHeader *>(a.ws + a.L.header)->flags, kFlagSortOverflow);
    const float4 *ents = reinterpret_cast<const float4 *>(a.ws + a.L.s_ents);
    const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol) + (int64_t)v * 3 * a.n;
    uint32_t *sorted = reinterpret_cast<uint32_t *>(a.ws + a.L.t_sorted);

    // sort keys (centre depth, surfel index) with the entry's place in the
    // list; the entries' box areas are summed for the frame status
    int np = 1;
    while (np < ns) np <<= 1;
    unsigned long long area = 0;
    for (int i = tid; i < np; i += NT) {
        if (i < ns) {
            const float4 *p = ents + (b0 + (uint64_t)i) * 4;
            const float4 r3 = p[3];
            const uint32_t lb = __float_as_uint(r3.x);
            area += (unsigned long long)(((lb >> 4) & 15u) - (lb & 15u) + 1u) * (((lb >> 12) & 15u) - ((lb >> 8) & 15u) + 1u);
            keys[i] = ((unsigned long long)fkey(r3.y) << 32) | __float_as_uint(p[2].w);
            kpos[i] = (uint16_t)i;
        } else {
            keys[i] = ~0ull;
            kpos[i] = 0xffff;
        }
    }
    block_add_area<NT>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->s_area, area);  // (synchronises)
    for (int k = 2; k <= np; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < np; i += NT) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long ki = keys[i], kl = keys[l];
                    const bool up = (i & k) == 0;
                    if ((ki > kl) == up) {
                        keys[i] = kl;
                        keys[l] = ki;
                        const uint16_t pi = kpos[i];
                        kpos[i] = kpos[l];
                        kpos[l] = pi;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = tid; i < ns; i += NT) sorted[b0 + i] = (uint32_t)(b0 + kpos[i]);

    // the pixel's nearest surfel with alpha > 0 (smaller index on a tie)
    int front_k = -1;
    if (a.front_first) {
        unsigned long long best = ~0ull;
        float bestz = __int_as_float(0x7f800000);
        for (int k0 = 0; k0 < ns; k0 += NT) {
            __syncthreads();
            if (k0 + tid < ns) {
                const uint64_t pos = b0 + kpos[k0 + tid];
                TRec e = load_trec(ents, pos);
                e.c0 = ents[pos * 4 + 2].z;  // zmin: no FP32 hit of the disc is nearer
                recs[tid] = e;
                lbs[tid] = e.lb;
            }
            __syncthreads();
            const int nb = min(NT, ns - k0);
            const int cnt = wave_compact(lbs, nb, wv * RW, wv * RW + RW - 1, mylist, lane);
            for (int q = 0; q < cnt; q += 4) {
                uint32_t le[4];
                TRec e4[4];
                read4(mylist, q, recs, le, e4);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    // an entry whose nearest point is beyond the pixel's current
                    // nearest hit cannot replace it (strictly: no tie to break)
                    if (inside & in_lbox(le[u] >> 16, lx, ly) & !(e4[u].c0 > bestz)) {
                        const THit h = thit(e4[u], xr, yr, zn);
                        if (h.alpha > 0.f) {
                            const unsigned long long key =
                                ((unsigned long long)__float_as_uint(h.z) << 32) | __float_as_uint(e4[u].r2.w);
                            if (key < best) {
                                best = key;
                                bestz = h.z;
                                front_k = k0 + (int)(le[u] & 0xffffu);
                            }
                        }
                    }
                }
            }
        }
    }

    // the blend
    float Tr = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, Tb = 1.f;
    int last_k = -1;
    if (front_k >= 0) {
        const TRec e = load_trec(ents, b0 + kpos[front_k]);
        const THit h = thit(e, xr, yr, zn);
        const int id = (int)__float_as_uint(e.r2.w);
        const float w = h.alpha;  // > 0
        C0 += w * scol[id];
        C1 += w * scol[a.n + id];
        C2 += w * scol[2 * a.n + id];
        D += w * h.z;
        Tr = 1.f - h.alpha;
    }
    bool done = !inside || Tr == 0.f;
    for (int k0 = 0; k0 < ns; k0 += NT) {
        __syncthreads();
        if (tid == 0) s_any = 0;
        if (k0 + tid < ns) {
            TRec e = load_trec(ents, b0 + kpos[k0 + tid]);
            const int id = (int)__float_as_uint(e.r2.w);
            e.c0 = scol[id];
            e.c1 = scol[a.n + id];
            e.c2 = scol[2 * a.n + id];
            recs[tid] = e;
            lbs[tid] = e.lb;
        }
        __syncthreads();
        if (!done) atomicOr(&s_any, 1);
        __syncthreads();
        if (s_any == 0) break;  // block-uniform: every pixel of the tile is opaque
        const int nb = min(NT, ns - k0);
        const int cnt = wave_compact(lbs, nb, wv * RW, wv * RW + RW - 1, mylist, lane);
        for (int q = 0; q < cnt; q += 4) {
            if (__ballot((int)!done) == 0ull) break;  // wave-uniform: the wave's pixels are opaque
            uint32_t le[4];
            TRec e4[4];
            read4(mylist, q, recs, le, e4);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + (int)(le[u] & 0xffffu);
                if (!done & (k != front_k) & in_lbox(le[u] >> 16, lx, ly)) {
                    const THit h = thit(e4[u], xr, yr, zn);
                    if (h.alpha > 0.f) {
                        const float w = Tr * h.alpha;
                        C0 += w * e4[u].c0;
                        C1 += w * e4[u].c1;
                        C2 += w * e4[u].c2;
                        D += w * h.z;
                        Tb = Tr;
                        Tr = Tr * (1.f - h.alpha);
                        last_k = k;
                        done = Tr == 0.f;
                    }
                }
            }
        }
    }
    if (inside) {
        const int64_t lp = (int64_t)py * V.W + px;
        const int64_t P = (int64_t)V.W * V.H;
        float *cp = color + 3 * V.pix_off + lp;
        cp[0] = C0 + Tr * V.bg[0];
        cp[P] = C1 + Tr * V.bg[1];
        cp[2 * P] = C2 + Tr * V.bg[2];
        alpha_out[V.pix_off + lp] = 1.f - Tr;
        depth_out[V.pix_off + lp] = D;
        front_out[V.pix_off + lp] = front_k >= 0 ? (int32_t)__float_as_uint(ents[(b0 + kpos[front_k]) * 4 + 2].w) : -1;
        float *st = reinterpret_cast<float *>(a.ws + a.L.t_state);
        const int64_t tp = (int64_t)a.L.pixels;
        st[V.pix_off + lp] = last_k >= 0 ? Tb : 1.f;
        reinterpret_cast<int32_t *>(st + tp)[V.pix_off + lp] = last_k;
        reinterpret_cast<int32_t *>(st + 2 * tp)[V.pix_off + lp] = front_k;
    }
}

// x of another lane by a DPP move; lanes the move does not write get 0.
template <int Ctrl, int RowMask>
__device__ __forceinline__ float dpp_or_zero(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), Ctrl, RowMask, 0xf, false));
}

// Sum over the wave's 64 lanes, by DPP row shifts (each row of 16 lanes
// into its lane 15) and then row broadcasts (rows 0+1 into lane 31, 2+3
// into lane 63, then both): the same fixed tree in every call, no LDS
// traffic.  The total is valid in lane 63 only.  Every lane must be active.
__device__ __forceinline__ float wave_sum63(float x) {
    x += dpp_or_zero<0x111, 0xf>(x);  // row_shr:1
    x += dpp_or_zero<0x112, 0xf>(x);  // row_shr:2
    x += dpp_or_zero<0x114, 0xf>(x);  // row_shr:4
    x += dpp_or_zero<0x118, 0xf>(x);  // row_shr:8
    x += dpp_or_zero<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_or_zero<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return x;
}

// The 13 terms of one (pixel, entry): dL/dU, dL/dV, dL/dn (3 each: the
// record's vectors against the ray r = (xr, yr, 1)), dL/dw_mod, dL/dc (3).
struct TTerms {
    float v[kTPartials];
};

__device__ __forceinline__ void hit_terms(const TRec &e, const THit &h, float dLda, const float dc[3], float xr,
                                          float yr, TTerms &o) {
    // alpha = w G, G = 255^-(rho2), rho2 = (au^2 + bv^2) / c^2 (unclamped)
    float gU = 0.f, gV = 0.f, gN = 0.f, gw = 0.f;
    if (!h.clamp) {
        gw = dLda * h.G;
        const float g = dLda * e.r2.z * h.G * (-(float)kLn255);  // dL/d(rho2)
        const float ic = __builtin_amdgcn_rcpf(h.c), ic2 = ic * ic;
        const float rho2 = (h.au * h.au + h.bv * h.bv) * ic2;
        gU = g * 2.f * h.au * ic2;
        gV = g * 2.f * h.bv * ic2;
        gN = g * -2.f * rho2 * ic;
    }
    o.v[0] = gU * xr; o.v[1] = gU * yr; o.v[2] = gU;
    o.v[3] = gV * xr; o.v[4] = gV * yr; o.v[5] = gV;
    o.v[6] = gN * xr; o.v[7] = gN * yr; o.v[8] = gN;
    o.v[9] = gw;
    o.v[10] = dc[0]; o.v[11] = dc[1]; o.v[12] = dc[2];
}

template <int T>
__global__ void __launch_bounds__(T * T) k_tblend_bwd(FrameArgs a, const float *d_color) {
    constexpr int NT = T * T, NW = NT / 64, RW = 64 / T;  // RW: tile rows per wave
    __shared__ TRec recs[kBwdBatch];
    __shared__ uint32_t lbs[kBwdBatch];
    __shared__ __align__(16) uint32_t wlist[NW][kBwdBatch + 4];
    __shared__ uint32_t slots[kBwdBatch];
    __shared__ float wpart[NW][kBwdBatch][kTPartials];
    __shared__ int s_max;
    const TileOrd o = reinterpret_cast<const TileOrd *>(a.ws + a.L.s_ord)[blockIdx.x];
    const int t = (int)o.tile;
    const int v = view_of_rtile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.rt_off;
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lx = tid % T, ly = tid / T;
    const int px = (lt % V.rtx) * T + lx, py = (lt / V.rtx) * T + ly;
    const bool inside = px < V.W && py < V.H;
    const float xr = ((float)px + 0.5f - V.cx) / V.fx, yr = ((float)py + 0.5f - V.cy) / V.fy;
    const float zn = V.znear;
    uint32_t *const mylist = wlist[wv];
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);
    const int count = (int)(b1 - b0);
    const int ns = count < kSortCap ? count : kSortCap;
    const float4 *ents = reinterpret_cast<const float4 *>(a.ws + a.L.s_ents);
    const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol) + (int64_t)v * 3 * a.n;
    const uint32_t *sorted = reinterpret_cast<const uint32_t *>(a.ws + a.L.t_sorted);
    float *part = reinterpret_cast<float *>(a.ws + a.L.t_part);

    // entries past the sort's capacity took no part: their partials are zero
    for (int i = ns + tid; i < count; i += NT) {
        const uint32_t sl = __float_as_uint(ents[(b0 + (uint64_t)i) * 4 + 3].w);
        for (int c = 0; c < kTPartials; ++c) part[(uint64_t)sl * kTPartials + c] = 0.f;
    }
    float dC[3] = {0.f, 0.f, 0.f};
    float Tb_last = 1.f;
    int last_k = -1, front_k = -1;
    const int64_t lp = (int64_t)py * V.W + px;
    if (inside) {
        const int64_t P = (int64_t)V.W * V.H;
        const float *dg = d_color + 3 * V.pix_off + lp;
        dC[0] = dg[0];
        dC[1] = dg[P];
        dC[2] = dg[2 * P];
        const float *st = reinterpret_cast<const float *>(a.ws + a.L.t_state);
        const int64_t tp = (int64_t)a.L.pixels;
        Tb_last = st[V.pix_off + lp];
        last_k = reinterpret_cast<const int32_t *>(st + tp)[V.pix_off + lp];
        front_k = reinterpret_cast<const int32_t *>(st + 2 * tp)[V.pix_off + lp];
    }
    // colour behind the entry being processed, and T before the entry after it
    float S0 = V.bg[0], S1 = V.bg[1], S2 = V.bg[2];
    float Tn = Tb_last;
    bool first = true;  // the next blended entry met is the last one
    // the tile's last blended place: entries past it get zero partials
    // without being staged
    if (tid == 0) s_max = -1;
    __syncthreads();
    if (last_k >= 0) atomicMax(&s_max, last_k);
    __syncthreads();
    const int klast = s_max;
    for (int i = klast + 1 + tid; i < ns; i += NT) {
        const uint32_t sl = __float_as_uint(ents[(uint64_t)sorted[b0 + i] * 4 + 3].w);
        for (int c = 0; c < kTPartials; ++c) part[(uint64_t)sl * kTPartials + c] = 0.f;
    }
    // descending batches over places [0, klast]
    for (int k1 = klast + 1; k1 > 0; k1 -= kBwdBatch) {
        const int kb0 = k1 - kBwdBatch > 0 ? k1 - kBwdBatch : 0, nb = k1 - kb0;
        __syncthreads();
        if (tid < nb) {
            const uint32_t pos = sorted[b0 + kb0 + tid];
            TRec e = load_trec(ents, pos);
            slots[tid] = __float_as_uint(ents[(uint64_t)pos * 4 + 3].w);
            const int id = (int)__float_as_uint(e.r2.w);
            e.c0 = scol[id];
            e.c1 = scol[a.n + id];
            e.c2 = scol[2 * a.n + id];
            recs[tid] = e;
            lbs[tid] = e.lb;
        }
        // the wave's sums start at zero: entries off its rows keep them
        for (int i = lane; i < nb * kTPartials; i += 64) (&wpart[wv][0][0])[i] = 0.f;
        __syncthreads();
        const int cnt = wave_compact(lbs, nb, wv * RW, wv * RW + RW - 1, mylist, lane);
        for (int q = cnt - 1; q >= 0; --q) {
            {
                const uint32_t wd = mylist[q];
                const int kk = (int)(wd & 0xffffu);
                const int k = kb0 + kk;
                TTerms tm;
#pragma unroll
                for (int c = 0; c < kTPartials; ++c) tm.v[c] = 0.f;
                bool have = false, geo = false;
                if (inside & (k <= last_k) & (k != front_k) & in_lbox(wd >> 16, lx, ly)) {
                    const TRec &e = recs[kk];
                    const THit h = thit(e, xr, yr, zn);
                    if (h.alpha > 0.f) {
                        const float Tk = first ? Tb_last : Tn / (1.f - h.alpha);
                        first = false;
                        const float3 ck = make_float3(e.c0, e.c1, e.c2);
                        const float dLda = Tk * (dC[0] * (ck.x - S0) + dC[1] * (ck.y - S1) + dC[2] * (ck.z - S2));
                        const float wa = h.alpha * Tk;
                        const float dc[3] = {dC[0] * wa, dC[1] * wa, dC[2] * wa};
                        hit_terms(e, h, dLda, dc, xr, yr, tm);
                        S0 = h.alpha * ck.x + (1.f - h.alpha) * S0;
                        S1 = h.alpha * ck.y + (1.f - h.alpha) * S1;
                        S2 = h.alpha * ck.z + (1.f - h.alpha) * S2;
                        Tn = Tk;
                        have = true;
                        geo = !h.clamp;
                    }
                }
                if (__ballot((int)have) != 0ull) {  // wave-uniform
                    // where alpha is clamped at 1 only the colour terms are nonzero
                    // (the clamped inner disc of a surfel with w > 1)
                    if (__ballot((int)geo) != 0ull) {
#pragma unroll
                        for (int c = 0; c < 10; ++c) {
                            const float sum = wave_sum63(tm.v[c]);
                            if (lane == 63) wpart[wv][kk][c] = sum;
                        }
                    }
#pragma unroll
                    for (int c = 10; c < kTPartials; ++c) {
                        const float sum = wave_sum63(tm.v[c]);
                        if (lane == 63) wpart[wv][kk][c] = sum;
                    }
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < nb * kTPartials; i += NT) {
            const int kk = i / kTPartials, c = i - kk * kTPartials;
            float sum = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) sum += wpart[w][kk][c];
            part[(uint64_t)slots[kk] * kTPartials + c] = sum;
        }
    }
    // the front entries (blended first: T = 1, the colour behind is S now)
    TTerms tf;
#pragma unroll
    for (int c = 0; c < kTPartials; ++c) tf.v[c] = 0.f;
    if (inside && front_k >= 0) {
        const TRec e = load_trec(ents, sorted[b0 + front_k]);
        const THit h = thit(e, xr, yr, zn);
        const int id = (int)__float_as_uint(e.r2.w);
        const float c0 = scol[id], c1 = scol[a.n + id], c2 = scol[2 * a.n + id];
        const float dLda = dC[0] * (c0 - S0) + dC[1] * (c1 - S1) + dC[2] * (c2 - S2);
        const float dc[3] = {dC[0] * h.alpha, dC[1] * h.alpha, dC[2] * h.alpha};
        hit_terms(e, h, dLda, dc, xr, yr, tf);
    }
    if (!a.front_first) return;  // block-uniform
    __syncthreads();
    if (tid == 0) s_max = -1;
    __syncthreads();
    if (front_k >= 0) atomicMax(&s_max, front_k);
    __syncthreads();
    const int kmax = s_max;
    for (int kb0 = 0; kb0 <= kmax; kb0 += kBwdBatch) {
        const int nb = min(kBwdBatch, kmax + 1 - kb0);
        __syncthreads();
        if (tid < nb) slots[tid] = __float_as_uint(ents[(uint64_t)sorted[b0 + kb0 + tid] * 4 + 3].w);
        for (int kk = 0; kk < nb; ++kk) {
            const bool mine = front_k == kb0 + kk;
            if (__ballot((int)mine) != 0ull) {
#pragma unroll
                for (int c = 0; c < kTPartials; ++c) {
                    const float sum = wave_sum63(mine ? tf.v[c] : 0.f);
                    if (lane == 63) wpart[wv][kk][c] = sum;
                }
            } else if (lane == 63) {
#pragma unroll
                for (int c = 0; c < kTPartials; ++c) wpart[wv][kk][c] = 0.f;
            }
        }
        __syncthreads();
        for (int i = tid; i < nb * kTPartials; i += NT) {
            const int kk = i / kTPartials, c = i - kk * kTPartials;
            float sum = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) sum += wpart[w][kk][c];
            if (sum != 0.f) {
                float *dst = part + (uint64_t)slots[kk] * kTPartials + c;
                *dst = *dst + sum;  // this block wrote it above; the same thread order every run
            }
        }
    }
}

// Per surfel: gradients of the surfel's centre p, quaternion q, scales s,
// modulation w and SH from its entries' partials.  Per view the record was
//   mu = Rc p + t; tu, tv, n0 = Rc Rq(q / |q|) columns; w0 = n0 . mu;
//   n = sign(w0) n0, wp = |w0|; U = (wp tu - (mu . tu) n) / (s_u R),
//   V = (wp tv - (mu . tv) n) / (s_v R)   (R = sqrt(2 ln 255)),
// and the colour max(0, 1/2 + sum SH Y(d)), d = (o - p) / |o - p| (Eq. 1).
template <int K>
__global__ void __launch_bounds__(kTsBlock) k_tsurfels(FrameArgs a, float *g_mean, float *g_quat, float *g_scale,
                                                       float *g_w, float *g_sh) {
    using D = double;
    constexpr int KS = 3 * K, KP = 3 * K + 1;  // SH floats per surfel; LDS row stride (odd: no bank conflicts)
    __shared__ float s_sh[kTsBlock * KP];
    const int64_t n = a.n;
    const int64_t jb = (int64_t)blockIdx.x * kTsBlock;
    const int tid = (int)threadIdx.x;
    const int64_t j = jb + tid;
    const bool valid = j < n;
    const int nb = (int)(n - jb < kTsBlock ? n - jb : kTsBlock);
    // the block's SH, [surfel][K][3] contiguous in memory: one coalesced read,
    // a full block's loads all issued before the first wait
    if (nb == kTsBlock) {
        float t[KS];
#pragma unroll
        for (int r = 0; r < KS; ++r) t[r] = a.S.sh[jb * KS + tid + r * kTsBlock];
#pragma unroll
        for (int r = 0; r < KS; ++r) {
            const int i = tid + r * kTsBlock;
            s_sh[(i / KS) * KP + i % KS] = t[r];
        }
    } else {
        for (int i = tid; i < nb * KS; i += kTsBlock) s_sh[(i / KS) * KP + i % KS] = a.S.sh[jb * KS + i];
    }
    __syncthreads();
    const int64_t jr = valid ? j : jb;  // a valid surfel to read for the tail's idle threads
    const D p0 = a.S.mean[jr], p1 = a.S.mean[n + jr], p2 = a.S.mean[2 * n + jr];
    const D q0 = a.S.quat[jr], q1 = a.S.quat[n + jr], q2 = a.S.quat[2 * n + jr], q3 = a.S.quat[3 * n + jr];
    const D su = a.S.scale[jr], sv = a.S.scale[n + jr];
    const D R = a.opt.surfel_radius;
    const D qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    D gp[3] = {0, 0, 0}, gRq[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gsu = 0, gsv = 0, gw = 0;
    float gsh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    const bool ok = valid && qn > 0 && su > 0 && sv > 0;
    D Rq[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (ok) quat_rot(q0 / qn, q1 / qn, q2 / qn, q3 / qn, Rq);
    const uint32_t *boff = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff);
    const float *part = reinterpret_cast<const float *>(a.ws + a.L.t_part);
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const int T = a.opt.raster_tile;
    for (int v = 0; v < a.n_views && ok; ++v) {
        const int64_t vj = (int64_t)v * n + j;
        int x0, y0, x1, y1;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
        if (x0 > x1) continue;
        D P[kTPartials];
#pragma unroll
        for (int c = 0; c < kTPartials; ++c) P[c] = 0;
        const uint64_t k0 = boff[vj];
        const int ntile = (x1 / T - x0 / T + 1) * (y1 / T - y0 / T + 1);
        bool any = false;
        for (int kk = 0; kk < ntile; ++kk) {  // no occluders: every slot the count walked is used
            if (k0 + kk >= cap) break;
            any = true;
            const float *src = part + (k0 + kk) * kTPartials;
#pragma unroll
            for (int c = 0; c < kTPartials; ++c) P[c] += (D)src[c];
        }
        if (!any) continue;
        const ViewDev &V = a.views[v];
        D Rc[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Rc[c] = V.R[c];
        D mu[3], tu[3], tv[3], nn[3];
        for (int r = 0; r < 3; ++r) {
            mu[r] = Rc[3 * r] * p0 + Rc[3 * r + 1] * p1 + Rc[3 * r + 2] * p2 + V.t[r];
            tu[r] = Rc[3 * r] * Rq[0] + Rc[3 * r + 1] * Rq[3] + Rc[3 * r + 2] * Rq[6];
            tv[r] = Rc[3 * r] * Rq[1] + Rc[3 * r + 1] * Rq[4] + Rc[3 * r + 2] * Rq[7];
            nn[r] = Rc[3 * r] * Rq[2] + Rc[3 * r + 1] * Rq[5] + Rc[3 * r + 2] * Rq[8];
        }
        const D w0 = nn[0] * mu[0] + nn[1] * mu[1] + nn[2] * mu[2];
        const D sg = w0 < 0 ? -1.0 : 1.0;
        D nf[3] = {sg * nn[0], sg * nn[1], sg * nn[2]};
        const D wp = sg * w0;
        const D mut = mu[0] * tu[0] + mu[1] * tu[1] + mu[2] * tu[2];
        const D muv = mu[0] * tv[0] + mu[1] * tv[1] + mu[2] * tv[2];
        const D iu = 1.0 / (su * R), iv = 1.0 / (sv * R);
        const D gU[3] = {P[0], P[1], P[2]}, gV[3] = {P[3], P[4], P[5]};
        D gn[3] = {P[6], P[7], P[8]};
        gw += P[9];
        // U = (wp tu - mut n) iu, V = (wp tv - muv n) iv
        D gwp = 0, gmut = 0, gmuv = 0, gtu[3], gtv[3], gmu[3] = {0, 0, 0};
        D Uv = 0, Vv = 0;  // U . gU, V . gV (for the scales)
        for (int c = 0; c < 3; ++c) {
            const D Uc = (wp * tu[c] - mut * nf[c]) * iu, Vc = (wp * tv[c] - muv * nf[c]) * iv;
            Uv += Uc * gU[c];
            Vv += Vc * gV[c];
            gwp += (gU[c] * tu[c]) * iu + (gV[c] * tv[c]) * iv;
            gtu[c] = gU[c] * wp * iu;
            gtv[c] = gV[c] * wp * iv;
            gmut -= gU[c] * nf[c] * iu;
            gmuv -= gV[c] * nf[c] * iv;
            gn[c] -= mut * gU[c] * iu + muv * gV[c] * iv;
        }
        gsu -= Uv / su;
        gsv -= Vv / sv;
        // wp = n . mu, mut = mu . tu, muv = mu . tv
        for (int c = 0; c < 3; ++c) {
            gn[c] += gwp * mu[c];
            gmu[c] += gwp * nf[c] + gmut * tu[c] + gmuv * tv[c];
            gtu[c] += gmut * mu[c];
            gtv[c] += gmuv * mu[c];
        }
        // n = sg n0; tu, tv, n0 = Rc (columns of Rq); mu = Rc p + t
        for (int c = 0; c < 3; ++c) {
            gRq[3 * c] += Rc[c] * gtu[0] + Rc[3 + c] * gtu[1] + Rc[6 + c] * gtu[2];
            gRq[3 * c + 1] += Rc[c] * gtv[0] + Rc[3 + c] * gtv[1] + Rc[6 + c] * gtv[2];
            gRq[3 * c + 2] += sg * (Rc[c] * gn[0] + Rc[3 + c] * gn[1] + Rc[6 + c] * gn[2]);
            gp[c] += Rc[c] * gmu[0] + Rc[3 + c] * gmu[1] + Rc[6 + c] * gmu[2];
        }
        // colour: c = max(0, 1/2 + sum SH Y(d)); the forward's clamp decision
        // is read back from the stored colour (0: clamped)
        const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol) + (int64_t)v * 3 * n;
        float dx = V.o[0] - (float)p0, dy = V.o[1] - (float)p1, dz = V.o[2] - (float)p2;
        const float idl = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= idl; dy *= idl; dz *= idl;
        float Y[K];
        sh_basis(dx, dy, dz, K, Y);
        float wdir[K];
#pragma unroll
        for (int k = 0; k < K; ++k) wdir[k] = 0.f;
        const float *sh = s_sh + tid * KP;
        for (int ch = 0; ch < 3; ++ch) {
            if (!(scol[ch * n + j] > 0.f)) continue;
            const float gc = (float)P[10 + ch];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                gsh[k][ch] += Y[k] * gc;
                wdir[k] += gc * sh[k * 3 + ch];
            }
        }
        float gd[3];
        sh_grad_dot(dx, dy, dz, K, wdir, gd);
        const float dot = gd[0] * dx + gd[1] * dy + gd[2] * dz;
        gp[0] -= (D)((gd[0] - dot * dx) * idl);
        gp[1] -= (D)((gd[1] - dot * dy) * idl);
        gp[2] -= (D)((gd[2] - dot * dz) * idl);
    }
    // rotation matrix of the normalised quaternion -> its components, then
    // the normalisation (as for the Gaussians)
    D gq[4] = {0, 0, 0, 0};
    if (ok) {
        const D qw = q0 / qn, qx = q1 / qn, qy = q2 / qn, qz = q3 / qn;
        const D *gR = gRq;
        const D gqw = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
        const D gqx = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                             qw * gR[7] - 2.0 * qx * gR[8]);
        const D gqy = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                             qz * gR[7] - 2.0 * qy * gR[8]);
        const D gqz = 2.0 * (-2.0 * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.0 * qz * gR[4] +
                             qy * gR[5] + qx * gR[6] + qy * gR[7]);
        const D dq = gqw * qw + gqx * qx + gqy * qy + gqz * qz;
        gq[0] = (gqw - dq * qw) / qn;
        gq[1] = (gqx - dq * qx) / qn;
        gq[2] = (gqy - dq * qy) / qn;
        gq[3] = (gqz - dq * qz) / qn;
    }
    if (valid) {
        for (int c = 0; c < 3; ++c) put_nt(g_mean + c * n + j, (float)gp[c]);
        for (int c = 0; c < 4; ++c) put_nt(g_quat + c * n + j, (float)gq[c]);
        put_nt(g_scale + j, (float)gsu);
        put_nt(g_scale + n + j, (float)gsv);
        put_nt(g_w + j, (float)gw);
    }
    // the SH gradient through the same LDS rows: one coalesced write
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) s_sh[tid * KP + k * 3 + ch] = gsh[k][ch];
    __syncthreads();
    if (nb == kTsBlock) {
#pragma unroll
        for (int r = 0; r < KS; ++r) {
            const int i = tid + r * kTsBlock;
            put_nt(g_sh + jb * KS + i, s_sh[(i / KS) * KP + i % KS]);
        }
    } else {
        for (int i = tid; i < nb * KS; i += kTsBlock) put_nt(g_sh + jb * KS + i, s_sh[(i / KS) * KP + i % KS]);
    }
}

}  // namespace

hipError_t launch_tblend(const FrameArgs &a, float *color, float *alpha, float *depth, int32_t *front, hipStream_t s) {
    const dim3 grid((unsigned)a.L.rtiles);
    if (a.opt.raster_tile == 8)
        hipLaunchKernelGGL(k_tblend<8>, grid, dim3(64), 0, s, a, color, alpha, depth, front);
    else
        hipLaunchKernelGGL(k_tblend<16>, grid, dim3(256), 0, s, a, color, alpha, depth, front);
    return hipGetLastError();
}

hipError_t launch_tblend_bwd(const FrameArgs &a, const float *d_color, hipStream_t s) {
    const dim3 grid((unsigned)a.L.rtiles);
    if (a.opt.raster_tile == 8)
        hipLaunchKernelGGL(k_tblend_bwd<8>, grid, dim3(64), 0, s, a, d_color);
    else
        hipLaunchKernelGGL(k_tblend_bwd<16>, grid, dim3(256), 0, s, a, d_color);
    return hipGetLastError();
}

hipError_t launch_tsurfels(const FrameArgs &a, float *g_mean, float *g_quat, float *g_scale, float *g_w, float *g_sh,
                           hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + kTsBlock - 1) / kTsBlock)), block(kTsBlock);
    switch (a.ks) {
        case 1: hipLaunchKernelGGL(k_tsurfels<1>, grid, block, 0, s, a, g_mean, g_quat, g_scale, g_w, g_sh); break;
        case 4: hipLaunchKernelGGL(k_tsurfels<4>, grid, block, 0, s, a, g_mean, g_quat, g_scale, g_w, g_sh); break;
        case 9: hipLaunchKernelGGL(k_tsurfels<9>, grid, block, 0, s, a, g_mean, g_quat, g_scale, g_w, g_sh); break;
        default: hipLaunchKernelGGL(k_tsurfels<16>, grid, block, 0, s, a, g_mean, g_quat, g_scale, g_w, g_sh); break;
    }
    return hipGetLastError();
}

}  // namespace ges
