// Backward kernels: gradient of a loss L given dL/dC for the parameters the
// joint optimisation stage trains (Sec. 4.2): Gaussian p, r, s, sigma, SH
// and surfel SH.  No float atomics: every float sum runs in a fixed order
// (and the one sum taken with atomics is in integers), so the result is
// bitwise reproducible and independent of the Gaussian order.
//
// Per pixel, from Eq. 5 with S = W_s + W_G:
//   dL/dC_s = W_s g / S,   dL/dC_G = g / S,   dL/dW_G = -sum_c g_c C_c / S.
//
//   gauss tiles   per splat tile: one thread per (list entry, row of the
//                 entry's box inside the tile) walks the row, recomputing
//                 alpha exactly as the forward did, and sums dL/d(sigma,
//                 p_hat, conic, colour); the row sums of an entry are added
//                 in row order: one partial per list entry, stored at the
//                 entry's slot.
//   surfel tiles  per raster tile: the pixels are grouped by their winning
//                 surfel (LDS hash table of ids) and each group's dL/dC_s is
//                 summed in 64-bit fixed point (LDS integer atomics, exact
//                 and order-free): one partial per (surfel, tile) that shows
//                 it, at its slot; the other slots were zeroed first.
//   gaussians     per Gaussian: its partials are one contiguous slot run per
//                 view (the tiles of its box in row order, views in order),
//                 then the chain rule through the conic inverse, the EWA
//                 projection (Jacobian with its clamp), the projected centre,
//                 Sigma3 = R S S R^T, the quaternion normalisation and the SH
//                 colour including its view-direction dependence.
//   surfels       per surfel: partials summed the same way, times the SH
//                 basis (zero where the colour clamp is active).
#include "ges_internal.h"

namespace ges {

namespace {

constexpr int kPartials = kGaussPartials;

template <int TW, int TH>
__device__ void bwd_gauss_tile(const FrameArgs &a, const TileOrd o, const float *depth, const float *color_s,
                               const float *accum, const float *d_image) {
    const int t = (int)o.tile;
    constexpr int NT = TW * TH;
    // per-pixel state with rows padded to TW + 1: lanes that walk different
    // rows of one column would otherwise hit the same few LDS banks
    constexpr int RS = TW + 1;
    constexpr int kWin = 64;  // list entries looked at per batch: one per lane of wave 0
    __shared__ float s_g[TH * RS][3];
    __shared__ float s_gw[TH * RS];
    __shared__ float s_ds[TH * RS];
    __shared__ GRec s_rec[kWin];
    __shared__ uint32_t s_lb[kWin], s_slot[kWin], s_fb[kWin];
    __shared__ uint8_t s_fe[NT];              // fragment -> entry of the batch
    __shared__ float s_pb[kPartials][NT];     // fragment (row) sums
    __shared__ int s_nb, s_nf;
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int tx0 = (lt % V.stx) * TW, ty0 = (lt / V.stx) * TH;
    const int tid = (int)threadIdx.x;
    const int64_t P = (int64_t)V.W * V.H;
    const float ws = a.opt.w_s;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, gw = 0.f, ds = -__int_as_float(0x7f800000);
    {
        const int px = tx0 + tid % TW, py = ty0 + tid / TW;
        if (px < V.W && py < V.H) {
            const int64_t lp = (int64_t)py * V.W + px;
            const float *cs = color_s + 3 * V.pix_off + lp;
            const float *ac = accum + 4 * V.pix_off + lp;
            const float *dg = d_image + 3 * V.pix_off + lp;
            const float inv = 1.f / (ws + ac[3 * P]);
            const float c0 = (ws * cs[0] + ac[0]) * inv;
            const float c1 = (ws * cs[P] + ac[P]) * inv;
            const float c2 = (ws * cs[2 * P] + ac[2 * P]) * inv;
            g0 = dg[0] * inv;
            g1 = dg[P] * inv;
            g2 = dg[2 * P] * inv;
            gw = -(g0 * c0 + g1 * c1 + g2 * c2);
            ds = depth[V.pix_off + lp];
        }
    }
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);
    if (b0 >= b1) return;  // no Gaussian reaches this tile
    {
        const int li = (tid / TW) * RS + tid % TW;
        s_g[li][0] = g0;
        s_g[li][1] = g1;
        s_g[li][2] = g2;
        s_gw[li] = gw;
        s_ds[li] = ds;
    }

    const GEnt *ents = reinterpret_cast<const GEnt *>(a.ws + a.L.g_ents);
    float *part = reinterpret_cast<float *>(a.ws + a.L.g_part);
    const float amin = a.opt.alpha_min;
    // Batches of list entries whose box rows inside the tile number at most
    // NT: every (entry, box row) is a fragment, one per thread, which walks
    // its row left to right and sums the entry's nine terms over it.  The
    // row sums of an entry are then added in row order, so each partial is
    // the same sum whichever thread computed which row, and the whole is
    // independent of the list order.  One fragment per thread keeps the
    // lanes of a wave on rows of similar length instead of running each
    // wave as long as the largest of its entries.
    for (uint64_t next = b0; next < b1;) {
        if (tid < 64) {
            const uint64_t pos = next + (uint64_t)tid;
            const bool have = pos < b1;
            // the 64-byte entry as four 16-byte loads: the record, then
            // (slot, lbox, gauss, pad)
            float4 e0 = {}, e1 = {}, e2 = {}, e3 = {};
            int h = 0;
            if (have) {
                const float4 *src = reinterpret_cast<const float4 *>(ents + pos);
                e0 = src[0];
                e1 = src[1];
                e2 = src[2];
                e3 = src[3];
                const uint32_t lb = __float_as_uint(e3.y);
                h = (int)((lb >> 12) & 15) - (int)((lb >> 8) & 15) + 1;
            }
            const int incl = wave_scan_add(h, true);
            const bool take = have && incl <= NT;
            if (take) {
                float4 *dst = reinterpret_cast<float4 *>(&s_rec[tid]);
                dst[0] = e0;
                dst[1] = e1;
                dst[2] = e2;
                s_slot[tid] = __float_as_uint(e3.x);
                s_lb[tid] = __float_as_uint(e3.y);
                s_fb[tid] = (uint32_t)(incl - h);
                for (int r = 0; r < h; ++r) s_fe[incl - h + r] = (uint8_t)tid;
            }
            const uint64_t tm = __ballot(take);
            const int nb = __popcll(tm);  // a prefix of the lanes: heights are >= 1
            if (tid == nb - 1) {
                s_nb = nb;
                s_nf = incl;
            }
        }
        __syncthreads();
        const int nb = s_nb, nf = s_nf;
        if (tid < nf) {
            const int e = s_fe[tid];
            const GRec g = s_rec[e];
            const uint32_t lb = s_lb[e];
            const int x0 = tx0 + (int)(lb & 15), x1 = tx0 + (int)((lb >> 4) & 15);
            const int yy = ty0 + (int)((lb >> 8) & 15) + (tid - (int)s_fb[e]);
            const float cr = g.r * (float)kFixInv, cg = g.g * (float)kFixInv, cb = g.b * (float)kFixInv;
            const float isig = 1.f / g.sigma;
            float acc[kPartials];
#pragma unroll
            for (int k = 0; k < kPartials; ++k) acc[k] = 0.f;
            const int row = (yy - ty0) * RS - tx0;
            for (int xx = x0; xx <= x1; ++xx) {
                const int lp = row + xx;
                float dx, dy, q;
                const float al = gauss_alpha(g, (float)xx + 0.5f, (float)yy + 0.5f, dx, dy, q);
                if (!((al >= amin) & (g.dme < s_ds[lp]))) continue;
                const float G0 = s_g[lp][0], G1 = s_g[lp][1], G2 = s_g[lp][2];
                const float dLda = G0 * cr + G1 * cg + G2 * cb + s_gw[lp];
                acc[0] += dLda * al * isig;
                const float t1 = al * dLda;
                acc[1] += t1 * (g.ca * dx + g.cb * dy);
                acc[2] += t1 * (g.cb * dx + g.cc * dy);
                const float dq = -0.5f * t1;
                acc[3] += dq * dx * dx;
                acc[4] += dq * 2.f * dx * dy;
                acc[5] += dq * dy * dy;
                acc[6] += al * G0;
                acc[7] += al * G1;
                acc[8] += al * G2;
            }
#pragma unroll
            for (int k = 0; k < kPartials; ++k) s_pb[k][tid] = acc[k];
        }
        __syncthreads();
        for (int i = tid; i < nb * kPartials; i += NT) {
            const int e = i / kPartials, k = i - e * kPartials;
            const uint32_t lb = s_lb[e];
            const int h = (int)((lb >> 12) & 15) - (int)((lb >> 8) & 15) + 1;
            const float *src = &s_pb[k][s_fb[e]];
            float sum = src[0];
            for (int r = 1; r < h; ++r) sum += src[r];
            part[(uint64_t)s_slot[e] * kPartials + k] = sum;  // slot order
        }
        next += (uint64_t)nb;
        __syncthreads();  // the next batch reuses the entry and fragment tables
    }
}

// dL/dC_s summed per (raster tile, visible surfel) over the pixels that show
// that surfel.  The tile's pixels are grouped by their surfel through an LDS
// hash table of the ids (open addressing, twice as many slots as pixels, so
// a free slot always exists), and each pixel adds its three terms into its
// surfel's slot as 64-bit fixed point: the scale is the power of two that
// puts the tile's largest term just under 2^54, so a sum of at most 256
// terms stays below 2^62 and every term keeps its bits down to 2^-54 of that
// largest one.  Integer addition is associative: the sums do not depend on
// the order of the atomics, and they are reproducible.  One thread per
// occupied slot stores the sum at the surfel's slot for this tile (its slot
// run offset plus the tile's place in its box); slots of surfels that win no
// pixel here keep the zero written before this kernel.
template <int T>
__device__ void bwd_surfel_tile(const FrameArgs &a, int t, const int32_t *sid, const float *accum,
                                const float *d_image) {
    constexpr int NT = T * T;
    constexpr int NW = NT / 64;
    constexpr int HS = 2 * NT;  // hash slots (a power of two)
    __shared__ uint32_t h_id[HS];
    __shared__ unsigned long long h_acc[3][HS];
    __shared__ uint32_t w_max[NW];
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_toff);
    if (toff[t * kCounterCopies] >= toff[(t + 1) * kCounterCopies]) return;  // no surfel reaches this tile
    const int v = view_of_rtile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.rt_off;
    const int tx = lt % V.rtx, ty = lt / V.rtx;
    const int px = tx * T + tid % T, py = ty * T + tid / T;  // a point of the sample grid
    const int64_t P = (int64_t)V.W * V.H;
    const float ws = a.opt.w_s;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    int id = -1;
    if (px < V.sW && py < V.sH) {
        id = sid[V.s_off + (int64_t)py * V.sW + px];
        // the pixel of this sample; with 4 samples each carries a quarter of C_s
        const int half = V.sW > V.W ? 1 : 0;
        const int64_t lp = (int64_t)(py >> half) * V.W + (px >> half);
        if (id >= 0) {
            const float inv = (half ? 0.25f * ws : ws) / (ws + accum[4 * V.pix_off + 3 * P + lp]);
            const float *dg = d_image + 3 * V.pix_off + lp;
            g0 = dg[0] * inv;
            g1 = dg[P] * inv;
            g2 = dg[2 * P] * inv;
        }
    }
    for (int i = tid; i < HS; i += NT) {
        h_id[i] = 0xFFFFFFFFu;
        h_acc[0][i] = h_acc[1][i] = h_acc[2][i] = 0ull;
    }
    // the tile's largest |term|, as float bits (non-negative floats order as their bits)
    const uint32_t mb = wave_max_u32(__float_as_uint(fmaxf(fabsf(g0), fmaxf(fabsf(g1), fabsf(g2)))));
    if (lane == 0) w_max[wv] = mb;
    __syncthreads();
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) m = max(m, w_max[w]);
    // |term| < 2^E with E from the exponent field (denormals: E = -126); a
    // non-finite term (exponent field 255) makes every partial of the tile NaN
    const bool finite = ((m >> 23) & 255u) != 255u;
    const int E = finite ? (int)((m >> 23) & 255u) - 126 : 0;
    const int sh = 54 - E;  // scale 2^sh: terms below 2^54
    if (id >= 0) {
        if (!finite) g0 = g1 = g2 = 0.f;  // the slot's value is NaN regardless
        uint32_t h = ((uint32_t)id * 2654435761u) & (HS - 1);
        for (;;) {  // ends: fewer distinct ids than slots
            const uint32_t prev = atomicCAS(&h_id[h], 0xFFFFFFFFu, (uint32_t)id);
            if (prev == 0xFFFFFFFFu || prev == (uint32_t)id) break;
            h = (h + 1) & (HS - 1);
        }
        atomicAdd(&h_acc[0][h], (unsigned long long)__double2ll_rn(ldexp((double)g0, sh)));
        atomicAdd(&h_acc[1][h], (unsigned long long)__double2ll_rn(ldexp((double)g1, sh)));
        atomicAdd(&h_acc[2][h], (unsigned long long)__double2ll_rn(ldexp((double)g2, sh)));
    }
    __syncthreads();
    for (int i = tid; i < HS; i += NT) {
        const uint32_t sidv = h_id[i];
        if (sidv == 0xFFFFFFFFu) continue;
        const int64_t vj = (int64_t)v * a.n + (int64_t)sidv;
        int x0, y0, x1, y1;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
        const uint64_t k = (uint64_t)reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff)[vj] +
                           (uint64_t)((ty - y0 / T) * (x1 / T - x0 / T + 1) + (tx - x0 / T));
        if (k >= (uint64_t)a.L.s_cap) continue;  // overflowed frame: flagged by the scan total
        float *dst = reinterpret_cast<float *>(a.ws + a.L.s_part) + k * 3;
        const float nan = __int_as_float(0x7fc00000);
        dst[0] = finite ? (float)ldexp((double)(long long)h_acc[0][i], -sh) : nan;
        dst[1] = finite ? (float)ldexp((double)(long long)h_acc[1][i], -sh) : nan;
        dst[2] = finite ? (float)ldexp((double)(long long)h_acc[2][i], -sh) : nan;
    }
}

// Active Gaussians (a list entry in some view; g_act scanned into g_aoff)
// go to the dense active list in index order, so the FP64 chain below runs
// only on full waves of active ones.  Every gradient is zeroed here (whole
// cache lines; the chain overwrites the active ones afterwards).
// Gradient outputs are written once and not read again in the frame:
// non-temporal stores stream them out instead of leaving them dirty in the
// caches, where their write-back would fall into the next frame's first
// kernels and evict the parameters those kernels read.
__device__ __forceinline__ void put_nt(float *p, float v) { __builtin_nontemporal_store(v, p); }

__device__ void bwd_compact_one(const FrameArgs &a, const ges_gradients &gr, int64_t i) {
    if (i >= a.m) return;
    const int64_t m = a.m;
    const uint32_t *off = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_aoff);
    const uint32_t o = off[i];
    if (off[i + 1] > o && o < (uint64_t)m) reinterpret_cast<uint32_t *>(a.ws + a.L.g_alist)[o] = (uint32_t)i;
    for (int c = 0; c < 3; ++c) put_nt(gr.mean + c * m + i, 0.f);
    for (int c = 0; c < 4; ++c) put_nt(gr.quat + c * m + i, 0.f);
    for (int c = 0; c < 3; ++c) put_nt(gr.scale + c * m + i, 0.f);
    put_nt(gr.opacity + i, 0.f);
    // the SH gradient is [m][K][3]; it is cleared whole here, as 3K runs of
    // m floats so that a wave's stores stay contiguous
    for (int k = 0; k < 3 * a.kg; ++k) put_nt(gr.sh + k * m + i, 0.f);
}

// Per active Gaussian: partials gathered in a fixed order, then the chain
// rule in FP64 (parameter gradients are sums of terms of both signs; FP64
// keeps their cancellation far below the FP32 rounding of the inputs).  row:
// the Gaussian's SH coefficients ([K][3], in LDS); the SH gradient replaces
// them there.  MV: several views, whose SH gradients add up in registers;
// with one view each channel's gradient overwrites its coefficients as soon
// as it is known (48 fewer live registers).  With one view the partial sums
// come gathered by the wave (Pg; gathered: the Gaussian kept a tile).
template <int K, bool MV>
__device__ void bwd_gaussian_one(const FrameArgs &a, const ges_gradients &gr, int64_t i, float *row,
                                 const double (&Pg)[kGaussPartials], bool gathered) {
    using D = double;
    const int64_t m = a.m;
    bool sh_done = false;  // one view: the row holds gradients (else coefficients)
    const D px = a.G.mean[i], py = a.G.mean[m + i], pz = a.G.mean[2 * m + i];
    const D q0 = a.G.quat[i], q1 = a.G.quat[m + i], q2 = a.G.quat[2 * m + i], q3 = a.G.quat[3 * m + i];
    const D s0 = a.G.scale[i], s1 = a.G.scale[m + i], s2 = a.G.scale[2 * m + i];
    const D qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const D qw = q0 / qn, qx = q1 / qn, qy = q2 / qn, qz = q3 / qn;
    // Sigma3 (symmetric: xx, xy, xz, yy, yz, zz)
    D S3[6];
    {
        D Rq[9];
        quat_rot(qw, qx, qy, qz, Rq);
        D Mm[9];
        for (int r = 0; r < 3; ++r) {
            Mm[3 * r] = Rq[3 * r] * s0;
            Mm[3 * r + 1] = Rq[3 * r + 1] * s1;
            Mm[3 * r + 2] = Rq[3 * r + 2] * s2;
        }
        auto dot3 = [&](int r, int c) { return Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2]; };
        S3[0] = dot3(0, 0); S3[1] = dot3(0, 1); S3[2] = dot3(0, 2);
        S3[3] = dot3(1, 1); S3[4] = dot3(1, 2); S3[5] = dot3(2, 2);
    }
    // Mip-GES world-space filter: the projection sees Sigma3 + v I and the
    // opacity is scaled by c3 = prod s / sqrt(s^2 + v) (v: an input, no gradient)
    const D v3 = a.G.filter3d ? (D)a.G.filter3d[i] : 0.0;
    const D c3 = a.G.filter3d ? (s0 / sqrt(s0 * s0 + v3)) * (s1 / sqrt(s1 * s1 + v3)) * (s2 / sqrt(s2 * s2 + v3)) : 1.0;
    const D Sf[9] = {S3[0] + v3, S3[1], S3[2], S3[1], S3[3] + v3, S3[4], S3[2], S3[4], S3[5] + v3};
    const D sig = a.G.opacity[i];
    const bool mip = a.opt.mip_2d > 0.f;
    D gc3 = 0;  // dL/dc3

    D gp0 = 0, gp1 = 0, gp2 = 0;  // dL/dp (world)
    D gS[6] = {0, 0, 0, 0, 0, 0};  // dL/dSigma3 (symmetric, full-matrix convention)
    D gsig = 0;
    float gsh[MV ? K : 1][3];
    if (MV) {
#pragma unroll
        for (int k = 0; k < (MV ? K : 1); ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    }

    const uint32_t *boff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_boff);
    const uint32_t *nkept = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_nkept);
    const float *part = reinterpret_cast<const float *>(a.ws + a.L.g_part);

    for (int v = 0; v < a.n_views; ++v) {
        const int64_t vi = (int64_t)v * m + i;
        int x0, y0, x1, y1;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.gbox)[vi], x0, y0, x1, y1);
        if (x0 > x1) continue;
        const ViewDev &V = a.views[v];
        D P[kPartials];
#pragma unroll
        for (int k = 0; k < kPartials; ++k) P[k] = 0;
        // the partials of the tiles the depth cull kept are the first nk
        // places of the Gaussian's run (kept tiles in row order; a place lost
        // to an overflow holds zeros): kGather of them per round of loads,
        // added in that order
        if (!MV) {
#pragma unroll
            for (int k = 0; k < kPartials; ++k) P[k] = Pg[k];
        }
        const uint64_t k0 = boff[vi];
        const uint32_t nk = MV ? nkept[vi] : 0u;
        const bool any = MV ? nk > 0 : gathered;
        constexpr int kGather = 4;
        for (uint32_t kk0 = 0; kk0 < nk; kk0 += kGather) {
            float pv[kGather][kPartials];
#pragma unroll
            for (int u = 0; u < kGather; ++u) {
                const float *src = part + (k0 + kk0 + u) * kPartials;  // the run is contiguous
#pragma unroll
                for (int c = 0; c < kPartials; ++c) pv[u][c] = kk0 + u < nk ? src[c] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kGather; ++u)
                if (kk0 + u < nk) {
#pragma unroll
                    for (int c = 0; c < kPartials; ++c) P[c] += (D)pv[u][c];
                }
        }
        if (!any) continue;
        D Rc[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) Rc[c] = V.R[c];
        const D fx = V.fx, fy = V.fy;
        const D mx = Rc[0] * px + Rc[1] * py + Rc[2] * pz + V.t[0];
        const D my = Rc[3] * px + Rc[4] * py + Rc[5] * pz + V.t[1];
        const D mz = Rc[6] * px + Rc[7] * py + Rc[8] * pz + V.t[2];
        const D iz = 1.0 / mz;
        const D rx = mx * iz, ry = my * iz;
        const D limx = V.limx, limy = V.limy;
        const D ux = fmin(fmax(rx, -limx), limx);
        const D uy = fmin(fmax(ry, -limy), limy);
        const D J00 = fx * iz, J02 = -fx * ux * iz;
        const D J11 = fy * iz, J12 = -fy * uy * iz;
        D T[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T[c] = J00 * Rc[c] + J02 * Rc[6 + c];
            T[3 + c] = J11 * Rc[3 + c] + J12 * Rc[6 + c];
        }
        D TS[6];  // T Sigma3
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                TS[3 * r + c] = T[3 * r] * Sf[c] + T[3 * r + 1] * Sf[3 + c] + T[3 * r + 2] * Sf[6 + c];
        const D dil = mip ? (D)a.opt.mip_2d : (D)a.opt.dilation;
        const D bxx = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2];
        const D cxy = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
        const D byy = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5];
        const D cxx = bxx + dil, cyy = byy + dil;
        const D idet = 1.0 / (cxx * cyy - cxy * cxy);
        const D A00 = cyy * idet, A01 = -cxy * idet, A11 = cxx * idet;
        // dL/dSigma2 = -A G_A A with G_A = [[ga, gb/2], [gb/2, gc]]
        const D ga = P[3], gb = 0.5 * P[4], gc = P[5];
        const D B00 = ga * A00 + gb * A01, B01 = ga * A01 + gb * A11;
        const D B10 = gb * A00 + gc * A01, B11 = gb * A01 + gc * A11;
        D G00 = -(A00 * B00 + A01 * B10);
        D G01 = -(A00 * B01 + A01 * B11);
        D G11 = -(A01 * B01 + A11 * B11);
        // P[0] is dL/d(sigma_eff), sigma_eff = sigma c3 c2
        D c2 = 1.0;
        if (mip) {
            // c2 = sqrt(det B / det(B + e I)), B the unfiltered Sigma2:
            // dc2 = c2/2 tr((B^-1 - (B + e I)^-1) dB)
            const D detb = bxx * byy - cxy * cxy;
            c2 = detb > 0 ? sqrt(detb * idet) : 0.0;
            if (detb > 0) {
                const D ib = 1.0 / detb;
                const D g2 = P[0] * sig * c3 * 0.5 * c2;
                G00 += g2 * (byy * ib - A00);
                G01 += g2 * (-cxy * ib - A01);
                G11 += g2 * (bxx * ib - A11);
            }
        }
        gc3 += P[0] * sig * c2;
        // dL/dSigma3 += T^T G2 T
        auto tgt = [&](int r, int c) {
            return T[r] * (G00 * T[c] + G01 * T[3 + c]) + T[3 + r] * (G01 * T[c] + G11 * T[3 + c]);
        };
        gS[0] += tgt(0, 0); gS[1] += tgt(0, 1); gS[2] += tgt(0, 2);
        gS[3] += tgt(1, 1); gS[4] += tgt(1, 2); gS[5] += tgt(2, 2);
        // dL/dT = 2 G2 T Sigma3 = 2 G2 TS; dL/dJ = dL/dT R^T
        D gT[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            gT[c] = 2.0 * (G00 * TS[c] + G01 * TS[3 + c]);
            gT[3 + c] = 2.0 * (G01 * TS[c] + G11 * TS[3 + c]);
        }
        const D gJ00 = gT[0] * Rc[0] + gT[1] * Rc[1] + gT[2] * Rc[2];
        const D gJ02 = gT[0] * Rc[6] + gT[1] * Rc[7] + gT[2] * Rc[8];
        const D gJ11 = gT[3] * Rc[3] + gT[4] * Rc[4] + gT[5] * Rc[5];
        const D gJ12 = gT[3] * Rc[6] + gT[4] * Rc[7] + gT[5] * Rc[8];
        D gmx = 0, gmy = 0, gmz = 0;
        const D iz2 = iz * iz;
        gmz += -fx * iz2 * gJ00 - fy * iz2 * gJ11 + fx * ux * iz2 * gJ02 + fy * uy * iz2 * gJ12;
        if (rx > -limx && rx < limx) {  // x/z not clamped: J02 depends on it
            const D gux = gJ02 * (-fx * iz);
            gmx += gux * iz;
            gmz += -gux * mx * iz2;
        }
        if (ry > -limy && ry < limy) {
            const D guy = gJ12 * (-fy * iz);
            gmy += guy * iz;
            gmz += -guy * my * iz2;
        }
        // projected centre
        gmx += P[1] * fx * iz;
        gmy += P[2] * fy * iz;
        gmz += -(P[1] * fx * mx + P[2] * fy * my) * iz2;
        // mu = R p + t
        gp0 += Rc[0] * gmx + Rc[3] * gmy + Rc[6] * gmz;
        gp1 += Rc[1] * gmx + Rc[4] * gmy + Rc[7] * gmz;
        gp2 += Rc[2] * gmx + Rc[5] * gmy + Rc[8] * gmz;
        gsig += P[0] * c3 * c2;
        // colour: c = max(0, 1/2 + sum SH Y(d)), d = (o - p)/|o - p|.  Its
        // gradient terms are plain products (no cancellation): FP32, as in
        // the forward, which also decides the clamp.
        float dx = V.o[0] - (float)px, dy = V.o[1] - (float)py, dz = V.o[2] - (float)pz;
        const float idl = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= idl; dy *= idl; dz *= idl;
        float Y[K];
        sh_basis(dx, dy, dz, K, Y);
        float w[K];
#pragma unroll
        for (int k2 = 0; k2 < K; ++k2) w[k2] = 0.f;
        for (int ch = 0; ch < 3; ++ch) {
            float coef[K];
            float raw = 0.5f;
#pragma unroll
            for (int k2 = 0; k2 < K; ++k2) {
                coef[k2] = row[k2 * 3 + ch];
                raw += coef[k2] * Y[k2];
            }
            if (!(raw > 0.f)) {  // clamped channel: no gradient
                if (!MV) {
#pragma unroll
                    for (int k2 = 0; k2 < K; ++k2) row[k2 * 3 + ch] = 0.f;
                }
                continue;
            }
            const float gcol = (float)P[6 + ch];
#pragma unroll
            for (int k2 = 0; k2 < K; ++k2) w[k2] += gcol * coef[k2];
            if (MV) {
#pragma unroll
                for (int k2 = 0; k2 < (MV ? K : 1); ++k2) {
                    if (ch == 0) gsh[k2][0] += Y[k2] * gcol;
                    else if (ch == 1) gsh[k2][1] += Y[k2] * gcol;
                    else gsh[k2][2] += Y[k2] * gcol;
                }
            } else {
#pragma unroll
                for (int k2 = 0; k2 < K; ++k2) row[k2 * 3 + ch] = Y[k2] * gcol;
            }
        }
        sh_done = true;
        float gd[3];
        sh_grad_dot(dx, dy, dz, K, w, gd);
        const float dot = gd[0] * dx + gd[1] * dy + gd[2] * dz;
        gp0 -= (D)((gd[0] - dot * dx) * idl);
        gp1 -= (D)((gd[1] - dot * dy) * idl);
        gp2 -= (D)((gd[2] - dot * dz) * idl);
    }

    // Sigma3 = M M^T, M = Rq diag(s): dL/dM = 2 gS M (gS symmetric)
    D Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    const D s[3] = {s0, s1, s2};
    const D gSf[9] = {gS[0], gS[1], gS[2], gS[1], gS[3], gS[4], gS[2], gS[4], gS[5]};
    D gs[3] = {0, 0, 0}, gR[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // (gS M)_{rc} with M_{kc} = Rq_{kc} s_c
            const D gm = 2.0 * (gSf[3 * r] * Rq[c] + gSf[3 * r + 1] * Rq[3 + c] + gSf[3 * r + 2] * Rq[6 + c]) * s[c];
            gs[c] += gm * Rq[3 * r + c];
            gR[3 * r + c] = gm * s[c];
        }
    // rotation matrix of the normalised quaternion -> its components
    const D gqw = 2.0 * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    const D gqx = 2.0 * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.0 * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                         qw * gR[7] - 2.0 * qx * gR[8]);
    const D gqy = 2.0 * (-2.0 * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                         qz * gR[7] - 2.0 * qy * gR[8]);
    const D gqz = 2.0 * (-2.0 * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.0 * qz * gR[4] +
                         qy * gR[5] + qx * gR[6] + qy * gR[7]);
    // normalisation q_bar = q / |q|
    const D dq = gqw * qw + gqx * qx + gqy * qy + gqz * qz;
    const D iqn = 1.0 / qn;
    put_nt(gr.quat + i, (float)((gqw - dq * qw) * iqn));
    put_nt(gr.quat + m + i, (float)((gqx - dq * qx) * iqn));
    put_nt(gr.quat + 2 * m + i, (float)((gqy - dq * qy) * iqn));
    put_nt(gr.quat + 3 * m + i, (float)((gqz - dq * qz) * iqn));
    put_nt(gr.mean + i, (float)gp0);
    put_nt(gr.mean + m + i, (float)gp1);
    put_nt(gr.mean + 2 * m + i, (float)gp2);
    if (a.G.filter3d) {  // dc3/ds_k = c3 v / (s_k (s_k^2 + v))
        gs[0] += gc3 * c3 * v3 / (s0 * (s0 * s0 + v3));
        gs[1] += gc3 * c3 * v3 / (s1 * (s1 * s1 + v3));
        gs[2] += gc3 * c3 * v3 / (s2 * (s2 * s2 + v3));
    }
    put_nt(gr.scale + i, (float)gs[0]);
    put_nt(gr.scale + m + i, (float)gs[1]);
    put_nt(gr.scale + 2 * m + i, (float)gs[2]);
    put_nt(gr.opacity + i, (float)gsig);
    if (MV) {
#pragma unroll
        for (int k = 0; k < (MV ? K : 1); ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) row[k * 3 + ch] = gsh[k][ch];
    } else if (!sh_done) {  // no kept tile reached (lost to an overflow): zero gradient
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) row[k] = 0.f;
    }
}

// The wave's active Gaussians (a prefix of its lanes) are handled one per
// lane; their SH runs ([m][K][3], 3K floats each) move between HBM and LDS
// with consecutive lanes on consecutive words of the runs, so a load or store
// instruction covers a few whole runs instead of one word of 64 scattered
// ones.  Rows are padded to 3K + 1 words: lanes reading their own rows hit
// distinct LDS banks.  The grid holds as many blocks as can be resident at
// once and strides over the active list (its length is known only on the
// device): a grid over all m Gaussians spent most of the kernel's time
// dispatching blocks with nothing to do through the few slots the working
// blocks (one wave per SIMD at this register count) left free.
// With one view the wave gathers the partial sums of its Gaussians
// together: the kept places of all 64 runs are numbered in lane order (a
// wave scan of the counts), each round loads 256 of them, four per lane,
// into LDS, and every lane then adds its own places in run order -- the
// order a lane walking its run alone would take, in a few rounds instead of
// one round per four places of the longest run in the wave.
constexpr int kGatherRound = 256;

template <int K, bool MV>
__global__ void __launch_bounds__(128) k_bwd_gaussians(FrameArgs a, ges_gradients gr) {
    constexpr int SK = 3 * K, RS = SK + 1;
    __shared__ float rows[2][64 * RS];
    __shared__ uint32_t ids[2][64];
    __shared__ float gbuf[MV ? 1 : 2][MV ? 1 : kGatherRound * kGaussPartials];
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    const uint64_t n_active = reinterpret_cast<const WsHeader *>(a.ws + a.L.header)->g_active;
    const uint64_t n = n_active < (uint64_t)a.m ? n_active : (uint64_t)a.m;
    float *wrow = rows[wv];
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t tid = base + threadIdx.x;
        const bool valid = tid < n;
        const unsigned long long vm = __ballot((int)valid);
        if (vm == 0ull) continue;  // wave-uniform
        const int nv = __popcll(vm);  // tid rises with the lane: the valid lanes are lanes 0 .. nv-1
        const int64_t i = valid ? (int64_t)reinterpret_cast<const uint32_t *>(a.ws + a.L.g_alist)[tid] : 0;
        ids[wv][lane] = (uint32_t)i;
        // the runs to LDS: all of a round's loads are issued before any store
        // (a store to LDS between two loads would make each load wait for
        // the one before); the run's Gaussian index comes from its lane
        constexpr int kRound = SK < 16 ? SK : 16;  // loads in flight per lane and round
        for (int c0 = 0; c0 < nv * SK; c0 += 64 * kRound) {
            float v[kRound];
#pragma unroll
            for (int u = 0; u < kRound; ++u) {
                const int c = c0 + lane + 64 * u, g = c / SK;
                const uint32_t id = (uint32_t)__shfl((int)i, g < 64 ? g : 63);
                v[u] = c < nv * SK ? a.G.sh[(int64_t)id * SK + (c - g * SK)] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kRound; ++u) {
                const int c = c0 + lane + 64 * u, g = c / SK;
                if (c < nv * SK) wrow[g * RS + (c - g * SK)] = v[u];
            }
        }
        double Pg[kGaussPartials] = {};
        bool gathered = false;
        if (!MV) {
            int nk = 0;
            uint64_t k0 = 0;
            if (valid) {
                int x0, y0, x1, y1;
                unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.gbox)[i], x0, y0, x1, y1);
                if (x0 <= x1) {
                    nk = (int)reinterpret_cast<const uint32_t *>(a.ws + a.L.g_nkept)[i];
                    k0 = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_boff)[i];
                }
            }
            gathered = nk > 0;
            const int incl = wave_scan_add(nk, true), excl = incl - nk;
            const int total = __shfl(incl, 63);
            const float *part = reinterpret_cast<const float *>(a.ws + a.L.g_part);
            float *buf = gbuf[MV ? 0 : wv];
            for (int f0 = 0; f0 < total; f0 += kGatherRound) {  // wave-uniform
                float pv[kGatherRound / 64][kGaussPartials];
#pragma unroll
                for (int u = 0; u < kGatherRound / 64; ++u) {
                    const int f = f0 + lane + 64 * u;
                    int o = 0;  // the last lane whose places start at or before f
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1)
                        if (__shfl(excl, o + step) <= f) o += step;
                    const int ex_o = __shfl(excl, o);
                    const uint64_t k0_o = ((uint64_t)(uint32_t)__shfl((int)(k0 >> 32), o) << 32) |
                                          (uint32_t)__shfl((int)(uint32_t)k0, o);
                    const float *src = part + (k0_o + (uint64_t)(f - ex_o)) * kGaussPartials;
#pragma unroll
                    for (int c = 0; c < kGaussPartials; ++c) pv[u][c] = f < total ? src[c] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < kGatherRound / 64; ++u)
#pragma unroll
                    for (int c = 0; c < kGaussPartials; ++c) buf[(lane + 64 * u) * kGaussPartials + c] = pv[u][c];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int b0 = excl > f0 ? excl : f0, b1 = incl < f0 + kGatherRound ? incl : f0 + kGatherRound;
                for (int f = b0; f < b1; ++f)
#pragma unroll
                    for (int c = 0; c < kGaussPartials; ++c) Pg[c] += (double)buf[(f - f0) * kGaussPartials + c];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // read before the next round writes
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid) bwd_gaussian_one<K, MV>(a, gr, i, wrow + lane * RS, Pg, gathered);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int c = lane; c < nv * SK; c += 64) {
            const int g = c / SK, q = c - g * SK;
            put_nt(gr.sh + (int64_t)ids[wv][g] * SK + q, wrow[g * RS + q]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // rows read before the next chunk writes them
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One view: the surfel's loads issued together before the visibility test.
// g receives the surfel's SH gradient (zero when it shows nowhere).
template <int K>
__device__ void bwd_surfel_one_view(const FrameArgs &a, int64_t j, float (&g)[K][3]) {
    const int64_t n = a.n;
    const unsigned char vis = a.ws[a.L.svis + j];
    const uint2 bx = reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[j];
    const uint64_t k0 = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff)[j];
    const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol);
    const float c0 = scol[j], c1 = scol[n + j], c2 = scol[2 * n + j];
    const float mx = a.S.mean[j], my = a.S.mean[n + j], mz = a.S.mean[2 * n + j];
    int x0, y0, x1, y1;
    unpack_box(bx, x0, y0, x1, y1);
    // the forward stored max(0, raw) for visible surfels: the clamp is
    // inactive exactly where that colour is positive (no SH re-read)
    const bool on0 = vis && c0 > 0.f, on1 = vis && c1 > 0.f, on2 = vis && c2 > 0.f;
    float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f;
    float Y[K];
#pragma unroll
    for (int k = 0; k < K; ++k) Y[k] = 0.f;
    if ((on0 || on1 || on2) && x0 <= x1) {
        const ViewDev &V = a.views[0];
        const int T = a.opt.raster_tile;
        const uint64_t cap = (uint64_t)a.L.s_cap;
        const float *part = reinterpret_cast<const float *>(a.ws + a.L.s_part);
        const int ntile = (x1 / T - x0 / T + 1) * (y1 / T - y0 / T + 1);
        // slots of tiles where the surfel won no pixel hold zero
        for (int kk = 0; kk < ntile; ++kk) {
            if (k0 + kk >= cap) break;
            const float *src = part + (k0 + kk) * 3;
            gc0 += src[0];
            gc1 += src[1];
            gc2 += src[2];
        }
        float dx = V.o[0] - mx, dy = V.o[1] - my, dz = V.o[2] - mz;
        const float idl = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= idl; dy *= idl; dz *= idl;
        sh_basis(dx, dy, dz, K, Y);
    }
    gc0 = on0 ? gc0 : 0.f;
    gc1 = on1 ? gc1 : 0.f;
    gc2 = on2 ? gc2 : 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        g[k][0] = Y[k] * gc0;
        g[k][1] = Y[k] * gc1;
        g[k][2] = Y[k] * gc2;
    }
}

// One surfel's SH gradient summed over the views: its partials are one
// contiguous run per view (slot order).  Zero past the last surfel.
template <int K, bool MV>
__device__ void bwd_surfel_one(const FrameArgs &a, int64_t j, float (&gsh)[K][3]) {
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    if (j >= a.n) return;
    if (!MV) {
        bwd_surfel_one_view<K>(a, j, gsh);
        return;
    }
    const int64_t n = a.n;
    const uint32_t *boff = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff);
    const float *part = reinterpret_cast<const float *>(a.ws + a.L.s_part);
    const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol);
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const int T = a.opt.raster_tile;
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t vj = (int64_t)v * n + j;
        if (!a.ws[a.L.svis + vj]) continue;
        const ViewDev &V = a.views[v];
        int x0, y0, x1, y1;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
        if (x0 > x1) continue;
        // the forward stored max(0, raw) for visible surfels: the clamp is
        // inactive exactly where that colour is positive (no SH re-read)
        bool on[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) on[c] = scol[((int64_t)v * 3 + c) * n + j] > 0.f;
        if (!(on[0] || on[1] || on[2])) continue;
        float gc[3] = {0.f, 0.f, 0.f};
        const uint64_t k0 = boff[vj];
        const int ntile = (x1 / T - x0 / T + 1) * (y1 / T - y0 / T + 1);
        // slots of tiles where the surfel won no pixel hold zero
        for (int kk = 0; kk < ntile; ++kk) {
            if (k0 + kk >= cap) break;
            const float *src = part + (k0 + kk) * 3;
            gc[0] += src[0];
            gc[1] += src[1];
            gc[2] += src[2];
        }
        float dx = V.o[0] - a.S.mean[j], dy = V.o[1] - a.S.mean[n + j], dz = V.o[2] - a.S.mean[2 * n + j];
        const float idl = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= idl; dy *= idl; dz *= idl;
        float Y[K];
        sh_basis(dx, dy, dz, K, Y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (!on[c]) continue;
#pragma unroll
            for (int k = 0; k < K; ++k) gsh[k][c] += Y[k] * gc[c];
        }
    }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_bwd_tiles(FrameArgs a, const float *depth, const float *color_s,
                                                       const float *accum, const float *d_image) {
    // tiles in the splat's launch order (longest list first)
    bwd_gauss_tile<TW, TH>(a, reinterpret_cast<const TileOrd *>(a.ws + a.L.g_ord)[blockIdx.x], depth, color_s,
                           accum, d_image);
}

template <int T>
__global__ void __launch_bounds__(T * T) k_bwd_surfel_tiles(FrameArgs a, const int32_t *sid, const float *accum,
                                                           const float *d_image) {
    bwd_surfel_tile<T>(a, xcd_tile((int)blockIdx.x, (int)gridDim.x), sid, accum, d_image);
}

__global__ void __launch_bounds__(256) k_bwd_compact(FrameArgs a, ges_gradients gr) {
    bwd_compact_one(a, gr, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// One surfel per lane.  The [n][K][3] gradient of a wave's 64 surfels is
// one contiguous run of 64 * 3K floats, almost all zero (a surfel that wins
// no pixel has none).  The few lanes with a gradient (at most kStage) put
// their 3K values in LDS, and the wave then writes the whole run once, with
// unit-stride stores that take each word from LDS or zero.  A wave with more
// such lanes zeroes the run first, waits until those stores are done, and
// then the lanes store their own values over it (the wait orders the two
// sets of stores).
template <int K, bool MV>
__global__ void __launch_bounds__(256) k_bwd_surfels(FrameArgs a, float *gsh_out) {
    constexpr int R = 3 * K, RS = R + 1;  // staged rows padded: distinct LDS banks per lane
    constexpr int kStage = 16;
    __shared__ float stage[4][kStage * RS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t jw = j - lane;  // the wave's first surfel
    if (jw >= a.n) return;        // whole wave past the end (wave-uniform)
    float g[K][3];
    bwd_surfel_one<K, MV>(a, j, g);
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) any |= (g[k][0] != 0.f) | (g[k][1] != 0.f) | (g[k][2] != 0.f);
    const int rows = (int)(a.n - jw < 64 ? a.n - jw : 64);
    float *run = gsh_out + jw * R;
    const unsigned long long am = __ballot((int)any);
    if (__popcll(am) <= kStage) {  // wave-uniform
        if (any) {
            const int slot = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(am >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)am, 0u));
            float *row = &stage[wv][slot * RS];
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) row[k * 3 + c] = g[k][c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (R % 4 == 0 && (reinterpret_cast<uintptr_t>(gsh_out) & 15u) == 0) {
            // 16-byte stores: a run starts on 16 bytes and a row holds whole quads
            for (int f = lane * 4; f < rows * R; f += 256) {
                const int r = f / R, q = f - r * R;
                typedef float f32x4 __attribute__((ext_vector_type(4)));
                f32x4 val = {0.f, 0.f, 0.f, 0.f};
                if ((am >> r) & 1ull) {
                    const float *src = &stage[wv][__popcll(am & ((1ull << r) - 1ull)) * RS + q];
                    val = f32x4{src[0], src[1], src[2], src[3]};
                }
                __builtin_nontemporal_store(val, reinterpret_cast<f32x4 *>(run + f));
            }
            return;
        }
        for (int f = lane; f < rows * R; f += 64) {
            const int r = f / R, q = f - r * R;  // word q of surfel jw + r
            float val = 0.f;
            if ((am >> r) & 1ull) val = stage[wv][__popcll(am & ((1ull << r) - 1ull)) * RS + q];
            put_nt(run + f, val);
        }
        return;
    }
    for (int f = lane; f < rows * R; f += 64) put_nt(run + f, 0.f);
    __builtin_amdgcn_s_waitcnt(0);  // the zero stores are complete before any value store is issued
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (any) {
        float *dst = gsh_out + j * R;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) put_nt(dst + k * 3 + c, g[k][c]);
    }
}

template <int K>
void launch_bwd_surfels_k(const FrameArgs &a, float *out, dim3 grid, dim3 block, hipStream_t s) {
    if (a.n_views > 1) hipLaunchKernelGGL((k_bwd_surfels<K, true>), grid, block, 0, s, a, out);
    else hipLaunchKernelGGL((k_bwd_surfels<K, false>), grid, block, 0, s, a, out);
}

template <int K>
void launch_bwd_gaussians_k(const FrameArgs &a, const ges_gradients &g, bool mv, int cus, hipStream_t s) {
    // as many blocks as are resident at once (the kernel's occupancy, looked
    // up once per instance), and no more than the Gaussians need
    static int per_cu[2] = {0, 0};
    int &pc = per_cu[mv ? 1 : 0];
    if (pc == 0) {
        int nb = 0;
        const hipError_t e = mv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bwd_gaussians<K, true>, 128, 0)
                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bwd_gaussians<K, false>, 128, 0);
        pc = (e == hipSuccess && nb > 0) ? nb : 1;
    }
    const int64_t need = (a.m + 127) / 128, resident = (int64_t)pc * (cus > 0 ? cus : 1);
    const dim3 grid((unsigned)(need < resident ? need : resident)), block(128);
    if (mv) hipLaunchKernelGGL((k_bwd_gaussians<K, true>), grid, block, 0, s, a, g);
    else hipLaunchKernelGGL((k_bwd_gaussians<K, false>), grid, block, 0, s, a, g);
}

}  // namespace

hipError_t launch_bwd_tiles(const FrameArgs &a, const float *depth, const float *color_s, const float *accum,
                            const float *d_image, hipStream_t s) {
    if (a.m == 0) return hipSuccess;
    const dim3 grid((unsigned)a.L.stiles);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_bwd_tiles<8, 8>), grid, dim3(64), 0, s, a, depth, color_s, accum, d_image);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_bwd_tiles<16, 8>), grid, dim3(128), 0, s, a, depth, color_s, accum, d_image);
    else
        hipLaunchKernelGGL((k_bwd_tiles<16, 16>), grid, dim3(256), 0, s, a, depth, color_s, accum, d_image);
    return hipGetLastError();
}

hipError_t launch_bwd_surfel_tiles(const FrameArgs &a, const int32_t *sid, const float *accum,
                                   const float *d_image, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid((unsigned)a.L.rtiles);
    if (a.opt.raster_tile == 8)
        hipLaunchKernelGGL(k_bwd_surfel_tiles<8>, grid, dim3(64), 0, s, a, sid, accum, d_image);
    else
        hipLaunchKernelGGL(k_bwd_surfel_tiles<16>, grid, dim3(256), 0, s, a, sid, accum, d_image);
    return hipGetLastError();
}

hipError_t launch_bwd_compact(const FrameArgs &a, const ges_gradients &g, hipStream_t s) {
    if (a.m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_compact, dim3((unsigned)((a.m + 255) / 256)), dim3(256), 0, s, a, g);
    return hipGetLastError();
}

hipError_t launch_bwd_gaussians(const FrameArgs &a, const ges_gradients &g, int cus, hipStream_t s) {
    if (a.m == 0) return hipSuccess;
    const bool mv = a.n_views > 1;
    switch (a.kg) {
        case 1: launch_bwd_gaussians_k<1>(a, g, mv, cus, s); break;
        case 4: launch_bwd_gaussians_k<4>(a, g, mv, cus, s); break;
        case 9: launch_bwd_gaussians_k<9>(a, g, mv, cus, s); break;
        default: launch_bwd_gaussians_k<16>(a, g, mv, cus, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_bwd_surfels(const FrameArgs &a, const ges_gradients &g, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    switch (a.ks) {
        case 1: launch_bwd_surfels_k<1>(a, g.surfel_sh, grid, block, s); break;
        case 4: launch_bwd_surfels_k<4>(a, g.surfel_sh, grid, block, s); break;
        case 9: launch_bwd_surfels_k<9>(a, g.surfel_sh, grid, block, s); break;
        default: launch_bwd_surfels_k<16>(a, g.surfel_sh, grid, block, s); break;
    }
    return hipGetLastError();
}

}  // namespace ges
