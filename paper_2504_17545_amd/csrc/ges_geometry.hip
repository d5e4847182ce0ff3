// Geometry channels of the frame (2D-GES smoothing, Eq. 10-12): the surfel
// normal map N_s, the Gaussian depth and normal sums D_G, N_G over the
// Gaussians that count at a pixel in pass 2, and the smoothed maps
// D_smooth = (D_s W_s + D_G) / (W_s + W_G), N_smooth likewise.
//
// One block per splat tile, one lane per pixel, over the tile's Gaussian
// list (the pass-2 lists of the frame): every entry is tested with the same
// FP32 alpha and depth-test decisions as pass 2, and d_i alpha and
// n_i alpha are summed in 2^-24 fixed point (64-bit), so the channels do
// not depend on the order of the Gaussian array or of the lists.  d_i is the
// Gaussian's centre depth, n_i its shortest axis in world space turned to
// face the camera (computed once per list entry when the batch is loaded).
// With 2D Gaussians (2D-GES proper) d_i is the planar depth at the pixel
// and n_i the splat's normal (k_geometry2d).
#include "ges_internal.h"

namespace ges {

namespace {

// Shortest axis of a Gaussian (the rotation's column of the smallest scale,
// the first on a tie), world space, facing the camera at o.
__device__ inline void shortest_axis(const FrameArgs &a, const ViewDev &V, uint32_t i, float n[3]) {
    const int64_t m = a.m;
    float qw = a.G.quat[i], qx = a.G.quat[m + i], qy = a.G.quat[2 * m + i], qz = a.G.quat[3 * m + i];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    const float s0 = a.G.scale[i], s1 = a.G.scale[m + i], s2 = a.G.scale[2 * m + i];
    const int k = (s1 < s0 && s1 <= s2) ? 1 : ((s2 < s0 && s2 < s1) ? 2 : 0);
    n[0] = Rq[k];
    n[1] = Rq[3 + k];
    n[2] = Rq[6 + k];
    const float tx = V.o[0] - a.G.mean[i], ty = V.o[1] - a.G.mean[m + i], tz = V.o[2] - a.G.mean[2 * m + i];
    if (n[0] * tx + n[1] * ty + n[2] * tz < 0.f) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    }
}

// The frontmost surfel's normal, world space, facing the camera (0 where
// no surfel covers the pixel).
__device__ inline void surfel_normal(const FrameArgs &a, const ViewDev &V, int id, float ns[3]) {
    ns[0] = ns[1] = ns[2] = 0.f;
    if (id < 0 || (int64_t)id >= a.n) return;
    const int64_t n = a.n;
    float qw = a.S.quat[id], qx = a.S.quat[n + id], qy = a.S.quat[2 * n + id], qz = a.S.quat[3 * n + id];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    ns[0] = Rq[2];
    ns[1] = Rq[5];
    ns[2] = Rq[8];
    const float tx = V.o[0] - a.S.mean[id], ty = V.o[1] - a.S.mean[n + id], tz = V.o[2] - a.S.mean[2 * n + id];
    if (ns[0] * tx + ns[1] * ty + ns[2] * tz < 0.f) {
        ns[0] = -ns[0];
        ns[1] = -ns[1];
        ns[2] = -ns[2];
    }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_geometry(FrameArgs a, const int32_t *sid, const float *depth,
                                                      const float *accum, ges_geometry_out out) {
    constexpr int NT = TW * TH;
    __shared__ GRec lds[NT];
    __shared__ float lnrm[NT][3];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int px = (lt % V.stx) * TW + (int)(threadIdx.x % TW);
    const int py = (lt / V.stx) * TH + (int)(threadIdx.x / TW);
    const bool inside = px < V.W && py < V.H;
    const int64_t lp = (int64_t)py * V.W + px;
    const int64_t P = (int64_t)V.W * V.H;
    const float ds = inside ? depth[V.pix_off + lp] : -__int_as_float(0x7f800000);
    const int id = inside ? sid[V.pix_off + lp] : -1;
    const float xf = (float)px + 0.5f, yf = (float)py + 0.5f;
    const float amin = a.opt.alpha_min;

    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_toff);
    const GEnt *ents = reinterpret_cast<const GEnt *>(a.ws + a.L.g_ents);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)toff[t], cap), b1 = umin64((uint64_t)toff[t + 1], cap);
    long long acc_d = 0, acc_x = 0, acc_y = 0, acc_z = 0;
    for (uint64_t base = b0; base < b1; base += NT) {
        const int cnt = (int)umin64((uint64_t)NT, b1 - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const GEnt &e = ents[base + threadIdx.x];
            lds[threadIdx.x] = e.g;
            float n[3] = {0.f, 0.f, 0.f};
            if ((int64_t)e.gauss < a.m) shortest_axis(a, V, e.gauss, n);
            lnrm[threadIdx.x][0] = n[0];
            lnrm[threadIdx.x][1] = n[1];
            lnrm[threadIdx.x][2] = n[2];
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const GRec g = lds[k];
            float dx, dy, q;
            const float al = gauss_alpha(g, xf, yf, dx, dy, q);
            if ((al >= amin) & (g.dme < ds)) {  // pass 2's decisions, bit for bit
                acc_d += __float2ll_rn(al * g.depth * kFixScale);
                acc_x += (long long)__float2int_rn(al * lnrm[k][0] * kFixScale);
                acc_y += (long long)__float2int_rn(al * lnrm[k][1] * kFixScale);
                acc_z += (long long)__float2int_rn(al * lnrm[k][2] * kFixScale);
            }
        }
    }
    if (!inside) return;
    float ns[3];
    surfel_normal(a, V, id, ns);
    const float dg = (float)((double)acc_d * kFixInv);
    const float ng[3] = {(float)((double)acc_x * kFixInv), (float)((double)acc_y * kFixInv),
                         (float)((double)acc_z * kFixInv)};
    const float ws = a.opt.w_s;
    const float inv = 1.f / (ws + accum[4 * V.pix_off + 3 * P + lp]);
    const float dsw = id >= 0 ? ds * ws : 0.f;  // no surfel: D_s W_s counts as 0
    if (out.normal_s)
        for (int c = 0; c < 3; ++c) out.normal_s[3 * V.pix_off + c * P + lp] = ns[c];
    if (out.depth_g) out.depth_g[V.pix_off + lp] = dg;
    if (out.normal_g)
        for (int c = 0; c < 3; ++c) out.normal_g[3 * V.pix_off + c * P + lp] = ng[c];
    if (out.depth_smooth) out.depth_smooth[V.pix_off + lp] = (dsw + dg) * inv;
    if (out.normal_smooth)
        for (int c = 0; c < 3; ++c) out.normal_smooth[3 * V.pix_off + c * P + lp] = (ns[c] * ws + ng[c]) * inv;
}

// 2D-GES with 2D Gaussians (Sec. 6.4): d_i is the planar depth at the
// pixel and n_i the splat's normal, both from the list entry; each entry
// is tested by g2_eval, as in pass 2.  The record's normal n is turned away
// from the camera (n . mu >= 0), so the world normal facing it is -R^T n.
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_geometry2d(FrameArgs a, const int32_t *sid, const float *depth,
                                                        const float *accum, ges_geometry_out out) {
    constexpr int NT = TW * TH;
    __shared__ G2Ent lds[NT];
    __shared__ float lnrm[NT][3];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int px = (lt % V.stx) * TW + (int)(threadIdx.x % TW);
    const int py = (lt / V.stx) * TH + (int)(threadIdx.x / TW);
    const bool inside = px < V.W && py < V.H;
    const int64_t lp = (int64_t)py * V.W + px;
    const int64_t P = (int64_t)V.W * V.H;
    const float ds = inside ? depth[V.pix_off + lp] : -__int_as_float(0x7f800000);
    const int id = inside ? sid[V.pix_off + lp] : -1;
    const float xr = ((float)px + 0.5f - V.cx) / V.fx, yr = ((float)py + 0.5f - V.cy) / V.fy;
    const float amin = a.opt.alpha_min, zn = V.znear;

    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_toff);
    const G2Ent *ents = reinterpret_cast<const G2Ent *>(a.ws + a.L.g_ents);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)toff[t], cap), b1 = umin64((uint64_t)toff[t + 1], cap);
    long long acc_d = 0, acc_x = 0, acc_y = 0, acc_z = 0;
    for (uint64_t base = b0; base < b1; base += NT) {
        const int cnt = (int)umin64((uint64_t)NT, b1 - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const G2Ent &e = ents[base + threadIdx.x];
            lds[threadIdx.x] = e;
            const float *R = V.R;
            lnrm[threadIdx.x][0] = -(R[0] * e.nx + R[3] * e.ny + R[6] * e.nz);
            lnrm[threadIdx.x][1] = -(R[1] * e.nx + R[4] * e.ny + R[7] * e.nz);
            lnrm[threadIdx.x][2] = -(R[2] * e.nx + R[5] * e.ny + R[8] * e.nz);
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            float al, z;
            if (g2_eval(lds[k], xr, yr, zn, amin, ds, al, z)) {  // pass 2's decisions, bit for bit
                acc_d += __float2ll_rn(al * z * kFixScale);
                acc_x += (long long)__float2int_rn(al * lnrm[k][0] * kFixScale);
                acc_y += (long long)__float2int_rn(al * lnrm[k][1] * kFixScale);
                acc_z += (long long)__float2int_rn(al * lnrm[k][2] * kFixScale);
            }
        }
    }
    if (!inside) return;
    float ns[3];
    surfel_normal(a, V, id, ns);
    const float dg = (float)((double)acc_d * kFixInv);
    const float ng[3] = {(float)((double)acc_x * kFixInv), (float)((double)acc_y * kFixInv),
                         (float)((double)acc_z * kFixInv)};
    const float ws = a.opt.w_s;
    const float inv = 1.f / (ws + accum[4 * V.pix_off + 3 * P + lp]);
    const float dsw = id >= 0 ? ds * ws : 0.f;
    if (out.normal_s)
        for (int c = 0; c < 3; ++c) out.normal_s[3 * V.pix_off + c * P + lp] = ns[c];
    if (out.depth_g) out.depth_g[V.pix_off + lp] = dg;
    if (out.normal_g)
        for (int c = 0; c < 3; ++c) out.normal_g[3 * V.pix_off + c * P + lp] = ng[c];
    if (out.depth_smooth) out.depth_smooth[V.pix_off + lp] = (dsw + dg) * inv;
    if (out.normal_smooth)
        for (int c = 0; c < 3; ++c) out.normal_smooth[3 * V.pix_off + c * P + lp] = (ns[c] * ws + ng[c]) * inv;
}

}  // namespace

hipError_t launch_geometry(const FrameArgs &a, const int32_t *sid, const float *depth, const float *accum,
                           const ges_geometry_out &out, hipStream_t s) {
    const dim3 grid((unsigned)a.L.stiles);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (a.G.dims == 2) {
        if (tw == 8 && th == 8)
            hipLaunchKernelGGL((k_geometry2d<8, 8>), grid, dim3(64), 0, s, a, sid, depth, accum, out);
        else if (tw == 16 && th == 8)
            hipLaunchKernelGGL((k_geometry2d<16, 8>), grid, dim3(128), 0, s, a, sid, depth, accum, out);
        else
            hipLaunchKernelGGL((k_geometry2d<16, 16>), grid, dim3(256), 0, s, a, sid, depth, accum, out);
        return hipGetLastError();
    }
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_geometry<8, 8>), grid, dim3(64), 0, s, a, sid, depth, accum, out);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_geometry<16, 8>), grid, dim3(128), 0, s, a, sid, depth, accum, out);
    else
        hipLaunchKernelGGL((k_geometry<16, 16>), grid, dim3(256), 0, s, a, sid, depth, accum, out);
    return hipGetLastError();
}

}  // namespace ges
