// Backward kernels: gradient of a loss L given dL/dC for the parameters the
// joint optimisation stage trains (Sec. 4.2): Gaussian p, r, s, sigma, SH
// and surfel SH.  No float atomics: every sum runs in a fixed order, so the
// result is bitwise reproducible and independent of the Gaussian order.
//
//   tiles     per splat tile.  Per pixel, from Eq. 5 with S = W_s + W_G:
//             dL/dC_s = W_s g / S, dL/dC_G = g / S, dL/dW_G = -sum_c g_c C_c / S.
//             (a) each lane takes one entry of the tile's Gaussian list and
//             walks that Gaussian's pixels inside the tile in row order,
//             recomputing alpha exactly as the forward did and summing
//             dL/d(sigma, p_hat, conic, colour) -> one partial per entry;
//             (b) the tile's pixels are grouped by surfel id; each group's
//             dL/dC_s is summed in pixel order -> (id, sum) entries.
//   gaussians per Gaussian: partials summed over views and tiles in a fixed
//             order (the back-map written by the list fill), then chained
//             through the conic inverse, the EWA projection (Jacobian with
//             its clamp), the projected centre, Sigma3 = R S S R^T, the
//             quaternion normalisation and the SH colour (incl. its
//             dependence on the view direction).
//   surfels   per surfel: tile entries gathered over views and tiles in a
//             fixed order, times the SH basis (zero where the colour clamp
//             is active).
#include "ges_internal.h"

namespace ges {

namespace {

constexpr int kPartials = 9;  // sigma, p_hat x/y, conic a/b/c, colour r/g/b

struct SurfEntry {
    int id;
    float r, g, b;
};

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_bwd_tiles(FrameArgs a, const int32_t *sid, const float *depth,
                                                       const float *color_s, const float *accum,
                                                       const float *d_image) {
    constexpr int NT = TW * TH;
    __shared__ float s_g[NT][3];
    __shared__ float s_gw[NT];
    __shared__ float s_ds[NT];
    __shared__ int s_id[NT];
    __shared__ int s_nent;
    const int t = blockIdx.x;
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int tx0 = (lt % V.stx) * TW, ty0 = (lt / V.stx) * TH;
    const int px = tx0 + (int)(threadIdx.x % TW);
    const int py = ty0 + (int)(threadIdx.x / TW);
    const int64_t P = (int64_t)V.W * V.H;
    const float ws = a.opt.w_s;

    // per-pixel adjoint state
    {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, gw = 0.f, ds = -__int_as_float(0x7f800000);
        int id = -1;
        if (px < V.W && py < V.H) {
            const int64_t lp = (int64_t)py * V.W + px;
            const float *cs = color_s + 3 * V.pix_off + lp;
            const float *ac = accum + 4 * V.pix_off + lp;
            const float *dg = d_image + 3 * V.pix_off + lp;
            const float wg = ac[3 * P];
            const float inv = 1.f / (ws + wg);
            const float c0 = (ws * cs[0] + ac[0]) * inv;
            const float c1 = (ws * cs[P] + ac[P]) * inv;
            const float c2 = (ws * cs[2 * P] + ac[2 * P]) * inv;
            g0 = dg[0] * inv;
            g1 = dg[P] * inv;
            g2 = dg[2 * P] * inv;
            gw = -(g0 * c0 + g1 * c1 + g2 * c2);
            ds = depth[V.pix_off + lp];
            id = sid[V.pix_off + lp];
        }
        s_g[threadIdx.x][0] = g0;
        s_g[threadIdx.x][1] = g1;
        s_g[threadIdx.x][2] = g2;
        s_gw[threadIdx.x] = gw;
        s_ds[threadIdx.x] = ds;
        s_id[threadIdx.x] = id;
        if (threadIdx.x == 0) s_nent = 0;
    }
    __syncthreads();

    // (b) surfel colour gradient, grouped by id in pixel order
    {
        const int me = threadIdx.x;
        const int id = s_id[me];
        bool leader = id >= 0;
        for (int k = 0; k < me && leader; ++k) leader = s_id[k] != id;
        if (leader) {
            float r = 0.f, g = 0.f, b = 0.f;
            for (int k = me; k < NT; ++k)
                if (s_id[k] == id) {
                    r += s_g[k][0];
                    g += s_g[k][1];
                    b += s_g[k][2];
                }
            const int slot = atomicAdd(&s_nent, 1);
            SurfEntry e;
            e.id = id;
            e.r = ws * r;
            e.g = ws * g;
            e.b = ws * b;
            reinterpret_cast<SurfEntry *>(a.ws + a.L.stile_ent)[(int64_t)t * NT + slot] = e;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) reinterpret_cast<int *>(a.ws + a.L.stile_n)[t] = s_nent;

    // (a) Gaussian partials, one list entry per lane
    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_toff);
    const uint32_t *list = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_list);
    const GRec *grec = reinterpret_cast<const GRec *>(a.ws + a.L.grec) + (int64_t)v * a.m;
    const uint2 *gbox = reinterpret_cast<const uint2 *>(a.ws + a.L.gbox) + (int64_t)v * a.m;
    float *part = reinterpret_cast<float *>(a.ws + a.L.partial);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)toff[t], cap), b1 = umin64((uint64_t)toff[t + 1], cap);
    const float amin = a.opt.alpha_min;
    for (uint64_t pos = b0 + threadIdx.x; pos < b1; pos += NT) {
        const uint32_t gi = list[pos];
        const GRec g = grec[gi];
        int x0, y0, x1, y1;
        unpack_box(gbox[gi], x0, y0, x1, y1);
        x0 = max(x0, tx0); y0 = max(y0, ty0);
        x1 = min(x1, tx0 + TW - 1); y1 = min(y1, ty0 + TH - 1);
        const float cr = g.r * (float)kFixInv, cg = g.g * (float)kFixInv, cb = g.b * (float)kFixInv;
        const float isig = 1.f / g.sigma;
        float acc[kPartials];
        for (int k = 0; k < kPartials; ++k) acc[k] = 0.f;
        for (int yy = y0; yy <= y1; ++yy)
            for (int xx = x0; xx <= x1; ++xx) {
                const int lp = (yy - ty0) * TW + (xx - tx0);
                float dx, dy, q;
                const float al = gauss_alpha(g, (float)xx + 0.5f, (float)yy + 0.5f, dx, dy, q);
                if (!(al >= amin && g.dme < s_ds[lp])) continue;
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
        for (int k = 0; k < kPartials; ++k) part[(uint64_t)k * cap + pos] = acc[k];
    }
}

__device__ inline void mat3_mul(const float *A, const float *B, float *C) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

__global__ void __launch_bounds__(128) k_bwd_gaussians(FrameArgs a, ges_gradients gr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    const int64_t m = a.m;
    const float px = a.G.mean[i], py = a.G.mean[m + i], pz = a.G.mean[2 * m + i];
    const float q0 = a.G.quat[i], q1 = a.G.quat[m + i], q2 = a.G.quat[2 * m + i], q3 = a.G.quat[3 * m + i];
    const float s[3] = {a.G.scale[i], a.G.scale[m + i], a.G.scale[2 * m + i]};
    const float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const float qw = q0 / qn, qx = q1 / qn, qy = q2 / qn, qz = q3 / qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    float Mm[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Mm[3 * r + c] = Rq[3 * r + c] * s[c];
    float S3[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S3[3 * r + c] = Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2];

    float gp[3] = {0.f, 0.f, 0.f};    // dL/dp (world)
    float gS3[9];                      // dL/dSigma3, summed over views
    for (int k = 0; k < 9; ++k) gS3[k] = 0.f;
    float gsig = 0.f;
    float gsh[16][3];
    for (int k = 0; k < 16; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;

    const uint32_t *gcnt = reinterpret_cast<const uint32_t *>(a.ws + a.L.gcnt);
    const uint32_t *gboff = reinterpret_cast<const uint32_t *>(a.ws + a.L.gboff);
    const uint32_t *back = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_back);
    const float *part = reinterpret_cast<const float *>(a.ws + a.L.partial);
    const uint64_t cap = (uint64_t)a.L.g_cap;

    for (int v = 0; v < a.n_views; ++v) {
        const int64_t vi = (int64_t)v * m + i;
        const uint32_t cnt = gcnt[vi];
        if (cnt == 0) continue;
        float P[kPartials];
        for (int k = 0; k < kPartials; ++k) P[k] = 0.f;
        const uint64_t base = gboff[vi];
        for (uint32_t k = 0; k < cnt; ++k) {
            if (base + k >= cap) break;
            const uint64_t pos = back[base + k];
            if (pos >= cap) continue;  // entry lost to an overflow
            for (int c = 0; c < kPartials; ++c) P[c] += part[(uint64_t)c * cap + pos];
        }
        const ViewDev &V = a.views[v];
        const float *Rc = V.R;
        const float mx = Rc[0] * px + Rc[1] * py + Rc[2] * pz + V.t[0];
        const float my = Rc[3] * px + Rc[4] * py + Rc[5] * pz + V.t[1];
        const float mz = Rc[6] * px + Rc[7] * py + Rc[8] * pz + V.t[2];
        const float iz = 1.f / mz;
        const float rx = mx * iz, ry = my * iz;
        const float ux = fminf(fmaxf(rx, -V.limx), V.limx);
        const float uy = fminf(fmaxf(ry, -V.limy), V.limy);
        const float J00 = V.fx * iz, J02 = -V.fx * ux * iz;
        const float J11 = V.fy * iz, J12 = -V.fy * uy * iz;
        float T[6];
        for (int c = 0; c < 3; ++c) {
            T[c] = J00 * Rc[c] + J02 * Rc[6 + c];
            T[3 + c] = J11 * Rc[3 + c] + J12 * Rc[6 + c];
        }
        float TS[6];  // T Sigma3
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c)
                TS[3 * r + c] = T[3 * r] * S3[c] + T[3 * r + 1] * S3[3 + c] + T[3 * r + 2] * S3[6 + c];
        const float cxx = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + a.opt.dilation;
        const float cxy = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
        const float cyy = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + a.opt.dilation;
        const float idet = 1.f / (cxx * cyy - cxy * cxy);
        const float A00 = cyy * idet, A01 = -cxy * idet, A11 = cxx * idet;
        // dL/dSigma2 = -A G_A A with G_A = [[ga, gb/2], [gb/2, gc]]
        const float ga = P[3], gb = 0.5f * P[4], gc = P[5];
        const float B00 = ga * A00 + gb * A01, B01 = ga * A01 + gb * A11;
        const float B10 = gb * A00 + gc * A01, B11 = gb * A01 + gc * A11;
        const float G00 = -(A00 * B00 + A01 * B10);
        const float G01 = -(A00 * B01 + A01 * B11);
        const float G11 = -(A01 * B01 + A11 * B11);
        const float G2[4] = {G00, G01, G01, G11};
        // dL/dSigma3 += T^T G2 T
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                gS3[3 * r + c] += T[r] * (G2[0] * T[c] + G2[1] * T[3 + c]) + T[3 + r] * (G2[2] * T[c] + G2[3] * T[3 + c]);
        // dL/dT = 2 G2 T Sigma3 = 2 G2 TS
        float gT[6];
        for (int c = 0; c < 3; ++c) {
            gT[c] = 2.f * (G2[0] * TS[c] + G2[1] * TS[3 + c]);
            gT[3 + c] = 2.f * (G2[2] * TS[c] + G2[3] * TS[3 + c]);
        }
        // dL/dJ = dL/dT R^T (only J00, J02, J11, J12 vary)
        const float gJ00 = gT[0] * Rc[0] + gT[1] * Rc[1] + gT[2] * Rc[2];
        const float gJ02 = gT[0] * Rc[6] + gT[1] * Rc[7] + gT[2] * Rc[8];
        const float gJ11 = gT[3] * Rc[3] + gT[4] * Rc[4] + gT[5] * Rc[5];
        const float gJ12 = gT[3] * Rc[6] + gT[4] * Rc[7] + gT[5] * Rc[8];
        float gmx = 0.f, gmy = 0.f, gmz = 0.f;
        const float iz2 = iz * iz;
        gmz += -V.fx * iz2 * gJ00 - V.fy * iz2 * gJ11 + V.fx * ux * iz2 * gJ02 + V.fy * uy * iz2 * gJ12;
        if (rx > -V.limx && rx < V.limx) {
            const float gux = gJ02 * (-V.fx * iz);
            gmx += gux * iz;
            gmz += -gux * mx * iz2;
        }
        if (ry > -V.limy && ry < V.limy) {
            const float guy = gJ12 * (-V.fy * iz);
            gmy += guy * iz;
            gmz += -guy * my * iz2;
        }
        // projected centre
        gmx += P[1] * V.fx * iz;
        gmy += P[2] * V.fy * iz;
        gmz += -(P[1] * V.fx * mx + P[2] * V.fy * my) * iz2;
        // mu = R p + t
        gp[0] += Rc[0] * gmx + Rc[3] * gmy + Rc[6] * gmz;
        gp[1] += Rc[1] * gmx + Rc[4] * gmy + Rc[7] * gmz;
        gp[2] += Rc[2] * gmx + Rc[5] * gmy + Rc[8] * gmz;
        gsig += P[0];
        // colour: c = max(0, 1/2 + sum SH Y(d)), d = (o - p)/|o - p|
        float dx = V.o[0] - px, dy = V.o[1] - py, dz = V.o[2] - pz;
        const float dl = sqrtf(dx * dx + dy * dy + dz * dz);
        const float idl = 1.f / dl;
        dx *= idl; dy *= idl; dz *= idl;
        float Y[16];
        sh_basis(dx, dy, dz, a.kg, Y);
        float dY[16][3];
        sh_basis_grad(dx, dy, dz, a.kg, dY);
        float gd[3] = {0.f, 0.f, 0.f};
        for (int ch = 0; ch < 3; ++ch) {
            float raw = 0.5f;
            for (int k = 0; k < a.kg; ++k) raw += a.G.sh[((int64_t)k * 3 + ch) * m + i] * Y[k];
            if (!(raw > 0.f)) continue;
            const float gcol = P[6 + ch];
            for (int k = 0; k < a.kg; ++k) {
                const float shk = a.G.sh[((int64_t)k * 3 + ch) * m + i];
                gsh[k][ch] += Y[k] * gcol;
                gd[0] += gcol * shk * dY[k][0];
                gd[1] += gcol * shk * dY[k][1];
                gd[2] += gcol * shk * dY[k][2];
            }
        }
        const float dot = gd[0] * dx + gd[1] * dy + gd[2] * dz;
        gp[0] -= (gd[0] - dot * dx) * idl;
        gp[1] -= (gd[1] - dot * dy) * idl;
        gp[2] -= (gd[2] - dot * dz) * idl;
    }

    // Sigma3 = M M^T, M = Rq diag(s): dL/dM = 2 gS3 M (gS3 symmetric)
    float gM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            gM[3 * r + c] = (gS3[3 * r] + gS3[r]) * Mm[c] + (gS3[3 * r + 1] + gS3[3 + r]) * Mm[3 + c] +
                            (gS3[3 * r + 2] + gS3[6 + r]) * Mm[6 + c];
    float gs[3], gR[9];
    for (int c = 0; c < 3; ++c) gs[c] = gM[c] * Rq[c] + gM[3 + c] * Rq[3 + c] + gM[6 + c] * Rq[6 + c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) gR[3 * r + c] = gM[3 * r + c] * s[c];
    // rotation matrix of the normalised quaternion -> its components
    const float gqw = 2.f * (-qz * gR[1] + qy * gR[2] + qz * gR[3] - qx * gR[5] - qy * gR[6] + qx * gR[7]);
    const float gqx = 2.f * (qy * gR[1] + qz * gR[2] + qy * gR[3] - 2.f * qx * gR[4] - qw * gR[5] + qz * gR[6] +
                             qw * gR[7] - 2.f * qx * gR[8]);
    const float gqy = 2.f * (-2.f * qy * gR[0] + qx * gR[1] + qw * gR[2] + qx * gR[3] + qz * gR[5] - qw * gR[6] +
                             qz * gR[7] - 2.f * qy * gR[8]);
    const float gqz = 2.f * (-2.f * qz * gR[0] - qw * gR[1] + qx * gR[2] + qw * gR[3] - 2.f * qz * gR[4] +
                             qy * gR[5] + qx * gR[6] + qy * gR[7]);
    // normalisation q_bar = q / |q|
    const float dq = gqw * qw + gqx * qx + gqy * qy + gqz * qz;
    const float iqn = 1.f / qn;
    gr.quat[i] = (gqw - dq * qw) * iqn;
    gr.quat[m + i] = (gqx - dq * qx) * iqn;
    gr.quat[2 * m + i] = (gqy - dq * qy) * iqn;
    gr.quat[3 * m + i] = (gqz - dq * qz) * iqn;
    gr.mean[i] = gp[0];
    gr.mean[m + i] = gp[1];
    gr.mean[2 * m + i] = gp[2];
    gr.scale[i] = gs[0];
    gr.scale[m + i] = gs[1];
    gr.scale[2 * m + i] = gs[2];
    gr.opacity[i] = gsig;
    for (int k = 0; k < a.kg; ++k)
        for (int ch = 0; ch < 3; ++ch) gr.sh[((int64_t)k * 3 + ch) * m + i] = gsh[k][ch];
}

__global__ void __launch_bounds__(256) k_bwd_surfels(FrameArgs a, float *gsh_out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const int64_t n = a.n;
    float gsh[16][3];
    for (int k = 0; k < 16; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    const int TW = a.opt.splat_tile_w, TH = a.opt.splat_tile_h, NT = TW * TH;
    const int *tn = reinterpret_cast<const int *>(a.ws + a.L.stile_n);
    const SurfEntry *ent = reinterpret_cast<const SurfEntry *>(a.ws + a.L.stile_ent);
    for (int v = 0; v < a.n_views; ++v) {
        const int64_t vj = (int64_t)v * n + j;
        if (!a.ws[a.L.svis + vj]) continue;
        const ViewDev &V = a.views[v];
        int x0, y0, x1, y1;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
        if (x0 > x1) continue;
        float gc[3] = {0.f, 0.f, 0.f};
        for (int ty = y0 / TH; ty <= y1 / TH; ++ty)
            for (int tx = x0 / TW; tx <= x1 / TW; ++tx) {
                const int t = V.st_off + ty * V.stx + tx;
                const int ne = tn[t];
                for (int e = 0; e < ne; ++e) {
                    const SurfEntry se = ent[(int64_t)t * NT + e];
                    if (se.id == (int)j) {
                        gc[0] += se.r;
                        gc[1] += se.g;
                        gc[2] += se.b;
                        break;
                    }
                }
            }
        float dx = V.o[0] - a.S.mean[j], dy = V.o[1] - a.S.mean[n + j], dz = V.o[2] - a.S.mean[2 * n + j];
        const float idl = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
        dx *= idl; dy *= idl; dz *= idl;
        float Y[16];
        sh_basis(dx, dy, dz, a.ks, Y);
        for (int ch = 0; ch < 3; ++ch) {
            float raw = 0.5f;
            for (int k = 0; k < a.ks; ++k) raw += a.S.sh[((int64_t)k * 3 + ch) * n + j] * Y[k];
            if (!(raw > 0.f)) continue;
            for (int k = 0; k < a.ks; ++k) gsh[k][ch] += Y[k] * gc[ch];
        }
    }
    for (int k = 0; k < a.ks; ++k)
        for (int ch = 0; ch < 3; ++ch) gsh_out[((int64_t)k * 3 + ch) * n + j] = gsh[k][ch];
}

}  // namespace

hipError_t launch_bwd_tiles(const FrameArgs &a, const int32_t *sid, const float *depth, const float *color_s,
                            const float *accum, const float *d_image, hipStream_t s) {
    const dim3 grid((unsigned)a.L.stiles);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_bwd_tiles<8, 8>), grid, dim3(64), 0, s, a, sid, depth, color_s, accum, d_image);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_bwd_tiles<16, 8>), grid, dim3(128), 0, s, a, sid, depth, color_s, accum, d_image);
    else
        hipLaunchKernelGGL((k_bwd_tiles<16, 16>), grid, dim3(256), 0, s, a, sid, depth, color_s, accum, d_image);
    return hipGetLastError();
}

hipError_t launch_bwd_gaussians(const FrameArgs &a, const ges_gradients &g, hipStream_t s) {
    if (a.m > 0)
        hipLaunchKernelGGL(k_bwd_gaussians, dim3((unsigned)((a.m + 127) / 128)), dim3(128), 0, s, a, g);
    return hipGetLastError();
}

hipError_t launch_bwd_surfels(const FrameArgs &a, const ges_gradients &g, hipStream_t s) {
    if (a.n > 0)
        hipLaunchKernelGGL(k_bwd_surfels, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, g.surfel_sh);
    return hipGetLastError();
}

}  // namespace ges
