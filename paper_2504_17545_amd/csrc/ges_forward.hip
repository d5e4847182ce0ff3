// Forward kernels of the two-pass, sorting-free GES render (gfx950).
//
//   project   per (view, primitive): Gaussian projection (Eq. 4 and the text
//             after it, eps of Sec. 5, colour of Eq. 1) and surfel disc
//             set-up (Sec. 3) with exact screen bounds; counts the raster
//             tiles each surfel touches.
//   surfel fill   per (view, surfel): writes surfel ids into per-tile lists
//             (counting-sort scatter, no sort inside a tile).
//   raster    per raster tile: each lane owns a pixel and keeps the minimum
//             (depth, id) over the tile's list staged through LDS: the
//             z-buffer of pass 1 without atomics.
//   shade / resolve  colour of visible surfels only (SoA SH reads), C_s per
//             pixel, per splat tile the largest D_s (a conservative Hi-Z).
//   gauss count / fill   per (view, Gaussian): per-tile lists of Gaussians
//             whose depth test can pass somewhere in the tile.
//   splat     per splat tile: lane-owns-pixel accumulation of C_G, W_G
//             (Eq. 2-3) in 2^-24 fixed point (int64), then Eq. 5.
#include <math.h>

#include "ges_internal.h"

namespace ges {

namespace {

__device__ inline void set_flag(WsHeader *h, uint32_t f) { atomicOr(&h->flags, f); }

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Inclusive pixel range whose centres (i + 0.5) fall in [lo, hi] (pixels),
// padded, clamped to [0, n-1]; returns false if empty.
__device__ inline bool pixel_range(double lo, double hi, int n, int &i0, int &i1) {
    if (!(lo <= hi)) return false;  // also rejects NaN
    lo = fmax(lo, -4.0);
    hi = fmin(hi, (double)n + 4.0);
    i0 = (int)ceil(lo - 0.5);
    i1 = (int)floor(hi - 0.5);
    i0 = clampi(i0, 0, n - 1);
    i1 = clampi(i1, 0, n - 1);
    if (hi < 0.5 || lo > (double)n - 0.5) return false;
    return i0 <= i1;
}

// ---------------------------------------------------------------------------
// Gaussians: projection

// The colour is not evaluated here: the count pass does it for the
// Gaussians that keep a list entry, so only their SH coefficients are read.
__device__ void project_gaussian(const FrameArgs &a, int v, int64_t i) {
    if (i >= a.m) return;
    const ViewDev &V = a.views[v];
    const int64_t m = a.m;
    const int64_t vi = (int64_t)v * m + i;
    GRec *rec = reinterpret_cast<GRec *>(a.ws + a.L.grec) + vi;
    uint2 *box = reinterpret_cast<uint2 *>(a.ws + a.L.gbox) + vi;
    uint32_t *nt = reinterpret_cast<uint32_t *>(a.ws + a.L.g_boff) + vi;
    *nt = 0;

    const float px = a.G.mean[i], py = a.G.mean[m + i], pz = a.G.mean[2 * m + i];
    float qw = a.G.quat[i], qx = a.G.quat[m + i], qy = a.G.quat[2 * m + i], qz = a.G.quat[3 * m + i];
    const float s0 = a.G.scale[i], s1 = a.G.scale[m + i], s2 = a.G.scale[2 * m + i];
    const float sigma = a.G.opacity[i];
    const float *Rc = V.R;
    const float mx = Rc[0] * px + Rc[1] * py + Rc[2] * pz + V.t[0];
    const float my = Rc[3] * px + Rc[4] * py + Rc[5] * pz + V.t[1];
    const float mz = Rc[6] * px + Rc[7] * py + Rc[8] * pz + V.t[2];

    *box = make_uint2(kEmptyBoxX, 0u);
    bool valid = (mz > V.znear) && (sigma >= a.opt.alpha_min) && isfinite(mx) && isfinite(my);
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    valid = valid && (qn > 0.f) && isfinite(qn);
    if (!valid) return;
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    // world covariance Sigma3 = (Rq S)(Rq S)^T
    float Mm[9];
    for (int r = 0; r < 3; ++r) {
        Mm[3 * r + 0] = Rq[3 * r + 0] * s0;
        Mm[3 * r + 1] = Rq[3 * r + 1] * s1;
        Mm[3 * r + 2] = Rq[3 * r + 2] * s2;
    }
    float S3[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S3[3 * r + c] = Mm[3 * r] * Mm[3 * c] + Mm[3 * r + 1] * Mm[3 * c + 1] + Mm[3 * r + 2] * Mm[3 * c + 2];
    // Mip-GES world-space filter: Sigma3 + v I, opacity times
    // sqrt(det Sigma3 / det(Sigma3 + v I)) = prod s / sqrt(s^2 + v)
    float sig_eff = sigma;
    if (a.G.filter3d) {
        const float v3 = a.G.filter3d[i];
        S3[0] += v3;
        S3[4] += v3;
        S3[8] += v3;
        sig_eff *= (s0 * rsqrtf(s0 * s0 + v3)) * (s1 * rsqrtf(s1 * s1 + v3)) * (s2 * rsqrtf(s2 * s2 + v3));
    }
    // Jacobian of the perspective map with 3DGS's clamp of x/z, y/z
    const float iz = 1.f / mz;
    const float ux = fminf(fmaxf(mx * iz, -V.limx), V.limx);
    const float uy = fminf(fmaxf(my * iz, -V.limy), V.limy);
    const float J00 = V.fx * iz, J02 = -V.fx * ux * iz;
    const float J11 = V.fy * iz, J12 = -V.fy * uy * iz;
    // T = J R (2x3)
    float T0[3], T1[3];
    for (int c = 0; c < 3; ++c) {
        T0[c] = J00 * Rc[c] + J02 * Rc[6 + c];
        T1[c] = J11 * Rc[3 + c] + J12 * Rc[6 + c];
    }
    float A0[3], A1[3];  // T Sigma3
    for (int c = 0; c < 3; ++c) {
        A0[c] = T0[0] * S3[c] + T0[1] * S3[3 + c] + T0[2] * S3[6 + c];
        A1[c] = T1[0] * S3[c] + T1[1] * S3[3 + c] + T1[2] * S3[6 + c];
    }
    // screen-space term: the 0.3 dilation, or the Mip-GES filter of variance
    // mip_2d with the opacity times sqrt(det Sigma2 / det(Sigma2 + mip_2d I))
    const bool mip = a.opt.mip_2d > 0.f;
    const float dil = mip ? a.opt.mip_2d : a.opt.dilation;
    const float bxx = A0[0] * T0[0] + A0[1] * T0[1] + A0[2] * T0[2];
    const float cxy = A0[0] * T1[0] + A0[1] * T1[1] + A0[2] * T1[2];
    const float byy = A1[0] * T1[0] + A1[1] * T1[1] + A1[2] * T1[2];
    const float cxx = bxx + dil, cyy = byy + dil;
    const float det = cxx * cyy - cxy * cxy;
    if (!(det > 0.f) || !isfinite(det)) return;
    const float idet = 1.f / det;
    if (mip) sig_eff *= sqrtf(fmaxf(bxx * byy - cxy * cxy, 0.f) * idet);

    GRec g;
    g.px = V.fx * mx * iz + V.cx;
    g.py = V.fy * my * iz + V.cy;
    g.ca = cyy * idet;
    g.cb = -cxy * idet;
    g.cc = cxx * idet;
    g.sigma = sig_eff;
    g.lsig = log2f(sig_eff);
    const float eps = a.opt.eps_const >= 0.f ? a.opt.eps_const : a.opt.eps_factor * (1.f / 3.f) * (s0 + s1 + s2);
    g.dme = mz - eps;
    g.depth = mz;
    g.r = g.g = g.b = 0.f;  // set by the count pass where the Gaussian keeps an entry
    *rec = g;

    // pixel box of the ellipse alpha >= alpha_min: q <= 2 ln(sigma / alpha_min)
    const float kq = 2.f * logf(sig_eff / a.opt.alpha_min);
    if (!(kq >= 0.f)) return;
    const float ex = sqrtf(kq * cxx) * 1.001f + 0.01f;
    const float ey = sqrtf(kq * cyy) * 1.001f + 0.01f;
    int x0, x1, y0, y1;
    if (!pixel_range((double)g.px - ex, (double)g.px + ex, V.W, x0, x1)) return;
    if (!pixel_range((double)g.py - ey, (double)g.py + ey, V.H, y0, y1)) return;
    *box = pack_box(x0, y0, x1, y1);
    const int TW = a.opt.splat_tile_w, TH = a.opt.splat_tile_h;
    *nt = (uint32_t)((x1 / TW - x0 / TW + 1) * (y1 / TH - y0 / TH + 1));
}

// ---------------------------------------------------------------------------
// 2D Gaussians (2D-GES, Sec. 6.4): plane set-up, support box, tile count

__device__ bool disc_box(const float mu[3], const float tu[3], const float tv[3], float su, float sv, float Rs,
                         double zext, float znear, float fx, float cx, int W, float fy, float cy, int H, int &x0,
                         int &y0, int &x1, int &y1);

// The splat's plane folded as a surfel's disc in units of its scales (see
// G2Rec), eps = (5/2)(s_u + s_v) (Sec. 5 with D = 2), and the pixel box of
// its support: alpha = sigma exp(-rho^2/2) >= alpha_min on the disc
// rho^2 <= 2 ln(sigma / alpha_min), boxed like a surfel's disc.  The
// colour is set by the count pass, as for 3D Gaussians.
__device__ void project_gauss2d(const FrameArgs &a, int v, int64_t i) {
    if (i >= a.m) return;
    const ViewDev &V = a.views[v];
    const int64_t m = a.m;
    const int64_t vi = (int64_t)v * m + i;
    G2Rec *rec = reinterpret_cast<G2Rec *>(a.ws + a.L.grec) + vi;
    uint2 *box = reinterpret_cast<uint2 *>(a.ws + a.L.gbox) + vi;
    uint32_t *nt = reinterpret_cast<uint32_t *>(a.ws + a.L.g_boff) + vi;
    *box = make_uint2(kEmptyBoxX, 0u);
    *nt = 0;

    const float px = a.G.mean[i], py = a.G.mean[m + i], pz = a.G.mean[2 * m + i];
    float qw = a.G.quat[i], qx = a.G.quat[m + i], qy = a.G.quat[2 * m + i], qz = a.G.quat[3 * m + i];
    const float su = a.G.scale[i], sv = a.G.scale[m + i];
    const float sigma = a.G.opacity[i];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qn > 0.f) || !isfinite(qn) || !(su > 0.f) || !(sv > 0.f) || !(sigma >= a.opt.alpha_min)) return;
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    const float *Rc = V.R;
    float mu[3], tu[3], tv[3], nn[3];
    for (int r = 0; r < 3; ++r) {
        mu[r] = Rc[3 * r] * px + Rc[3 * r + 1] * py + Rc[3 * r + 2] * pz + V.t[r];
        tu[r] = Rc[3 * r] * Rq[0] + Rc[3 * r + 1] * Rq[3] + Rc[3 * r + 2] * Rq[6];
        tv[r] = Rc[3 * r] * Rq[1] + Rc[3 * r + 1] * Rq[4] + Rc[3 * r + 2] * Rq[7];
        nn[r] = Rc[3 * r] * Rq[2] + Rc[3 * r + 1] * Rq[5] + Rc[3 * r + 2] * Rq[8];
    }
    if (!isfinite(mu[0] + mu[1] + mu[2])) return;
    float w = nn[0] * mu[0] + nn[1] * mu[1] + nn[2] * mu[2];
    if (w < 0.f) {
        w = -w;
        nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2];
    }
    if (!(w > 0.f)) return;  // plane through the camera centre: no hit in front
    const float mut = mu[0] * tu[0] + mu[1] * tu[1] + mu[2] * tu[2];
    const float muv = mu[0] * tv[0] + mu[1] * tv[1] + mu[2] * tv[2];
    const float iu = 1.f / su, iv = 1.f / sv;
    G2Rec g;
    g.Ux = (w * tu[0] - mut * nn[0]) * iu;
    g.Uy = (w * tu[1] - mut * nn[1]) * iu;
    g.Uz = (w * tu[2] - mut * nn[2]) * iu;
    g.Vx = (w * tv[0] - muv * nn[0]) * iv;
    g.Vy = (w * tv[1] - muv * nn[1]) * iv;
    g.Vz = (w * tv[2] - muv * nn[2]) * iv;
    g.nx = nn[0]; g.ny = nn[1]; g.nz = nn[2];
    g.w = w;
    g.sigma = sigma;
    g.eps = a.opt.eps_const >= 0.f ? a.opt.eps_const : a.opt.eps_factor * 0.5f * (su + sv);
    // support radius in scaled units, and the smallest depth over it
    // (lowered by 1e-4 relative: no FP32 planar depth w / c falls below it)
    const float Rs = sqrtf(2.f * logf(sigma / a.opt.alpha_min)) * 1.0001f + 1e-4f;
    const double az = (double)su * tu[2], bz = (double)sv * tv[2];
    const double zext = (double)Rs * sqrt(az * az + bz * bz);
    const double zlo = (double)mu[2] - zext;
    g.dme = (float)(zlo - 1e-4 * fabs(zlo) - 1e-6) - g.eps;
    g.r = g.g = g.b = 0.f;
    *rec = g;
    int x0, x1, y0, y1;
    if (!disc_box(mu, tu, tv, su, sv, Rs, zext, V.znear, V.fx, V.cx, V.W, V.fy, V.cy, V.H, x0, y0, x1, y1)) return;
    *box = pack_box(x0, y0, x1, y1);
    const int TW = a.opt.splat_tile_w, TH = a.opt.splat_tile_h;
    *nt = (uint32_t)((x1 / TW - x0 / TW + 1) * (y1 / TH - y0 / TH + 1));
}

// ---------------------------------------------------------------------------
// the screen box of a disc (the support of a 2D Gaussian)

// (The surfel set-up computes the same box inline: factored through this
// helper, the projection kernel needed 84 VGPRs instead of 78, one wave
// less per SIMD.)
// Pixel box, on a W x H grid with focal lengths fx, fy and principal point
// cx, cy, of the disc mu + Rs (x su tu + y sv tv), x^2 + y^2 <= 1 (camera
// space; tu, tv unit axes; zext its extent along z, Rs |(su tu_z, sv tv_z)|):
// the tangents of its dual conic where the disc
// lies wholly in front of the near plane, else the box of the square
// [-Rs, Rs]^2 clipped to z >= znear (it holds the visible part of the
// disc); widened by 1e-3 of its size plus 0.02 pixel.  False when no part
// of the disc is in front of the near plane or on the grid.  Double
// precision throughout.
__device__ bool disc_box(const float mu[3], const float tu[3], const float tv[3], float su, float sv, float Rs,
                         double zext, float znear, float fx, float cx, int W, float fy, float cy, int H, int &x0,
                         int &y0, int &x1, int &y1) {
    const double zmax = (double)mu[2] + zext, zmin = (double)mu[2] - zext;
    if (zmax < (double)znear) return false;
    double xlo, xhi, ylo, yhi;
    const double R2 = (double)Rs * Rs;
    const double ax = (double)su * tu[0], ay = (double)su * tu[1], azz = (double)su * tu[2];
    const double bx = (double)sv * tv[0], by = (double)sv * tv[1], bzz = (double)sv * tv[2];
    const double m0 = mu[0], m1 = mu[1], m2 = mu[2];
    if (zmin >= (double)znear) {
        // dual conic of the disc, H diag(R^2, R^2, -1) H^T with H = [a | b | mu]:
        // tangent lines x/z = k solve Q00 - 2 k Q02 + k^2 Q22 = 0
        const double Q00 = R2 * (ax * ax + bx * bx) - m0 * m0;
        const double Q11 = R2 * (ay * ay + by * by) - m1 * m1;
        const double Q22 = R2 * (azz * azz + bzz * bzz) - m2 * m2;
        const double Q02 = R2 * (ax * azz + bx * bzz) - m0 * m2;
        const double Q12 = R2 * (ay * azz + by * bzz) - m1 * m2;
        const double dxs = sqrt(fmax(Q02 * Q02 - Q00 * Q22, 0.0));
        const double dys = sqrt(fmax(Q12 * Q12 - Q11 * Q22, 0.0));
        const double kx0 = (Q02 + dxs) / Q22, kx1 = (Q02 - dxs) / Q22;
        const double ky0 = (Q12 + dys) / Q22, ky1 = (Q12 - dys) / Q22;
        xlo = fmin(kx0, kx1); xhi = fmax(kx0, kx1);
        ylo = fmin(ky0, ky1); yhi = fmax(ky0, ky1);
    } else {
        double P[4][3];
        const double sg[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        const double Rd = Rs;
        for (int k = 0; k < 4; ++k) {
            P[k][0] = m0 + Rd * (sg[k][0] * ax + sg[k][1] * bx);
            P[k][1] = m1 + Rd * (sg[k][0] * ay + sg[k][1] * by);
            P[k][2] = m2 + Rd * (sg[k][0] * azz + sg[k][1] * bzz);
        }
        xlo = ylo = 1e300;
        xhi = yhi = -1e300;
        const double zn = znear;
        for (int k = 0; k < 4; ++k) {
            const double *A = P[k], *B = P[(k + 1) & 3];
            if (A[2] >= zn) {
                xlo = fmin(xlo, A[0] / A[2]); xhi = fmax(xhi, A[0] / A[2]);
                ylo = fmin(ylo, A[1] / A[2]); yhi = fmax(yhi, A[1] / A[2]);
            }
            if ((A[2] >= zn) != (B[2] >= zn)) {
                const double tt = (zn - A[2]) / (B[2] - A[2]);
                const double X = A[0] + tt * (B[0] - A[0]), Yy = A[1] + tt * (B[1] - A[1]);
                xlo = fmin(xlo, X / zn); xhi = fmax(xhi, X / zn);
                ylo = fmin(ylo, Yy / zn); yhi = fmax(yhi, Yy / zn);
            }
        }
    }
    double plo = (double)fx * xlo + cx, phi = (double)fx * xhi + cx;
    double qlo = (double)fy * ylo + cy, qhi = (double)fy * yhi + cy;
    const double padx = 1e-3 * (phi - plo) + 0.02, pady = 1e-3 * (qhi - qlo) + 0.02;
    if (!pixel_range(plo - padx, phi + padx, W, x0, x1)) return false;
    if (!pixel_range(qlo - pady, qhi + pady, H, y0, y1)) return false;
    return true;
}

// ---------------------------------------------------------------------------
// surfels: disc set-up, exact screen box, raster-tile count

template <bool TL>  // translucent surfels: no occluders
__device__ void project_surfel(const FrameArgs &a, int v, int64_t j) {
    if (j >= a.n) return;
    const ViewDev &V = a.views[v];
    const int64_t n = a.n;
    const int64_t vj = (int64_t)v * n + j;
    SRec *rec = reinterpret_cast<SRec *>(a.ws + a.L.srec) + vj;
    uint2 *box = reinterpret_cast<uint2 *>(a.ws + a.L.sbox) + vj;
    uint32_t *nt = reinterpret_cast<uint32_t *>(a.ws + a.L.s_boff) + vj;
    *box = make_uint2(kEmptyBoxX, 0u);
    *nt = 0;

    const float px = a.S.mean[j], py = a.S.mean[n + j], pz = a.S.mean[2 * n + j];
    float qw = a.S.quat[j], qx = a.S.quat[n + j], qy = a.S.quat[2 * n + j], qz = a.S.quat[3 * n + j];
    const float su = a.S.scale[j], sv = a.S.scale[n + j];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qn > 0.f) || !isfinite(qn) || !(su > 0.f) || !(sv > 0.f)) return;
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    float Rq[9];
    quat_rot(qw, qx, qy, qz, Rq);
    const float *Rc = V.R;
    float mu[3], tu[3], tv[3], nn[3];
    for (int r = 0; r < 3; ++r) {
        mu[r] = Rc[3 * r] * px + Rc[3 * r + 1] * py + Rc[3 * r + 2] * pz + V.t[r];
        tu[r] = Rc[3 * r] * Rq[0] + Rc[3 * r + 1] * Rq[3] + Rc[3 * r + 2] * Rq[6];
        tv[r] = Rc[3 * r] * Rq[1] + Rc[3 * r + 1] * Rq[4] + Rc[3 * r + 2] * Rq[7];
        nn[r] = Rc[3 * r] * Rq[2] + Rc[3 * r + 1] * Rq[5] + Rc[3 * r + 2] * Rq[8];
    }
    if (!isfinite(mu[0] + mu[1] + mu[2])) return;
    float w = nn[0] * mu[0] + nn[1] * mu[1] + nn[2] * mu[2];
    if (w < 0.f) {
        w = -w;
        nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2];
    }
    if (!(w > 0.f)) return;  // plane through the camera centre: no hit in front
    const float Rs = a.opt.surfel_radius;
    const float mut = mu[0] * tu[0] + mu[1] * tu[1] + mu[2] * tu[2];
    const float muv = mu[0] * tv[0] + mu[1] * tv[1] + mu[2] * tv[2];
    const float iu = 1.f / (su * Rs), iv = 1.f / (sv * Rs);
    SRec s;
    s.Ux = (w * tu[0] - mut * nn[0]) * iu;
    s.Uy = (w * tu[1] - mut * nn[1]) * iu;
    s.Uz = (w * tu[2] - mut * nn[2]) * iu;
    s.Vx = (w * tv[0] - muv * nn[0]) * iv;
    s.Vy = (w * tv[1] - muv * nn[1]) * iv;
    s.Vz = (w * tv[2] - muv * nn[2]) * iv;
    s.nx = nn[0]; s.ny = nn[1]; s.nz = nn[2];
    s.w = w;
    // exact extent of the disc along camera z
    const double az = (double)su * tu[2], bz = (double)sv * tv[2];
    const double zext = (double)Rs * sqrt(az * az + bz * bz);
    // lowered by 1e-4 relative so that no FP32 hit depth w / c of this disc
    // falls below it (the raster's occlusion cull compares against it)
    const double zlo = (double)mu[2] - zext, zhi = (double)mu[2] + zext;
    s.zmin = (float)(zlo - 1e-4 * fabs(zlo) - 1e-6);
    s.zmax = (float)(zhi + 1e-4 * fabs(zhi) + 1e-6);
    // translucent surfels have no occluders (zmax is not needed): the slot
    // carries the centre depth, the key of their blend order
    if (TL) s.zmax = mu[2];
    *rec = s;
    reinterpret_cast<float *>(a.ws + a.L.s_zmin)[vj] = s.zmin;  // the count pass reads it alone
    const double zmax = (double)mu[2] + zext, zmin = (double)mu[2] - zext;
    if (zmax < (double)V.znear) return;

    // screen box of the disc, in double precision
    double xlo, xhi, ylo, yhi;
    const double R2 = (double)Rs * Rs;
    const double ax = (double)su * tu[0], ay = (double)su * tu[1], azz = (double)su * tu[2];
    const double bx = (double)sv * tv[0], by = (double)sv * tv[1], bzz = (double)sv * tv[2];
    const double m0 = mu[0], m1 = mu[1], m2 = mu[2];
    if (zmin >= (double)V.znear) {
        // dual conic of the disc, H diag(R^2, R^2, -1) H^T with H = [a | b | mu]:
        // tangent lines x/z = k solve Q00 - 2 k Q02 + k^2 Q22 = 0
        const double Q00 = R2 * (ax * ax + bx * bx) - m0 * m0;
        const double Q11 = R2 * (ay * ay + by * by) - m1 * m1;
        const double Q22 = R2 * (azz * azz + bzz * bzz) - m2 * m2;
        const double Q02 = R2 * (ax * azz + bx * bzz) - m0 * m2;
        const double Q12 = R2 * (ay * azz + by * bzz) - m1 * m2;
        const double dxs = sqrt(fmax(Q02 * Q02 - Q00 * Q22, 0.0));
        const double dys = sqrt(fmax(Q12 * Q12 - Q11 * Q22, 0.0));
        const double kx0 = (Q02 + dxs) / Q22, kx1 = (Q02 - dxs) / Q22;
        const double ky0 = (Q12 + dys) / Q22, ky1 = (Q12 - dys) / Q22;
        xlo = fmin(kx0, kx1); xhi = fmax(kx0, kx1);
        ylo = fmin(ky0, ky1); yhi = fmax(ky0, ky1);
    } else {
        // disc straddles the near plane: box of the square [-R,R]^2 clipped
        // to z >= znear (contains the visible part of the disc)
        double P[4][3];
        const double sg[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        const double Rd = Rs;
        for (int k = 0; k < 4; ++k) {
            P[k][0] = m0 + Rd * (sg[k][0] * ax + sg[k][1] * bx);
            P[k][1] = m1 + Rd * (sg[k][0] * ay + sg[k][1] * by);
            P[k][2] = m2 + Rd * (sg[k][0] * azz + sg[k][1] * bzz);
        }
        xlo = ylo = 1e300;
        xhi = yhi = -1e300;
        const double zn = V.znear;
        for (int k = 0; k < 4; ++k) {
            const double *A = P[k], *B = P[(k + 1) & 3];
            if (A[2] >= zn) {
                xlo = fmin(xlo, A[0] / A[2]); xhi = fmax(xhi, A[0] / A[2]);
                ylo = fmin(ylo, A[1] / A[2]); yhi = fmax(yhi, A[1] / A[2]);
            }
            if ((A[2] >= zn) != (B[2] >= zn)) {
                const double tt = (zn - A[2]) / (B[2] - A[2]);
                const double X = A[0] + tt * (B[0] - A[0]), Yy = A[1] + tt * (B[1] - A[1]);
                xlo = fmin(xlo, X / zn); xhi = fmax(xhi, X / zn);
                ylo = fmin(ylo, Yy / zn); yhi = fmax(yhi, Yy / zn);
            }
        }
    }
    // (in the surfel pass's sample grid)
    double plo = (double)V.sfx * xlo + V.scx, phi = (double)V.sfx * xhi + V.scx;
    double qlo = (double)V.sfy * ylo + V.scy, qhi = (double)V.sfy * yhi + V.scy;
    const double padx = 1e-3 * (phi - plo) + 0.02, pady = 1e-3 * (qhi - qlo) + 0.02;
    int x0, x1, y0, y1;
    if (!pixel_range(plo - padx, phi + padx, V.sW, x0, x1)) return;
    if (!pixel_range(qlo - pady, qhi + pady, V.sH, y0, y1)) return;
    *box = pack_box(x0, y0, x1, y1);
    const int T = a.opt.raster_tile;
    const int ntx = x1 / T - x0 / T + 1, nty = y1 / T - y0 / T + 1;
    *nt = (uint32_t)(ntx * nty);
    if (TL) {  // every surfel on screen gets its colour; no occluders
        a.ws[a.L.svis + vj] = 1;
        return;
    }
    // occluder: a disc wholly in front of the near plane whose projection
    // (an ellipse, convex) holds the four corner pixel centres of a tile's
    // in-image part holds every pixel of it, so the tile's final depth is at
    // most the disc's zmax.  The corners are tested against the disc shrunk
    // to 0.99 R^2, far beyond the FP32 error of the raster's own test (and of
    // the reciprocal focal lengths used here).  Only tiles whole inside the
    // disc's pixel box can be covered.
    if (zmin > (double)V.znear * 1.001 && ntx * nty <= kOccluderTiles) {
        unsigned int *tocc = reinterpret_cast<unsigned int *>(a.ws + a.L.s_tocc);
        const unsigned int zbits = __float_as_uint(s.zmax);  // positive floats order as their bits
        const float ifx = 1.f / V.sfx, ify = 1.f / V.sfy;
        for (int ty = (y0 + T - 1) / T; ty * T + T - 1 <= y1 || (ty * T <= y1 && y1 == V.sH - 1); ++ty)
            for (int tx = (x0 + T - 1) / T; tx * T + T - 1 <= x1 || (tx * T <= x1 && x1 == V.sW - 1); ++tx) {
                const int ti = V.rt_off + ty * V.rtx + tx;
                const int cx0 = tx * T, cx1 = min(tx * T + T - 1, V.sW - 1);
                const int cy0 = ty * T, cy1 = min(ty * T + T - 1, V.sH - 1);
                bool cover = true;
                for (int c4 = 0; c4 < 4 && cover; ++c4) {
                    const float xr = ((float)((c4 & 1) ? cx1 : cx0) + 0.5f - V.scx) * ifx;
                    const float yr = ((float)((c4 & 2) ? cy1 : cy0) + 0.5f - V.scy) * ify;
                    const float c = s.nx * xr + s.ny * yr + s.nz;
                    const float au = s.Ux * xr + s.Uy * yr + s.Uz;
                    const float bv = s.Vx * xr + s.Vy * yr + s.Vz;
                    cover = (c > 0.f) && (au * au + bv * bv <= 0.99f * c * c);
                }
                if (cover) atomicMin(tocc + ti, zbits);  // no return value: nothing waits on it
            }
    }
}

// Both projections in one launch (they are independent): blocks below
// gblocks take Gaussians, the others surfels; blockIdx.y is the view.
// (The modes are template arguments: the opaque 3D instance keeps the
// register budget, and so the occupancy, of a kernel without them.)
template <bool G2, bool TL>
__global__ void __launch_bounds__(256) k_project(FrameArgs a, int gblocks) {
    const int v = blockIdx.y;
    if ((int)blockIdx.x < gblocks) {
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (G2) project_gauss2d(a, v, i);
        else project_gaussian(a, v, i);
    } else project_surfel<TL>(a, v, (int64_t)(blockIdx.x - gblocks) * blockDim.x + threadIdx.x);
}

// Count pass: one atomic per (surfel, raster tile) that the tile's occluder
// does not hide; the returned position in the tile's list is kept in the
// surfel's slot run (kNoSlot for a hidden tile).  Hidden: the surfel's
// smallest z is strictly beyond the tile's occluder depth, so every hit of
// it is farther than the occluder's hit at the same pixel and it can win no
// pixel (the occluder itself is never hidden: its zmin <= its zmax).
// The pass is bound by the device's rate of global atomics (about 24 G/s
// on MI355X whatever their scope, layout or use of the return value), so
// its time follows the number of pairs the occluders leave.
__global__ void __launch_bounds__(256) k_surfel_count(FrameArgs a) {
    const int v = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const ViewDev &V = a.views[v];
    const int64_t vj = (int64_t)v * a.n + j;
    int x0, y0, x1, y1;
    unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
    if (x0 > x1) return;
    uint32_t *tcount = reinterpret_cast<uint32_t *>(a.ws + a.L.s_tcnt);
    uint32_t *slot = reinterpret_cast<uint32_t *>(a.ws + a.L.s_slot);
    const float *tocc = reinterpret_cast<const float *>(a.ws + a.L.s_tocc);
    const float zmin = reinterpret_cast<const float *>(a.ws + a.L.s_zmin)[vj];
    const uint64_t base = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff)[vj];
    const int T = a.opt.raster_tile;
    // a slot run past capacity stops the walk; the scan total flags it
    TileWalk w(x0 / T, y0 / T, x1 / T, y1 / T, base, (uint64_t)a.L.s_cap);
    const int t0 = V.rt_off, tw = V.rtx;  // in registers: no reload after each atomic
    const uint32_t copy = counter_copy();
    for (int64_t i0 = 0; i0 < w.count; i0 += kWalkBatch) {
        uint32_t r[kWalkBatch];
        int t[kWalkBatch];
        float occ[kWalkBatch];
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b)
            if (i0 + b < w.count) {
                t[b] = t0 + w.ty * tw + w.tx;
                occ[b] = tocc[t[b]];
                w.next();
            }
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b)  // all atomics of a batch in flight before the first wait
            if (i0 + b < w.count)
                r[b] = zmin > occ[b] ? kNoSlot
                                     : atomicAdd(&tcount[((int64_t)t[b] * kCounterCopies + copy) * kCounterStride], 1u);
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b)
            if (i0 + b < w.count)  // a position past kCopyPosMask exceeds the capacity: the total flags it
                slot[base + i0 + b] = r[b] == kNoSlot ? kNoSlot : (copy << kCopyShift) | (r[b] & kCopyPosMask);
    }
}

// Launch order of a tile pass (TileOrd): one block of 256 threads counts
// the tiles per class of list length in LDS, turns the counts into the
// classes' start positions (longest class first) and places every tile at
// the next position of its class.  toff: the scanned per-tile offsets, the
// tile's at toff[t * copies].  It runs as the first block of the fill launch
// (the other blocks fill the lists), so the pass that follows finds it done.
__device__ void order_tiles(const uint32_t *toff, int copies, int ntiles, TileOrd *ord) {
    __shared__ uint32_t cls_pos[kOrdClasses];
    const int tid = (int)threadIdx.x;
    if (tid < kOrdClasses) cls_pos[tid] = 0u;
    __syncthreads();
#pragma unroll 4
    for (int t = tid; t < ntiles; t += 256)
        atomicAdd(&cls_pos[ord_class(toff[(int64_t)(t + 1) * copies] - toff[(int64_t)t * copies])], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int c = kOrdClasses - 1; c >= 0; --c) {
            const uint32_t k = cls_pos[c];
            cls_pos[c] = run;
            run += k;
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int t = tid; t < ntiles; t += 256) {
        const uint32_t b0 = toff[(int64_t)t * copies], b1 = toff[(int64_t)(t + 1) * copies];
        const uint32_t at = atomicAdd(&cls_pos[ord_class(b1 - b0)], 1u);
        ord[at] = TileOrd{(uint32_t)t, b0, b1, 0u};
    }
}

// Launch order of the splat tiles (pass 2 and its backward read 16 to 44
// bytes per pixel, and a 16-pixel tile row is half of a 128-byte line that
// its right or left neighbour shares): as order_tiles, but by horizontal
// pairs of tiles (class: the longer list of the two), and the pair's tiles
// go to blocks b and b + 8, which the dispatcher hands to the same XCD, so
// a shared line is fetched by one L2.  A view's odd last column takes the
// places after every pair.  Sequence place s of a pair's tile (2 q, 2 q + 1
// for the q-th pair) becomes block (s / 16) 16 + (s % 2) 8 + (s / 2) % 8
// in whole groups of 16, s itself in the last partial group.
__device__ void order_tile_pairs(const ViewDev *views, int n_views, const uint32_t *toff, int ntiles,
                                 TileOrd *ord) {
    __shared__ uint32_t cls_pos[2 * kOrdClasses];  // pairs' classes, then singles'
    const int tid = (int)threadIdx.x;
    if (tid < 2 * kOrdClasses) cls_pos[tid] = 0u;
    __syncthreads();
    // Units: a view's tile columns 2c, 2c + 1 of a row (a pair), or its odd
    // last column alone; per view (its sizes uniform) thread tid takes units
    // tid, tid + 256, ...
    for (int v = 0; v < n_views; ++v) {
        const int sx = views[v].stx, pcx = (sx + 1) >> 1, nu = pcx * views[v].sty, off = views[v].st_off;
#pragma unroll 4
        for (int u = tid; u < nu; u += 256) {
            const int row = u / pcx, tx = 2 * (u - row * pcx), t = off + row * sx + tx;
            const bool pair = tx + 1 < sx;
            const uint32_t len = toff[t + 1] - toff[t], len2 = pair ? toff[t + 2] - toff[t + 1] : 0u;
            atomicAdd(&cls_pos[(pair ? 0 : kOrdClasses) + ord_class(len > len2 ? len : len2)], 1u);
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;  // in pairs, longest class first
        for (int c = kOrdClasses - 1; c >= 0; --c) {
            const uint32_t k = cls_pos[c];
            cls_pos[c] = run;
            run += k;
        }
        uint32_t run1 = 2 * run;  // singles: sequence places after the pairs
        for (int c = kOrdClasses - 1; c >= 0; --c) {
            const uint32_t k = cls_pos[kOrdClasses + c];
            cls_pos[kOrdClasses + c] = run1;
            run1 += k;
        }
    }
    __syncthreads();
    const uint32_t full = (uint32_t)(ntiles / 16) * 16;  // whole groups of 16 sequence places
    auto block_of = [&](uint32_t sq) -> uint32_t {
        return sq < full ? (sq / 16) * 16 + (sq % 2) * 8 + (sq / 2) % 8 : sq;
    };
    for (int v = 0; v < n_views; ++v) {
        const int sx = views[v].stx, pcx = (sx + 1) >> 1, nu = pcx * views[v].sty, off = views[v].st_off;
#pragma unroll 4
        for (int u = tid; u < nu; u += 256) {
            const int row = u / pcx, tx = 2 * (u - row * pcx), t = off + row * sx + tx;
            const uint32_t b0 = toff[t], b1 = toff[t + 1];
            if (tx + 1 < sx) {
                const uint32_t b2 = toff[t + 2], len = b1 - b0, len2 = b2 - b1;
                const uint32_t sq = 2 * atomicAdd(&cls_pos[ord_class(len > len2 ? len : len2)], 1u);
                ord[block_of(sq)] = TileOrd{(uint32_t)t, b0, b1, 0u};
                ord[block_of(sq + 1)] = TileOrd{(uint32_t)(t + 1), b1, b2, 0u};
            } else {
                const uint32_t sq = atomicAdd(&cls_pos[kOrdClasses + ord_class(b1 - b0)], 1u);
                ord[block_of(sq)] = TileOrd{(uint32_t)t, b0, b1, 0u};
            }
        }
    }
}

// Fill pass: entry toff[t] + slot gets the surfel's raster record, its
// index and its box inside the tile -- one aligned 64-byte line, no atomics.
// The lines are written four lanes to a line: each lane stages its surfel's
// record in LDS, the wave compacts the kept entries of one tile of the walk
// (ballot + rank), and lanes 4e .. 4e+3 store the four 16-byte quarters of
// entry e, so a store instruction writes 16 whole lines instead of 64
// scattered quarters.
template <bool TL>  // translucent surfels: the entries carry centre depth, w and slot
__global__ void __launch_bounds__(256) k_surfel_fill(FrameArgs a) {
    __shared__ float4 rec_l[4][64][3];   // per wave: each lane's record
    __shared__ uint32_t pos_l[4][64];    // per wave: compacted entries of one walk step
    __shared__ uint32_t src_l[4][64];    // (lane | lbox << 8)
    __shared__ uint32_t k_l[4][64];      // translucent: the entries' slot indices
    __shared__ float2 tz_l[4][64];       // translucent: each lane's centre depth and w_mod
    const int v = blockIdx.y;
    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_toff);
    if (blockIdx.x == 0) {  // block-uniform: the raster's launch order, once
        if (blockIdx.y == 0) {
            // the persistent raster's tile queues start empty
            WsHeader *hdr = reinterpret_cast<WsHeader *>(a.ws + a.L.header);
            if (threadIdx.x < 8) hdr->raster_q[threadIdx.x * kCounterStride] = 0u;
            order_tiles(toff, kCounterCopies, a.L.rtiles, reinterpret_cast<TileOrd *>(a.ws + a.L.s_ord));
        }
        return;
    }
    const int64_t j = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const ViewDev &V = a.views[v];
    const uint32_t *slot = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_slot);
    float4 *ents = reinterpret_cast<float4 *>(a.ws + a.L.s_ents);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(a.ws + a.L.header);
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const int T = a.opt.raster_tile;
    int x0 = 1, y0 = 0, x1 = 0, y1 = 0;
    uint64_t base = 0;
    if (j < a.n) {
        const int64_t vj = (int64_t)v * a.n + j;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.sbox)[vj], x0, y0, x1, y1);
        const float4 *rec = reinterpret_cast<const float4 *>(a.ws + a.L.srec) + vj * 3;
        rec_l[wv][lane][0] = rec[0];
        rec_l[wv][lane][1] = rec[1];
        float4 r2 = rec[2];
        if (TL) tz_l[wv][lane] = make_float2(r2.w, a.w_mod[j]);  // centre depth (in zmax's slot), w
        r2.w = __uint_as_float((uint32_t)j);
        rec_l[wv][lane][2] = r2;
        base = reinterpret_cast<const uint32_t *>(a.ws + a.L.s_boff)[vj];
    }
    TileWalk w(x0 / T, y0 / T, x1 / T, y1 / T, base, cap);
    const int64_t cnt = x0 > x1 ? 0 : w.count;
    if (x0 <= x1 && w.count < w.total) set_flag(hdr, kFlagSurfelOverflow);
    const int t0 = V.rt_off, tw = V.rtx;
    for (int64_t i0 = 0; __any((int)(i0 < cnt)); i0 += kWalkBatch) {
        uint32_t sl[kWalkBatch], to[kWalkBatch], lb[kWalkBatch];
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b)  // the batch's loads in flight together
            if (i0 + b < cnt) {
                sl[b] = slot[base + i0 + b];
                to[b] = sl[b] == kNoSlot ? 0u : toff[(t0 + w.ty * tw + w.tx) * kCounterCopies + (sl[b] >> kCopyShift)];
                lb[b] = pack_lbox(x0, y0, x1, y1, w.tx * T, w.ty * T, T, T);
                w.next();
            }
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b) {
            bool keep = false;
            uint64_t pos = 0;
            if (i0 + b < cnt && sl[b] != kNoSlot) {  // kNoSlot: hidden by the tile's occluder
                pos = (uint64_t)to[b] + (sl[b] & kCopyPosMask);
                keep = pos < cap;
                if (!keep) {
                    set_flag(hdr, kFlagSurfelOverflow);
                    if (TL) {  // lost to the overflow: its backward partial reads zero
                        float *tp = reinterpret_cast<float *>(a.ws + a.L.t_part) + (base + i0 + b) * kTPartials;
                        for (int c = 0; c < kTPartials; ++c) tp[c] = 0.f;
                    }
                }
            }
            const unsigned long long m = __ballot((int)keep);
            if (m == 0ull) continue;  // wave-uniform
            const int total = __popcll(m);
            if (keep) {
                const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                pos_l[wv][r] = (uint32_t)pos;  // pos < cap <= 2^29
                src_l[wv][r] = (uint32_t)lane | (lb[b] << 8);
                k_l[wv][r] = (uint32_t)(base + i0 + b);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int e0 = 0; e0 < total; e0 += 16) {
                const int e = e0 + (lane >> 2), q = lane & 3;
                if (e < total) {
                    const uint32_t sv = src_l[wv][e];
                    // the record; then the box inside the tile and, for translucent
                    // surfels, the centre depth, w and the entry's slot index
                    const float2 tz = TL ? tz_l[wv][sv & 63u] : make_float2(0.f, 0.f);
                    const float4 val = q < 3 ? rec_l[wv][sv & 63u][q]
                                             : make_float4(__uint_as_float(sv >> 8), tz.x, tz.y,
                                                           __uint_as_float(k_l[wv][e]));
                    ents[(uint64_t)pos_l[wv][e] * 4 + q] = val;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // reads done before the next step's writes
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// ---------------------------------------------------------------------------
// pass 1: z-buffer by per-lane minimum over the tile's list

// Front to back with occlusion culling.  A batch of list entries is ordered
// by each disc's smallest camera z (conservative: no hit of the disc is
// nearer; a counting sort into 64 depth buckets, nearest first), then
// rasterised in groups of 64: before each group, the tile's
// far depth (largest current depth over its in-image pixels, infinite while
// any is uncovered) is taken, and an entry whose smallest z is strictly
// beyond it cannot win any pixel of the tile and is skipped.  Strictly: a
// hit at exactly the current depth could still win its pixel by a smaller
// id.
//
// Inside a group the work is split by (entry, box row, 8-pixel half of the
// tile row): a wave scan of the entries' fragment counts gives each fragment
// a slot, and a lane tests only the pixels of its fragment against that
// surfel, folding hits into the tile's z-buffer with an LDS 64-bit minimum.
// The minimum of the packed keys (depth bits << 32 | id) does not depend on
// the order of the updates, so the ids are bit-identical to a plain pass over
// all entries.  The hit depth w / c uses the hardware reciprocal (w * rcp(c),
// within 2 ulp), the same expression in every tile shape.
// (64 VGPRs at most: with the LDS under 20 KB, eight blocks of 256 share a CU)
template <int T>
__device__ __forceinline__ unsigned long long raster_tile(const FrameArgs &a, const TileOrd o, int32_t *sid,
                                                          float *depth) {
    const int t = (int)o.tile;
    constexpr int NT = T * T;
    constexpr int NH = T / 8;   // 8-pixel halves per tile row
    constexpr int GS = 64;      // entries per front-to-back group (one wave scans them)
    static_assert(NT <= 256 && T <= 16, "fragment codes hold an 8-bit entry, a 4-bit row and a half");
    __shared__ float4 lds[NT * 3];
    __shared__ uint32_t lbx[NT];
    constexpr int NB = 64;      // depth buckets of the batch sort
    __shared__ uint8_t order[NT];
    __shared__ uint16_t frag[GS * T * NH];
    __shared__ int hist[NB];
    __shared__ uint32_t wmin[NT / 64], wmax[NT / 64];
    // z-buffer rows padded to T + 1 entries: the 64-bit minima of a wave's
    // fragments (different rows, the same column offset) would otherwise
    // fall on a few banks (a row of T entries is a multiple of the bank count
    // in 4-byte words); the pads hold key 0, which never raises the far depth
    constexpr int ZS = T + 1;
    constexpr int NZ = T * ZS;
    __shared__ unsigned long long zb[NZ];
    __shared__ float xrs[T], yrs[T];
    __shared__ int gtotal;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    const int v = view_of_rtile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.rt_off;
    const int tx = lt % V.rtx, ty = lt / V.rtx;
    const int px = tx * T + tid % T, py = ty * T + tid / T;  // a point of the sample grid
    const float zn = V.znear;
    // out-of-image samples start at key 0: never hit, never hold the far depth up
    const int zi = (tid / T) * ZS + tid % T;  // this thread's pixel in the padded z-buffer
    zb[zi] = (px < V.sW && py < V.sH) ? ~0ull : 0ull;
    if (tid < T) zb[tid * ZS + T] = 0ull;  // the pads
    if (tid < T) xrs[tid] = ((float)(tx * T + tid) + 0.5f - V.scx) / V.sfx;
    else if (tid < 2 * T) yrs[tid - T] = ((float)(ty * T + tid - T) + 0.5f - V.scy) / V.sfy;

    const float4 *ents = reinterpret_cast<const float4 *>(a.ws + a.L.s_ents);
    const uint64_t cap = (uint64_t)a.L.s_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);
    __syncthreads();
    float xv[T];  // pixel-centre rays of the tile's columns, held in registers
#pragma unroll
    for (int i = 0; i < T; ++i) xv[i] = xrs[i];

    unsigned long long area = 0;  // box pixels of the fragments this thread evaluates
    for (uint64_t base = b0; base < b1; base += NT) {
        const int cnt = (int)umin64((uint64_t)NT, b1 - base);
        __syncthreads();  // the previous batch is done with the records
        uint32_t zkey = 0;
        if (tid < cnt) {
            const float4 *e = ents + (base + tid) * 4;
            lds[tid * 3] = e[0];
            lds[tid * 3 + 1] = e[1];
            const float4 r2 = e[2];
            lds[tid * 3 + 2] = r2;
            lbx[tid] = __float_as_uint(e[3].x);
            const uint32_t zb32 = __float_as_uint(r2.z);  // zmin as an order-preserving unsigned key
            zkey = (zb32 & 0x80000000u) ? ~zb32 : (zb32 | 0x80000000u);
        }
        // counting sort by zmin into NB buckets spread linearly over the
        // batch's key range: block min / max, one LDS atomic per entry for its
        // rank in the bucket, a scan of the bucket sizes.  The order only
        // schedules the work (the cull compares the exact zmin and every
        // result is order-independent), so ranks in a bucket may come in any
        // order.
        uint32_t kmin = wave_min_u32(tid < cnt ? zkey : ~0u), kmax = wave_max_u32(tid < cnt ? zkey : 0u);
        if (lane == 0) {
            wmin[tid >> 6] = kmin;
            wmax[tid >> 6] = kmax;
        }
        if (tid < NB) hist[tid] = 0;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            kmin = min(kmin, wmin[w]);
            kmax = max(kmax, wmax[w]);
        }
        int bkt = 0, rank = 0;
        if (tid < cnt) {
            const float scale = (float)NB / ((float)(kmax - kmin) + 1.f);
            bkt = min(NB - 1, (int)((float)(zkey - kmin) * scale));
            rank = atomicAdd(&hist[bkt], 1);
        }
        __syncthreads();
        static_assert(NB == 64, "one wave scans the buckets");
        if (tid < NB) hist[tid] = wave_scan_add(hist[tid], false);  // exclusive
        __syncthreads();
        if (tid < cnt) order[hist[bkt] + rank] = (uint8_t)tid;
        __syncthreads();  // records and order visible
        // groups of GS entries (a smaller first group, to start culling
        // earlier, measured slower: 32 -> +1 us, 16 -> +5 us)
        for (int g = 0, gs = GS; g < cnt; g += gs) {
            if (tid < GS) {  // wave 0: far depth, culling and the group's fragment slots
                // depth bits of the keys: positive floats order as their bits,
                // an uncovered pixel reads all ones (a NaN, which culls nothing)
                uint32_t far = 0;
#pragma unroll
                for (int i = 0; i < (NZ + GS - 1) / GS; ++i)
                    if (tid + i * GS < NZ) far = max(far, (uint32_t)(zb[tid + i * GS] >> 32));
                const float zfar = __uint_as_float(wave_max_u32(far));
                int nf = 0, h = 0, nh = 0, h0 = 0, k = 0;
                if (tid < gs && g + tid < cnt) {
                    k = order[g + tid];
                    if (!(lds[k * 3 + 2].z > zfar)) {
                        const uint32_t lb = lbx[k];
                        const int x0 = (int)(lb & 15), x1 = (int)((lb >> 4) & 15);
                        h = (int)((lb >> 12) & 15) - (int)((lb >> 8) & 15) + 1;
                        h0 = x0 >> 3;
                        nh = (x1 >> 3) - h0 + 1;
                        nf = h * nh;
                    }
                }
                const int inc = wave_scan_add(nf, true);
                if (lane == 63) gtotal = inc;
                int ex = inc - nf;
                // fragment code: entry | row << 8 | half << 12
                for (int r = 0; r < h; ++r)
                    for (int j = 0; j < nh; ++j) frag[ex++] = (uint16_t)(k | (r << 8) | ((h0 + j) << 12));
            }
            __syncthreads();
            const int total = gtotal;
            for (int f = tid; f < total; f += NT) {
                const uint32_t e = frag[f];
                const int k = (int)(e & 255), hf = (int)(e >> 12);
                const uint32_t lb = lbx[k];
                // r0 = (Ux,Uy,Uz,Vx) r1 = (Vy,Vz,nx,ny) r2 = (nz,w,zmin,id)
                const float4 r0 = lds[k * 3], r1 = lds[k * 3 + 1], r2 = lds[k * 3 + 2];
                const int x0 = (int)(lb & 15) - hf * 8, x1 = (int)((lb >> 4) & 15) - hf * 8;  // half-local
                const int y = (int)((lb >> 8) & 15) + (int)((e >> 8) & 15);
                area += (unsigned long long)(min(x1, 7) - max(x0, 0) + 1);
                const float yr = yrs[y];
                const float cy = fmaf(r1.w, yr, r2.x);
                const float ay = fmaf(r0.y, yr, r0.z);
                const float by = fmaf(r1.x, yr, r1.y);
                const unsigned long long idk = (unsigned long long)__float_as_uint(r2.w);
                unsigned long long *zrow = zb + y * ZS + hf * 8;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float xr = (NH > 1 && hf) ? xv[(8 + i) % T] : xv[i];
                    const float c = fmaf(r1.z, xr, cy);
                    const float au = fmaf(r0.x, xr, ay);
                    const float bv = fmaf(r0.w, xr, by);
                    // one predicate (bitwise &: no branch per condition)
                    const bool hit = (i >= x0) & (i <= x1) & (c > 0.f) & (fmaf(au, au, bv * bv) <= c * c) &
                                     (r2.y >= zn * c);
                    if (hit) {
                        const float z = r2.y * __builtin_amdgcn_rcpf(c);
                        const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | idk;
                        __hip_atomic_fetch_min(zrow + i, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
            __syncthreads();  // the group's hits are in the z-buffer
        }
    }
    // (the last group's barrier has put every hit in the z-buffer; each
    // thread reads back its own pixel)
    if (px < V.sW && py < V.sH) {
        const unsigned long long best = zb[zi];
        const int64_t p = V.s_off + (int64_t)py * V.sW + px;
        if (best == ~0ull) {
            sid[p] = -1;
            depth[p] = __int_as_float(0x7f800000);
        } else {
            const uint32_t id = (uint32_t)(best & 0xffffffffu);
            sid[p] = (int32_t)id;
            depth[p] = __uint_as_float((uint32_t)(best >> 32));
            unsigned char *vis = a.ws + a.L.svis + (int64_t)v * a.n;
            vis[id] = 1;
        }
    }
    return area;
}

// One block per raster tile, in the launch order of the surfel fill.
template <int T>
__global__ void __launch_bounds__(T * T) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_raster(FrameArgs a, int32_t *sid, float *depth) {
    const TileOrd o = reinterpret_cast<const TileOrd *>(a.ws + a.L.s_ord)[blockIdx.x];
    const unsigned long long area = raster_tile<T>(a, o, sid, depth);
    block_add_area<T * T>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->s_area, area);
}

// Persistent variant: a fixed number of blocks per CU take raster tiles from
// work queues until none is left.  Queue x holds the launch-order positions
// x, x + 8, x + 16, ... (each XCD starts on long tiles too); a block serves
// the queue of the XCD it runs on first, then the others in turn, taking
// kQueueChunk consecutive positions of a queue per claim (atomics on one
// address serialise: one claim per tile made the claims the kernel's
// critical path).  A queue is an atomic counter in the frame's header
// (zeroed by the surfel fill launch, which runs just before); a claim past a
// queue's end only leaves the counter above it.  Every block leaves the loop
// once all eight queues are exhausted.  The tile's work is the same code as
// above: the result does not depend on which block rasterises a tile.
constexpr int kQueueChunk = 4;

// First claim index of a chunk, its queue and its length (-1 when every
// queue is done).
__device__ inline int claim_raster_chunk(unsigned int *q, int n, int &x_out, int &len) {
    const int per = n >> 3, rem = n & 7;
    const int x0 = (int)counter_copy();
    for (int k = 0; k < 8; ++k) {
        const int x = (x0 + k) & 7;
        const unsigned int cnt = (unsigned int)(per + (x < rem ? 1 : 0));  // positions x + 8 i < n
        if (__hip_atomic_load(&q[x * kCounterStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= cnt) continue;
        const unsigned int i = atomicAdd(&q[x * kCounterStride], (unsigned int)kQueueChunk);
        if (i < cnt) {
            len = (int)min((unsigned int)kQueueChunk, cnt - i);
            x_out = x;
            return (int)i;
        }
    }
    len = 0;
    x_out = 0;
    return -1;
}

template <int T>
__global__ void __launch_bounds__(T * T) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_raster_queue(FrameArgs a, int32_t *sid, float *depth) {
    __shared__ int next, nq, nlen;
    unsigned int *q = reinterpret_cast<WsHeader *>(a.ws + a.L.header)->raster_q;
    const TileOrd *ord = reinterpret_cast<const TileOrd *>(a.ws + a.L.s_ord);
    unsigned long long area = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int x, len;
            next = claim_raster_chunk(q, a.L.rtiles, x, len);
            nq = x;
            nlen = len;
        }
        __syncthreads();
        const int i0 = next, x = nq, len = nlen;
        __syncthreads();  // every thread has read the claim before the next one
        if (i0 < 0) break;  // block-uniform
        for (int k = 0; k < len; ++k) {
            area += raster_tile<T>(a, ord[x + 8 * (i0 + k)], sid, depth);
            __syncthreads();  // the tile's last reads of its LDS are done
        }
    }
    block_add_area<T * T>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->s_area, area);
}

// ---------------------------------------------------------------------------
// colour of visible surfels (Eq. 1), then C_s per pixel and per-tile max D_s

// K (SH coefficients per channel) is a template argument so the 3K
// coefficient loads are unrolled and in flight together.
template <int K>
__global__ void __launch_bounds__(256) k_shade(FrameArgs a) {
    const int v = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = a.n;
    const bool vis = j < n && a.ws[a.L.svis + (int64_t)v * n + j];
    // visible surfels of the frame (every thread takes part in the block sum)
    block_add_area<256>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->s_visible, vis ? 1ull : 0ull);
    if (!vis) return;
    const ViewDev &V = a.views[v];
    float c[3][K];
    const float *sh = a.S.sh + j * (3 * K);  // [n][K][3]: this surfel's coefficients are one run
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) c[ch][k] = sh[k * 3 + ch];
    float dx = V.o[0] - a.S.mean[j], dy = V.o[1] - a.S.mean[n + j], dz = V.o[2] - a.S.mean[2 * n + j];
    const float dn = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= dn; dy *= dn; dz *= dn;
    float Y[K];
    sh_basis(dx, dy, dz, K, Y);
    float *scol = reinterpret_cast<float *>(a.ws + a.L.scol) + (int64_t)v * 3 * n;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc += c[ch][k] * Y[k];
        scol[ch * n + j] = fmaxf(acc, 0.f);
    }
}

// With 4 samples per pixel, C_s is the mean of the samples' colours (the
// background where a sample shows no surfel) and D_s the mean depth of the
// samples that hit a surfel (+inf if none): the 2x2 downsampling of the
// surfel pass rendered at twice the resolution.
template <int TW, int TH, int S>
__global__ void __launch_bounds__(TW * TH) k_resolve(FrameArgs a, const int32_t *sid, const float *sdepth,
                                                     float *depth, float *color_s) {
    constexpr int NT = TW * TH;
    __shared__ float red[NT / 64];
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int px = (lt % V.stx) * TW + (int)(threadIdx.x % TW);
    const int py = (lt / V.stx) * TH + (int)(threadIdx.x / TW);
    float dmax = -__int_as_float(0x7f800000);
    if (px < V.W && py < V.H) {
        const int64_t P = (int64_t)V.W * V.H;
        const int64_t lp = (int64_t)py * V.W + px;
        const float *scol = reinterpret_cast<const float *>(a.ws + a.L.scol) + (int64_t)v * 3 * a.n;
        float *cs = color_s + 3 * V.pix_off + lp;
        if (S == 1) {
            const int64_t p = V.pix_off + lp;
            const int id = sid[p];
            for (int ch = 0; ch < 3; ++ch) cs[ch * P] = id >= 0 ? scol[ch * a.n + id] : V.bg[ch];
            dmax = sdepth[p];
        } else {
            float c[3] = {0.f, 0.f, 0.f}, dsum = 0.f;
            int nh = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // (a, b) = (0,0), (1,0), (0,1), (1,1)
                const int64_t q = V.s_off + (int64_t)(2 * py + (k >> 1)) * V.sW + 2 * px + (k & 1);
                const int id = sid[q];
                for (int ch = 0; ch < 3; ++ch) c[ch] += id >= 0 ? scol[ch * a.n + id] : V.bg[ch];
                if (id >= 0) {
                    dsum += sdepth[q];
                    ++nh;
                }
            }
            for (int ch = 0; ch < 3; ++ch) cs[ch * P] = c[ch] * 0.25f;
            dmax = nh ? dsum / (float)nh : __int_as_float(0x7f800000);
            depth[V.pix_off + lp] = dmax;
        }
    }
    // block max of D_s
    for (int off = 32; off > 0; off >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mx = red[0];
        for (int k = 1; k < NT / 64; ++k) mx = fmaxf(mx, red[k]);
        reinterpret_cast<float *>(a.ws + a.L.tile_maxd)[t] = mx;
    }
}

// ---------------------------------------------------------------------------
// Gaussian binning with the conservative depth cull

// Count pass: per splat tile of the box, keep the tile iff the Gaussian's
// depth test can pass at one of its pixels (dme < the tile's largest D_s;
// the per-pixel test dme < D_s(x) implies it), take a list position with one
// atomic and keep it in the slot run (kNoSlot for a culled tile); the number
// of kept tiles goes to g_nkept (the backward's partials of a Gaussian are
// the first g_nkept places of its run, kept tiles in row order).  A Gaussian
// that keeps a tile then gets its colour (Eq. 1) for the list records: SH in
// the direction centre -> camera, plus 1/2, clamped at zero.  Its K x 3
// coefficients are one contiguous run ([m][K][3]); the wave loads the runs
// of its kept Gaussians into LDS a few at a time, consecutive lanes on
// consecutive words, so a load instruction covers whole runs.  K (SH
// coefficients per channel) is a template argument.
template <int K>
__global__ void __launch_bounds__(256) k_gauss_count(FrameArgs a) {
    constexpr int SK = 3 * K, RS = SK + 1;  // rows padded: distinct LDS banks per lane
    constexpr int R = 8;                    // kept Gaussians shaded per round
    __shared__ float rows[4][R * RS];
    __shared__ uint32_t ids[4][R];
    const int v = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    const ViewDev &V = a.views[v];
    const int64_t vi = (int64_t)v * a.m + i;
    bool kept = false;
    uint32_t nk = 0;
    int x0 = 1, y0 = 0, x1 = 0, y1 = 0;
    if (i < a.m) unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.gbox)[vi], x0, y0, x1, y1);
    if (x0 <= x1) {
        const float dme = a.G.dims == 2 ? reinterpret_cast<const G2Rec *>(a.ws + a.L.grec)[vi].dme
                                        : reinterpret_cast<const GRec *>(a.ws + a.L.grec)[vi].dme;
        const float *tmax = reinterpret_cast<const float *>(a.ws + a.L.tile_maxd);
        uint32_t *tcount = reinterpret_cast<uint32_t *>(a.ws + a.L.g_tcnt);
        uint32_t *slot = reinterpret_cast<uint32_t *>(a.ws + a.L.g_slot);
        const uint64_t base = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_boff)[vi];
        const uint64_t cap = (uint64_t)a.L.g_cap;
        const int TW = a.opt.splat_tile_w, TH = a.opt.splat_tile_h;
        TileWalk w(x0 / TW, y0 / TH, x1 / TW, y1 / TH, base, cap);
        const int t0 = V.st_off, tw = V.stx;  // in registers: no reload after each atomic
        for (int64_t i0 = 0; i0 < w.count; i0 += kWalkBatch) {
            int t[kWalkBatch];
            float dmax[kWalkBatch];
            uint32_t r[kWalkBatch];
#pragma unroll
            for (int b = 0; b < kWalkBatch; ++b)
                if (i0 + b < w.count) {
                    t[b] = t0 + w.ty * tw + w.tx;
                    dmax[b] = tmax[t[b]];
                    w.next();
                }
#pragma unroll
            for (int b = 0; b < kWalkBatch; ++b)
                if (i0 + b < w.count) {
                    const bool keep = dme < dmax[b];
                    r[b] = keep ? atomicAdd(&tcount[(int64_t)t[b] * kCounterStride], 1u) : kNoSlot;
                    kept |= keep;
                    nk += keep ? 1u : 0u;
                }
#pragma unroll
            for (int b = 0; b < kWalkBatch; ++b)
                if (i0 + b < w.count) slot[base + i0 + b] = r[b];
        }
        // the backward runs its chain rule only for Gaussians kept somewhere
        if (kept) reinterpret_cast<uint32_t *>(a.ws + a.L.g_act)[i] = 1u;
    }
    if (i < a.m) reinterpret_cast<uint32_t *>(a.ws + a.L.g_nkept)[vi] = nk;
    const unsigned long long km = __ballot((int)kept);
    const int total = __popcll(km);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    for (int r0 = 0; r0 < total; r0 += R) {  // wave-uniform
        const bool mine = kept && rank >= r0 && rank < r0 + R;
        if (mine) ids[wv][rank - r0] = (uint32_t)i;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int nr = min(R, total - r0);
        for (int c = lane; c < nr * SK; c += 64) {
            const int g = c / SK, q = c - g * SK;
            rows[wv][g * RS + q] = a.G.sh[(int64_t)ids[wv][g] * SK + q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (mine) {
            const float *c = &rows[wv][(rank - r0) * RS];
            const int64_t m = a.m;
            float dx = V.o[0] - a.G.mean[i], dy = V.o[1] - a.G.mean[m + i], dz = V.o[2] - a.G.mean[2 * m + i];
            const float dn = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
            dx *= dn; dy *= dn; dz *= dn;
            float Y[K];
            sh_basis(dx, dy, dz, K, Y);
            float col[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.5f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc += c[k * 3 + ch] * Y[k];
                col[ch] = fmaxf(acc, 0.f);
            }
            if (col[0] >= kColourMax || col[1] >= kColourMax || col[2] >= kColourMax)
                set_flag(reinterpret_cast<WsHeader *>(a.ws + a.L.header), kFlagColourRange);
            if (a.G.dims == 2) {
                G2Rec *rec = reinterpret_cast<G2Rec *>(a.ws + a.L.grec) + vi;
                rec->r = col[0] * kFixScale;
                rec->g = col[1] * kFixScale;
                rec->b = col[2] * kFixScale;
            } else {
                GRec *rec = reinterpret_cast<GRec *>(a.ws + a.L.grec) + vi;
                rec->r = col[0] * kFixScale;
                rec->g = col[1] * kFixScale;
                rec->b = col[2] * kFixScale;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // rows read before the next round writes
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Written four lanes to a 64-byte line, as in the surfel fill.
__global__ void __launch_bounds__(256) k_gauss_fill(FrameArgs a) {
    __shared__ float4 rec_l[4][64][3];   // per wave: each lane's record
    __shared__ uint32_t pos_l[4][64];    // per wave: compacted entries of one walk step
    __shared__ uint32_t k_l[4][64];      // their slot indices
    __shared__ uint32_t src_l[4][64];    // (lane | lbox << 8)
    __shared__ float4 col_l[4][64];      // 2D Gaussians: each lane's (dme, r, g, b)
    const int v = blockIdx.y;
    const bool g2 = a.G.dims == 2;
    const uint32_t *toff = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_toff);
    if (blockIdx.x == 0) {  // block-uniform: the splat's launch order, once
        if (blockIdx.y == 0)
            order_tile_pairs(a.views, a.n_views, toff, a.L.stiles, reinterpret_cast<TileOrd *>(a.ws + a.L.g_ord));
        return;
    }
    const int64_t i = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const ViewDev &V = a.views[v];
    const uint32_t *slot = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_slot);
    float4 *ents = reinterpret_cast<float4 *>(a.ws + a.L.g_ents);
    WsHeader *hdr = reinterpret_cast<WsHeader *>(a.ws + a.L.header);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const int TW = a.opt.splat_tile_w, TH = a.opt.splat_tile_h;
    int x0 = 1, y0 = 0, x1 = 0, y1 = 0;
    uint64_t base = 0;
    if (i < a.m) {
        const int64_t vi = (int64_t)v * a.m + i;
        unpack_box(reinterpret_cast<const uint2 *>(a.ws + a.L.gbox)[vi], x0, y0, x1, y1);
        const float4 *rec = reinterpret_cast<const float4 *>(a.ws + a.L.grec) + vi * (g2 ? 4 : 3);
        rec_l[wv][lane][0] = rec[0];
        rec_l[wv][lane][1] = rec[1];
        rec_l[wv][lane][2] = rec[2];
        if (g2) col_l[wv][lane] = rec[3];
        base = reinterpret_cast<const uint32_t *>(a.ws + a.L.g_boff)[vi];
    }
    TileWalk w(x0 / TW, y0 / TH, x1 / TW, y1 / TH, base, cap);
    const int64_t cnt = x0 > x1 ? 0 : w.count;
    if (x0 <= x1 && w.count < w.total) set_flag(hdr, kFlagGaussOverflow);
    const int t0 = V.st_off, tw = V.stx;
    uint32_t kr = 0;  // kept tiles so far: the entry's partial goes to place base + kr
    float *part = reinterpret_cast<float *>(a.ws + a.L.g_part);
    for (int64_t i0 = 0; __any((int)(i0 < cnt)); i0 += kWalkBatch) {
        uint32_t sl[kWalkBatch], to[kWalkBatch], lb[kWalkBatch];
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b)  // the batch's loads in flight together
            if (i0 + b < cnt) {
                sl[b] = slot[base + i0 + b];
                to[b] = toff[t0 + w.ty * tw + w.tx];
                lb[b] = pack_lbox(x0, y0, x1, y1, w.tx * TW, w.ty * TH, TW, TH);
                w.next();
            }
#pragma unroll
        for (int b = 0; b < kWalkBatch; ++b) {
            bool keep = false;
            uint64_t pos = 0;
            const uint64_t k = base + kr;  // base + kr <= base + i0 + b < cap
            if (i0 + b < cnt && sl[b] != kNoSlot) {
                ++kr;
                pos = (uint64_t)to[b] + sl[b];
                keep = pos < cap;
                if (!keep) {  // lost to an overflow: its partial reads zero in the backward
                    set_flag(hdr, kFlagGaussOverflow);
#pragma unroll
                    for (int c = 0; c < kGaussPartials; ++c) part[k * kGaussPartials + c] = 0.f;
                }
            }
            const unsigned long long m = __ballot((int)keep);
            if (m == 0ull) continue;  // wave-uniform
            const int total = __popcll(m);
            if (keep) {
                const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                pos_l[wv][r] = (uint32_t)pos;  // pos < cap < 2^31
                k_l[wv][r] = (uint32_t)k;
                src_l[wv][r] = (uint32_t)lane | (lb[b] << 8);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int e0 = 0; e0 < total; e0 += 16) {
                const int e = e0 + (lane >> 2), q = lane & 3;
                if (e < total) {
                    const uint32_t sv = src_l[wv][e];
                    // the Gaussian's record, the place of the backward
                    // partial of this entry, its box inside the tile and
                    // its index
                    const uint32_t gi = (uint32_t)((blockIdx.x - 1) * blockDim.x + wv * 64) + (sv & 63u);
                    float4 val;
                    if (q < 3) {
                        val = rec_l[wv][sv & 63u][q];
                    } else if (g2) {  // 2D: the colour around the box (G2Ent)
                        const float4 c4 = col_l[wv][sv & 63u];
                        val = make_float4(c4.y, __uint_as_float(sv >> 8), c4.z, c4.w);
                    } else {
                        val = make_float4(__uint_as_float(k_l[wv][e]), __uint_as_float(sv >> 8), __uint_as_float(gi),
                                          0.f);
                    }
                    ents[(uint64_t)pos_l[wv][e] * 4 + q] = val;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");  // reads done before the next step's writes
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// ---------------------------------------------------------------------------
// pass 2: order-independent accumulation (fixed point) + composite

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_splat(FrameArgs a, const float *depth, const float *color_s,
                                                   float *image, float *accum) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64, RW = 64 / TW;  // waves; tile rows per wave
    __shared__ GRec lds[NT];
    __shared__ uint8_t ovl[NT];       // per entry: bit w = its box meets wave w's rows
    __shared__ uint8_t wl[NW][NT];    // per wave: the entries that meet its rows
    // this block's tile and list bounds, in the launch order of the Gaussian fill
    const TileOrd o = reinterpret_cast<const TileOrd *>(a.ws + a.L.g_ord)[blockIdx.x];
    const int t = (int)o.tile;
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int px = (lt % V.stx) * TW + (int)(threadIdx.x % TW);
    const int py = (lt / V.stx) * TH + (int)(threadIdx.x / TW);
    const bool inside = px < V.W && py < V.H;
    const int64_t lp = (int64_t)py * V.W + px;
    const int64_t P = (int64_t)V.W * V.H;
    const float ds = inside ? depth[V.pix_off + lp] : -__int_as_float(0x7f800000);
    // the surfel colour is needed only at the end: loaded now, in flight
    // with the list loads instead of after the loop
    const float *cs = color_s + 3 * V.pix_off + lp;
    const float cs0 = inside ? cs[0] : 0.f, cs1 = inside ? cs[P] : 0.f, cs2 = inside ? cs[2 * P] : 0.f;
    const float xf = (float)px + 0.5f, yf = (float)py + 0.5f;
    const float amin = a.opt.alpha_min;

    const GEnt *ents = reinterpret_cast<const GEnt *>(a.ws + a.L.g_ents);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);

    long long acc_r = 0, acc_g = 0, acc_b = 0, acc_w = 0;
    unsigned long long area = 0;  // pixels of this thread's entries' boxes
    for (uint64_t base = b0; base < b1; base += NT) {
        const int cnt = (int)umin64((uint64_t)NT, b1 - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const GEnt &e = ents[base + threadIdx.x];
            lds[threadIdx.x] = e.g;
            const uint32_t lb = e.lbox;
            area += (unsigned long long)(((lb >> 4) & 15) - (lb & 15) + 1) * (((lb >> 12) & 15) - ((lb >> 8) & 15) + 1);
            // a kept alpha lies inside the entry's box: waves whose rows the
            // box misses can skip the entry
            const int r0 = (int)((lb >> 8) & 15), r1 = (int)((lb >> 12) & 15);
            uint32_t bits = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) bits |= (uint32_t)(r1 >= w * RW && r0 <= w * RW + RW - 1) << w;
            ovl[threadIdx.x] = (uint8_t)bits;
        }
        __syncthreads();
        // this wave's entries, in list order (ballot + rank; wave-local)
        const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63);
        int nw = 0;
        for (int c = 0; c < cnt; c += 64) {
            const int e = c + ln;
            const bool in = e < cnt && ((ovl[e] >> wv) & 1);
            const unsigned long long bm = __ballot((int)in);
            if (in) wl[wv][nw + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))] = (uint8_t)e;
            nw += __popcll(bm);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int kk = 0; kk < nw; ++kk) {
            const GRec g = lds[wl[wv][kk]];
            float dx, dy, q;
            const float al = gauss_alpha(g, xf, yf, dx, dy, q);
            if ((al >= amin) & (g.dme < ds)) {  // one predicate, no branch per condition
                acc_r += (long long)__float2int_rn(al * g.r);
                acc_g += (long long)__float2int_rn(al * g.g);
                acc_b += (long long)__float2int_rn(al * g.b);
                acc_w += (long long)__float2int_rn(al * kFixScale);
            }
        }
    }
    block_add_area<NT>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->g_area, area);
    if (inside) {
        const float cgr = (float)((double)acc_r * kFixInv);
        const float cgg = (float)((double)acc_g * kFixInv);
        const float cgb = (float)((double)acc_b * kFixInv);
        const float wg = (float)((double)acc_w * kFixInv);
        const float ws = a.opt.w_s;
        const float inv = 1.f / (ws + wg);
        float *img = image + 3 * V.pix_off + lp;
        img[0] = (ws * cs0 + cgr) * inv;
        img[P] = (ws * cs1 + cgg) * inv;
        img[2 * P] = (ws * cs2 + cgb) * inv;
        float *ac = accum + 4 * V.pix_off + lp;
        ac[0] = cgr;
        ac[P] = cgg;
        ac[2 * P] = cgb;
        ac[3 * P] = wg;
    }
}

// Pass 2 with 2D Gaussians (2D-GES, Sec. 6.4): as k_splat, each entry
// tested at the pixel's camera ray (g2_eval: the plane hit, alpha, the
// planar depth against D_s + eps) and summed in the same fixed point.
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_splat2d(FrameArgs a, const float *depth, const float *color_s,
                                                     float *image, float *accum) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64, RW = 64 / TW;  // waves; tile rows per wave
    __shared__ G2Ent lds[NT];
    __shared__ uint8_t ovl[NT];
    __shared__ uint8_t wl[NW][NT];
    const TileOrd o = reinterpret_cast<const TileOrd *>(a.ws + a.L.g_ord)[blockIdx.x];
    const int t = (int)o.tile;
    const int v = view_of_stile(a.views, a.n_views, t);
    const ViewDev &V = a.views[v];
    const int lt = t - V.st_off;
    const int px = (lt % V.stx) * TW + (int)(threadIdx.x % TW);
    const int py = (lt / V.stx) * TH + (int)(threadIdx.x / TW);
    const bool inside = px < V.W && py < V.H;
    const int64_t lp = (int64_t)py * V.W + px;
    const int64_t P = (int64_t)V.W * V.H;
    const float ds = inside ? depth[V.pix_off + lp] : -__int_as_float(0x7f800000);
    const float *cs = color_s + 3 * V.pix_off + lp;
    const float cs0 = inside ? cs[0] : 0.f, cs1 = inside ? cs[P] : 0.f, cs2 = inside ? cs[2 * P] : 0.f;
    const float xr = ((float)px + 0.5f - V.cx) / V.fx, yr = ((float)py + 0.5f - V.cy) / V.fy;
    const float amin = a.opt.alpha_min, zn = V.znear;

    const G2Ent *ents = reinterpret_cast<const G2Ent *>(a.ws + a.L.g_ents);
    const uint64_t cap = (uint64_t)a.L.g_cap;
    const uint64_t b0 = umin64((uint64_t)o.b0, cap), b1 = umin64((uint64_t)o.b1, cap);

    long long acc_r = 0, acc_g = 0, acc_b = 0, acc_w = 0;
    unsigned long long area = 0;
    for (uint64_t base = b0; base < b1; base += NT) {
        const int cnt = (int)umin64((uint64_t)NT, b1 - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const G2Ent &e = ents[base + threadIdx.x];
            lds[threadIdx.x] = e;
            const uint32_t lb = e.lbox;
            area += (unsigned long long)(((lb >> 4) & 15) - (lb & 15) + 1) * (((lb >> 12) & 15) - ((lb >> 8) & 15) + 1);
            const int r0 = (int)((lb >> 8) & 15), r1 = (int)((lb >> 12) & 15);
            uint32_t bits = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) bits |= (uint32_t)(r1 >= w * RW && r0 <= w * RW + RW - 1) << w;
            ovl[threadIdx.x] = (uint8_t)bits;
        }
        __syncthreads();
        const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63);
        int nw = 0;
        for (int c = 0; c < cnt; c += 64) {
            const int e = c + ln;
            const bool in = e < cnt && ((ovl[e] >> wv) & 1);
            const unsigned long long bm = __ballot((int)in);
            if (in) wl[wv][nw + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))] = (uint8_t)e;
            nw += __popcll(bm);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int kk = 0; kk < nw; ++kk) {
            const G2Ent &e = lds[wl[wv][kk]];
            float al, z;
            if (g2_eval(e, xr, yr, zn, amin, ds, al, z)) {
                acc_r += (long long)__float2int_rn(al * e.r);
                acc_g += (long long)__float2int_rn(al * e.g);
                acc_b += (long long)__float2int_rn(al * e.b);
                acc_w += (long long)__float2int_rn(al * kFixScale);
            }
        }
    }
    block_add_area<NT>(reinterpret_cast<WsHeader *>(a.ws + a.L.header)->g_area, area);
    if (inside) {
        const float cgr = (float)((double)acc_r * kFixInv);
        const float cgg = (float)((double)acc_g * kFixInv);
        const float cgb = (float)((double)acc_b * kFixInv);
        const float wg = (float)((double)acc_w * kFixInv);
        const float ws = a.opt.w_s;
        const float inv = 1.f / (ws + wg);
        float *img = image + 3 * V.pix_off + lp;
        img[0] = (ws * cs0 + cgr) * inv;
        img[P] = (ws * cs1 + cgg) * inv;
        img[2 * P] = (ws * cs2 + cgb) * inv;
        float *ac = accum + 4 * V.pix_off + lp;
        ac[0] = cgr;
        ac[P] = cgg;
        ac[2 * P] = cgb;
        ac[3 * P] = wg;
    }
}

inline dim3 prim_grid(int64_t count, int n_views) {
    return dim3((unsigned)((count + 255) / 256), (unsigned)n_views);
}

// the fill launches: block x = 0 of view 0 orders the tiles, x >= 1 fill
inline dim3 fill_grid(int64_t count, int n_views) {
    return dim3((unsigned)((count + 255) / 256 + 1), (unsigned)n_views);
}

}  // namespace

hipError_t launch_project(const FrameArgs &a, hipStream_t s) {
    const int gblocks = (int)((a.m + 255) / 256), sblocks = (int)((a.n + 255) / 256);
    if (gblocks + sblocks == 0) return hipSuccess;
    const dim3 g((unsigned)(gblocks + sblocks), (unsigned)a.n_views);
    if (a.G.dims == 2) hipLaunchKernelGGL((k_project<true, false>), g, dim3(256), 0, s, a, gblocks);
    else if (a.translucent) hipLaunchKernelGGL((k_project<false, true>), g, dim3(256), 0, s, a, gblocks);
    else hipLaunchKernelGGL((k_project<false, false>), g, dim3(256), 0, s, a, gblocks);
    return hipGetLastError();
}

hipError_t launch_surfel_count(const FrameArgs &a, hipStream_t s) {
    if (a.n > 0) hipLaunchKernelGGL(k_surfel_count, prim_grid(a.n, a.n_views), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_surfel_fill(const FrameArgs &a, hipStream_t s) {
    // launched with no surfels too: the raster needs the launch order
    if (a.translucent) hipLaunchKernelGGL(k_surfel_fill<true>, fill_grid(a.n, a.n_views), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_surfel_fill<false>, fill_grid(a.n, a.n_views), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_raster(const FrameArgs &a, int32_t *sid, float *depth, int cus, hipStream_t s) {
    const int k = a.opt.tile_queue;
    if (k > 0 && a.n > 0) {
        // persistent: k blocks per CU (no more than there are tiles)
        const int64_t blocks = (int64_t)k * cus < a.L.rtiles ? (int64_t)k * cus : a.L.rtiles;
        const dim3 grid((unsigned)(blocks > 0 ? blocks : 1));
        if (a.opt.raster_tile == 8) hipLaunchKernelGGL(k_raster_queue<8>, grid, dim3(64), 0, s, a, sid, depth);
        else hipLaunchKernelGGL(k_raster_queue<16>, grid, dim3(256), 0, s, a, sid, depth);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)a.L.rtiles);
    if (a.opt.raster_tile == 8) hipLaunchKernelGGL(k_raster<8>, grid, dim3(64), 0, s, a, sid, depth);
    else hipLaunchKernelGGL(k_raster<16>, grid, dim3(256), 0, s, a, sid, depth);
    return hipGetLastError();
}

hipError_t launch_shade(const FrameArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    const dim3 g = prim_grid(a.n, a.n_views);
    switch (a.ks) {
        case 1: hipLaunchKernelGGL(k_shade<1>, g, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_shade<4>, g, dim3(256), 0, s, a); break;
        case 9: hipLaunchKernelGGL(k_shade<9>, g, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_shade<16>, g, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

template <int S>
static void resolve_shape(const FrameArgs &a, const int32_t *sid, const float *sdepth, float *depth, float *color_s,
                          hipStream_t s) {
    const dim3 grid((unsigned)a.L.stiles);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_resolve<8, 8, S>), grid, dim3(64), 0, s, a, sid, sdepth, depth, color_s);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_resolve<16, 8, S>), grid, dim3(128), 0, s, a, sid, sdepth, depth, color_s);
    else
        hipLaunchKernelGGL((k_resolve<16, 16, S>), grid, dim3(256), 0, s, a, sid, sdepth, depth, color_s);
}

hipError_t launch_resolve(const FrameArgs &a, const int32_t *sid, const float *sdepth, float *depth, float *color_s,
                          hipStream_t s) {
    if (a.opt.surfel_samples == 4) resolve_shape<4>(a, sid, sdepth, depth, color_s, s);
    else resolve_shape<1>(a, sid, sdepth, depth, color_s, s);
    return hipGetLastError();
}

hipError_t launch_gauss_count(const FrameArgs &a, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    const dim3 g = prim_grid(a.m, a.n_views);
    switch (a.kg) {
        case 1: hipLaunchKernelGGL(k_gauss_count<1>, g, dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_gauss_count<4>, g, dim3(256), 0, s, a); break;
        case 9: hipLaunchKernelGGL(k_gauss_count<9>, g, dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL(k_gauss_count<16>, g, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_gauss_fill(const FrameArgs &a, hipStream_t s) {
    // launched with no Gaussians too: the splat needs the launch order
    hipLaunchKernelGGL(k_gauss_fill, fill_grid(a.m, a.n_views), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_splat(const FrameArgs &a, const float *depth, const float *color_s, float *image, float *accum,
                        hipStream_t s) {
    const dim3 grid((unsigned)a.L.stiles);
    const int tw = a.opt.splat_tile_w, th = a.opt.splat_tile_h;
    if (a.G.dims == 2) {
        if (tw == 8 && th == 8)
            hipLaunchKernelGGL((k_splat2d<8, 8>), grid, dim3(64), 0, s, a, depth, color_s, image, accum);
        else if (tw == 16 && th == 8)
            hipLaunchKernelGGL((k_splat2d<16, 8>), grid, dim3(128), 0, s, a, depth, color_s, image, accum);
        else
            hipLaunchKernelGGL((k_splat2d<16, 16>), grid, dim3(256), 0, s, a, depth, color_s, image, accum);
        return hipGetLastError();
    }
    if (tw == 8 && th == 8)
        hipLaunchKernelGGL((k_splat<8, 8>), grid, dim3(64), 0, s, a, depth, color_s, image, accum);
    else if (tw == 16 && th == 8)
        hipLaunchKernelGGL((k_splat<16, 8>), grid, dim3(128), 0, s, a, depth, color_s, image, accum);
    else
        hipLaunchKernelGGL((k_splat<16, 16>), grid, dim3(256), 0, s, a, depth, color_s, image, accum);
    return hipGetLastError();
}

}  // namespace ges
