// Size of the Mip-GES world-space filter (Sec. 6.1, after Mip-Splatting):
// per Gaussian, scale2 times the squared world size of a pixel of the
// finest camera that sees it, (z / f_x)^2 minimised over the cameras whose
// image [0, W] x [0, H] holds the projected centre with z > znear; 0 when no
// camera sees it.  Cameras go to the kernel by value, kMipCams per launch;
// the running minimum of z / f_x is kept in the output between launches.
#include "ges_internal.h"

namespace ges {

namespace {

__global__ void __launch_bounds__(256) k_mip_min(const float *mean, int64_t m, MipCams c, int first, float *best) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float px = mean[i], py = mean[m + i], pz = mean[2 * m + i];
    float b = first ? __int_as_float(0x7f800000) : best[i];
    for (int k = 0; k < c.n; ++k) {
        const float *R = c.R[k];
        const float x = R[0] * px + R[1] * py + R[2] * pz + c.t[k][0];
        const float y = R[3] * px + R[4] * py + R[5] * pz + c.t[k][1];
        const float z = R[6] * px + R[7] * py + R[8] * pz + c.t[k][2];
        if (!(z > c.znear[k])) continue;
        const float u = c.fx[k] * x / z + c.cx[k], w = c.fy[k] * y / z + c.cy[k];
        if (u >= 0.f && u <= c.W[k] && w >= 0.f && w <= c.H[k]) b = fminf(b, z / c.fx[k]);
    }
    best[i] = b;
}

__global__ void __launch_bounds__(256) k_mip_var(int64_t m, float scale2, float *best) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float b = best[i];
    best[i] = isfinite(b) ? scale2 * b * b : 0.f;
}

}  // namespace

hipError_t launch_mip_filter3d(const float *mean, int64_t m, const ges_camera *cams, int n_views, float scale2,
                               float *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const dim3 grid((unsigned)((m + 255) / 256));
    for (int v0 = 0; v0 < n_views; v0 += kMipCams) {
        MipCams c{};
        c.n = n_views - v0 < kMipCams ? n_views - v0 : kMipCams;
        for (int k = 0; k < c.n; ++k) {
            const ges_camera &cam = cams[v0 + k];
            for (int e = 0; e < 9; ++e) c.R[k][e] = cam.R[e];
            for (int e = 0; e < 3; ++e) c.t[k][e] = cam.t[e];
            c.fx[k] = cam.fx; c.fy[k] = cam.fy; c.cx[k] = cam.cx; c.cy[k] = cam.cy;
            c.W[k] = (float)cam.width; c.H[k] = (float)cam.height; c.znear[k] = cam.znear;
        }
        hipLaunchKernelGGL(k_mip_min, grid, dim3(256), 0, s, mean, m, c, v0 == 0 ? 1 : 0, out);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mip_var, grid, dim3(256), 0, s, m, scale2, out);
    return hipGetLastError();
}

}  // namespace ges
