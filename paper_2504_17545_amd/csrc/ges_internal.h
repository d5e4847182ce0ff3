// Internal declarations of the GES render library: device-side view table,
// per-primitive record layouts, workspace layout, device math shared by the
// forward and backward kernels, and the host-side launchers each kernel
// translation unit exports to the API layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ges.h"

namespace ges {

constexpr int kMaxViews = 1024;
constexpr float kFixScale = 16777216.0f;      // 2^24: fixed-point unit of C_G, W_G
constexpr double kFixInv = 1.0 / 16777216.0;
constexpr float kColourMax = 127.0f;          // c * 2^24 must stay below 2^31

// Flags in WsHeader::flags.
constexpr uint32_t kFlagSurfelOverflow = 1u;
constexpr uint32_t kFlagGaussOverflow = 2u;
constexpr uint32_t kFlagColourRange = 4u;
constexpr uint32_t kFlagSortOverflow = 8u;  // a tile's list exceeds the translucent blend's sort capacity

// One camera as the kernels see it (copied into the workspace by ges_project).
struct ViewDev {
    int W, H;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
    float bg[3];
    float o[3];          // camera centre in world space, -R^T t
    float limx, limy;    // 1.3 * half field of view (tangent) for the EWA clamp
    int rtx, rty;        // raster tiles along x, y
    int stx, sty;        // splat tiles along x, y
    int rt_off, st_off;  // first raster / splat tile of this view (flattened)
    long long pix_off;   // first pixel of this view in concatenated outputs
    // the surfel pass's sample grid: the image itself, or with 4 samples per
    // pixel the image at twice the resolution (sample (a, b) of pixel (i, j)
    // is grid point (2i + a, 2j + b)); raster tiles cover this grid
    int sW, sH;
    float sfx, sfy, scx, scy;
    long long s_off;     // first sample of this view in concatenated sample buffers
};

constexpr int kAreaSlots = 64;

struct WsHeader {
    uint32_t flags;
    uint32_t pad;
    unsigned long long s_pairs;  // (surfel, raster tile) list entries needed
    unsigned long long g_pairs;  // (Gaussian, splat tile) list entries needed
    unsigned long long s_slots;  // raster tiles inside all surfel boxes
    unsigned long long g_slots;  // splat tiles inside all Gaussian boxes
    unsigned long long g_active; // Gaussians with a list entry in some view
    unsigned long long pad2[2];
    // box-pixel totals of the surfel / Gaussian entries, spread over
    // kAreaSlots counters one 128-B line apart (one block adds to one of
    // them) so that the adds do not serialise on one address
    unsigned long long s_area[kAreaSlots * 16];
    unsigned long long g_area[kAreaSlots * 16];
    unsigned long long s_visible[kAreaSlots * 16];  // (view, surfel) pairs that won a pixel
    // work queues of the persistent raster: one counter per XCD, one 128-B
    // line each (indexed x * kCounterStride)
    unsigned int raster_q[8 * 32];
};

// Slot value of a tile the depth cull removed from a Gaussian's box.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr int kGaussPartials = 9;  // per Gaussian list entry: sigma, p_hat x/y, conic a/b/c, colour r/g/b
constexpr int kTPartials = 13;     // per translucent surfel entry: dL/dU (3), dL/dV (3), dL/dn (3), dL/dw_mod, dL/dc (3)

// Per-tile list counters are taken with device-scope atomics; the atomics on
// one cache line serialise, so each counter gets a 128-byte line of its own.
constexpr int kCounterStride = 32;

// Surfel tile lists are counted in kCounterCopies copies per tile, one per
// XCD (the block's accelerator complex, masked to 3 bits), so that an XCD's
// atomics touch lines no other XCD touches.  The copies of a tile are
// adjacent in the scan, so its list is their sub-lists back to back; which
// copy a block uses changes only the order inside the list.  A slot holds
// copy << kCopyShift | position in that copy's sub-list.
constexpr int kCounterCopies = 8;
constexpr int kCopyShift = 29;
constexpr uint32_t kCopyPosMask = (1u << kCopyShift) - 1;
__device__ __forceinline__ uint32_t counter_copy() {
    return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | 20) & (kCounterCopies - 1);  // hwreg XCC_ID[3:0]
}

// Per-(view, Gaussian) projected record, 12 floats, AoS so that a gather by
// Gaussian index reads one 48-byte run.
struct alignas(16) GRec {
    float px, py;        // projected centre p_hat (pixels)
    float ca, cb, cc;    // conic: q = ca dx^2 + 2 cb dx dy + cc dy^2
    float lsig;          // log2(sigma)
    float dme;           // centre depth minus eps (the test is dme < D_s)
    float r, g, b;       // colour * 2^24 (fixed-point scale folded in)
    float sigma;
    float depth;
};
static_assert(sizeof(GRec) == 48, "GRec must be 48 bytes");

// Per-(view, surfel) raster record, 12 floats.  With the camera ray
// r = (x', y', 1) of a pixel: hit iff c = n.r > 0, (U.r)^2 + (V.r)^2 <= c^2
// and w >= znear c; the hit depth is w / c.  U, V are the disc's scaled
// in-plane axes folded with the plane offset (see surfel set-up).
struct alignas(16) SRec {
    float Ux, Uy, Uz;
    float Vx, Vy, Vz;
    float nx, ny, nz;
    float w;             // n . mu  (>= 0: the normal is flipped to face the camera)
    float zmin;          // smallest camera z over the disc (lowered: no FP32 hit is nearer)
    float zmax;          // largest camera z over the disc (raised: no FP32 hit is farther)
};
static_assert(sizeof(SRec) == 48, "SRec must be 48 bytes");

// Tile list entries are whole 64-byte records: the fill pass writes one
// aligned line per (primitive, tile) -- the primitive's record with the
// entry's bookkeeping -- and a tile kernel streams its list with coalesced
// loads instead of gathering records by primitive index.
struct alignas(64) SEnt {
    float4 r0, r1, r2;   // SRec (U, V, n, w, zmin) with r2.w = the surfel index bits
    uint32_t lbox;       // box inside the tile (pack_lbox)
    uint32_t pad[3];
};
static_assert(sizeof(SEnt) == 64, "SEnt must be 64 bytes");

struct alignas(64) GEnt {
    GRec g;
    uint32_t slot;       // slot index: where the backward partial of this entry goes
    uint32_t lbox;       // box inside the tile (pack_lbox)
    uint32_t gauss;      // index of the Gaussian (the pruning scores reduce per Gaussian)
    uint32_t pad;
};
static_assert(sizeof(GEnt) == 64, "GEnt must be 64 bytes");
static_assert(offsetof(GEnt, slot) == 48 && offsetof(GEnt, lbox) == 52, "GEnt is read as four 16-byte words");

// Per-(view, 2D Gaussian) record of 2D-GES (Sec. 6.4): the splat's plane
// folded like a surfel's disc (SRec) but in units of its scales, so that
// with the camera ray r = (x', y', 1): c = n.r, u = U.r / c, v = V.r / c are
// the hit point's scaled local coordinates and w / c its planar depth.  The
// first 48 bytes are the list entry's record; dme (the smallest depth of the
// alpha >= alpha_min disc minus eps) feeds the binning's depth cull and the
// colour is set by the count pass.
struct alignas(16) G2Rec {
    float Ux, Uy, Uz;
    float Vx, Vy, Vz;
    float nx, ny, nz;
    float w;             // n . mu >= 0 (n turned away from the camera)
    float sigma;         // maximum opacity
    float eps;           // depth offset (5/2)(s_u + s_v), or the constant
    float dme;
    float r, g, b;       // colour * 2^24
};
static_assert(sizeof(G2Rec) == 64, "G2Rec must be 64 bytes");

// List entry of a 2D Gaussian: the record's first 48 bytes, the colour in
// the words a 3D entry uses for its slot, index and padding (2D Gaussians
// have no backward here), the box where every entry has it.
struct alignas(64) G2Ent {
    float Ux, Uy, Uz, Vx, Vy, Vz, nx, ny, nz, w, sigma, eps;
    float r;
    uint32_t lbox;
    float g, b;
};
static_assert(sizeof(G2Ent) == 64 && offsetof(G2Ent, lbox) == offsetof(GEnt, lbox), "G2Ent shares GEnt's box word");

// One tile of a tile pass's launch order, with its list bounds (unclamped
// scan offsets).  The passes run their tiles longest list first: the fill
// launch that precedes them sorts the tiles into classes by the bit length
// of their list length (the classes from the longest down, the tiles of a
// class in any order), so that the few tiles with several times the mean
// work start at the beginning of the launch instead of wherever they fall in
// the image.  Every tile's result is computed independently of the others,
// so the order changes only when a tile runs, never what it writes.
struct alignas(16) TileOrd {
    uint32_t tile, b0, b1, pad;
};
constexpr int kOrdClasses = 16;
__device__ __forceinline__ int ord_class(uint32_t len) {
    const int bits = len ? 32 - __builtin_clz(len) : 0;
    return bits < kOrdClasses - 1 ? bits : kOrdClasses - 1;
}

// Inclusive pixel bounding box packed as {x0 | y0 << 16, x1 | y1 << 16};
// empty when x0 > x1.
__host__ __device__ inline uint2 pack_box(int x0, int y0, int x1, int y1) {
    return make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
}
__host__ __device__ inline void unpack_box(uint2 b, int &x0, int &y0, int &x1, int &y1) {
    x0 = (int)(b.x & 0xFFFFu);
    y0 = (int)(b.x >> 16);
    x1 = (int)(b.y & 0xFFFFu);
    y1 = (int)(b.y >> 16);
}
constexpr uint32_t kEmptyBoxX = 0xFFFFu;  // x0 = 65535 > any x1

// A list entry's box inside its tile (tile-local, inclusive, tiles <= 16
// pixels wide/high): x0 | x1 << 4 | y0 << 8 | y1 << 12.
__device__ inline uint16_t pack_lbox(int x0, int y0, int x1, int y1, int tx0, int ty0, int TW, int TH) {
    const int a = max(x0 - tx0, 0), b = min(x1 - tx0, TW - 1);
    const int c = max(y0 - ty0, 0), d = min(y1 - ty0, TH - 1);
    return (uint16_t)(a | (b << 4) | (c << 8) | (d << 12));
}

// Tile of a tile kernel's block.  The dispatcher hands workgroups to the 8
// XCDs in turn (block b to XCD b % 8), and each XCD has its own L2; a tile
// row of a per-pixel float plane (8 or 16 pixels) is half a 128-byte line
// or less, shared with the neighbouring tile.  Giving each XCD a contiguous
// run of tiles keeps neighbours on one L2 and in dispatch order, so a line
// is fetched once instead of once per XCD.  A bijection of [0, n): only the
// traffic depends on it.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, s = b >> 3;
    const int per = n >> 3, rem = n & 7;  // XCD x takes per + (x < rem) tiles
    return x * per + min(x, rem) + s;
}

// Wave-wide reductions and scans of the device library (DPP row operations,
// no LDS round trip per step); every lane of the wave must be active.
extern "C" __device__ int __ockl_wfscan_add_i32(int, bool);
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) { return __ockl_wfred_min_u32(v); }
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) { return __ockl_wfred_max_u32(v); }
__device__ __forceinline__ int wave_scan_add(int v, bool inclusive) { return __ockl_wfscan_add_i32(v, inclusive); }

// Sum of v over a block of NT threads (a multiple of 64, at most 256), added
// by one thread to the block's counter of a spread set (every thread of the
// block must call).
template <int NT>
__device__ inline void block_add_area(unsigned long long *spread, unsigned long long v) {
    __shared__ unsigned long long part[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) t += part[w];
        if (t) atomicAdd(&spread[(blockIdx.x % kAreaSlots) * 16], t);
    }
}

// Row-order walk over the tiles [tx0, tx1] x [ty0, ty1] of a primitive's
// box, matching its slot run base, base + 1, ...; count stops at the slot
// capacity (total is the full tile count).  Count, fill and the backward
// walk boxes in batches of kWalkBatch so that a batch's memory operations
// are in flight together.
constexpr int kWalkBatch = 8;
// Surfels whose box spans more raster tiles than this skip the occluder test
// (a bound on the projection's work; fewer occluders only cull less).
constexpr int kOccluderTiles = 64;
struct TileWalk {
    int tx0, tx1, tx, ty;
    int64_t total, count;
    __device__ TileWalk(int tx0_, int ty0, int tx1_, int ty1, uint64_t base, uint64_t cap)
        : tx0(tx0_), tx1(tx1_), tx(tx0_), ty(ty0) {
        total = (int64_t)(tx1_ - tx0_ + 1) * (ty1 - ty0 + 1);
        const int64_t room = base < cap ? (int64_t)(cap - base) : 0;
        count = total < room ? total : room;
    }
    __device__ void next() {
        if (++tx > tx1) {
            tx = tx0;
            ++ty;
        }
    }
};

// Workspace layout: byte offsets of every region, computed on the host.
//
// Binning (both primitive kinds): the projection writes each primitive's
// pixel box and the number of tiles in it (nt); an exclusive scan of nt gives
// each primitive a run of "slots" (boff).  The count pass walks the box's
// tiles in row order and stores, per tile, the position atomically taken in
// that tile's list (or kNoSlot if culled); a scan of the per-tile counts gives
// the list offsets (toff) and the fill pass writes list[toff[t] + slot]
// without atomics.  The backward walks the same boxes in the same order and
// finds every entry of a primitive at toff[t] + slot: a fixed-order back-map.
struct WsLayout {
    size_t header, views;
    size_t grec, gbox, g_boff;            // per (view, Gaussian); g_boff: nt, scanned
    size_t srec, sbox, s_boff, s_zmin;    // per (view, surfel); s_zmin: the record's zmin alone
    size_t svis, scol;                    // per (view, surfel)
    size_t s_tcnt, s_toff, s_tocc;        // per raster tile: strided counters; offsets (+1); occluder depth
    size_t g_tcnt, g_toff, tile_maxd;     // per splat tile
    size_t s_ord, g_ord;                  // launch order of the raster / splat tiles (TileOrd)
    size_t s_ents, s_slot;                // surfel list entries (SEnt) / per-slot list positions
    size_t g_ents, g_slot;                // Gaussian list entries (GEnt) / per-slot list positions
    size_t g_nkept;                       // per (view, Gaussian): tiles kept by the depth cull
    size_t g_act, g_aoff, g_alist;        // per Gaussian: active flag (set by the forward); its
                                          // exclusive scan (m + 1, written by each backward); active list
    size_t g_part;                        // 9 floats per Gaussian slot, [slot][9]
    size_t s_part;                        // 3 floats per surfel slot, [slot][3]
    size_t scan_tmp, scan_tmp2;           // block sums of the scans (two scans can share launches)
    size_t s_cnt;                         // per surfel: pixel count of one view (pruning scores)
    size_t s_depth;                       // per sample: hit depth (4 samples per pixel only)
    size_t t_sorted;                      // translucent: per list position, the blend order (list positions)
    size_t t_state;                       // translucent: per pixel T before the last blended entry, its
                                          // place in the blend order, the front entry's list position
    size_t t_part;                        // translucent: kTPartials floats per surfel slot
    size_t status;                        // the frame's ges_run_status, assembled on the device
    size_t total;
    int64_t n, m;
    int32_t n_views;
    int64_t pixels;
    int64_t samples;                      // surfel-pass samples of all views (pixels x 1 or 4)
    int32_t rtiles, stiles;               // total raster / splat tiles
    int64_t s_cap, g_cap;                 // list entries (and slots) available
    int64_t scan_blocks;
};

// ---------------------------------------------------------------------------
// device math

// Real SH basis, Condon-Shortley phase, k = l^2 + l + m, at unit direction
// (x, y, z).  Constants: C0 = 1/(2 sqrt(pi)), C1 = sqrt(3/(4 pi)),
// C2a = sqrt(15/pi)/2, C2b = sqrt(5/pi)/4, C2c = sqrt(15/pi)/4,
// C3a = sqrt(35/(2 pi))/4, C3b = sqrt(105/pi)/2, C3c = sqrt(21/(2 pi))/4,
// C3d = sqrt(7/pi)/4, C3e = sqrt(105/pi)/4.
constexpr double kC0 = 0.28209479177387814;
constexpr double kC1 = 0.48860251190291992;
constexpr double kC2a = 1.0925484305920792;
constexpr double kC2b = 0.31539156525252005;
constexpr double kC2c = 0.54627421529603959;
constexpr double kC3a = 0.59004358992664352;
constexpr double kC3b = 2.8906114426405538;
constexpr double kC3c = 0.45704579946446572;
constexpr double kC3d = 0.37317633259011540;
constexpr double kC3e = 1.4453057213202769;

template <typename T>
__device__ inline void sh_basis(T x, T y, T z, int K, T *Y) {
    Y[0] = T(kC0);
    if (K > 1) {
        Y[1] = -T(kC1) * y;
        Y[2] = T(kC1) * z;
        Y[3] = -T(kC1) * x;
    }
    if (K > 4) {
        const T xx = x * x, yy = y * y, zz = z * z;
        Y[4] = T(kC2a) * x * y;
        Y[5] = -T(kC2a) * y * z;
        Y[6] = T(kC2b) * (T(2) * zz - xx - yy);
        Y[7] = -T(kC2a) * x * z;
        Y[8] = T(kC2c) * (xx - yy);
        if (K > 9) {
            Y[9] = -T(kC3a) * y * (T(3) * xx - yy);
            Y[10] = T(kC3b) * x * y * z;
            Y[11] = -T(kC3c) * y * (T(4) * zz - xx - yy);
            Y[12] = T(kC3d) * z * (T(2) * zz - T(3) * xx - T(3) * yy);
            Y[13] = -T(kC3c) * x * (T(4) * zz - xx - yy);
            Y[14] = T(kC3e) * z * (xx - yy);
            Y[15] = -T(kC3a) * x * (xx - T(3) * yy);
        }
    }
}

// sum_k w_k grad Y_k(x, y, z) without materialising the 16x3 gradient table
// (the SH view-direction term of the backward).
template <typename T>
__device__ inline void sh_grad_dot(T x, T y, T z, int K, const T *w, T *g) {
    g[0] = g[1] = g[2] = T(0);
    if (K > 1) {
        g[1] += -T(kC1) * w[1];
        g[2] += T(kC1) * w[2];
        g[0] += -T(kC1) * w[3];
    }
    if (K > 4) {
        g[0] += T(kC2a) * y * w[4];             g[1] += T(kC2a) * x * w[4];
        g[1] += -T(kC2a) * z * w[5];            g[2] += -T(kC2a) * y * w[5];
        g[0] += -T(2) * T(kC2b) * x * w[6];     g[1] += -T(2) * T(kC2b) * y * w[6];
        g[2] += T(4) * T(kC2b) * z * w[6];
        g[0] += -T(kC2a) * z * w[7];            g[2] += -T(kC2a) * x * w[7];
        g[0] += T(2) * T(kC2c) * x * w[8];      g[1] += -T(2) * T(kC2c) * y * w[8];
        if (K > 9) {
            const T xx = x * x, yy = y * y, zz = z * z;
            g[0] += -T(kC3a) * T(6) * x * y * w[9];
            g[1] += -T(kC3a) * (T(3) * xx - T(3) * yy) * w[9];
            g[0] += T(kC3b) * y * z * w[10];
            g[1] += T(kC3b) * x * z * w[10];
            g[2] += T(kC3b) * x * y * w[10];
            g[0] += T(kC3c) * T(2) * x * y * w[11];
            g[1] += -T(kC3c) * (T(4) * zz - xx - T(3) * yy) * w[11];
            g[2] += -T(kC3c) * T(8) * y * z * w[11];
            g[0] += -T(kC3d) * T(6) * x * z * w[12];
            g[1] += -T(kC3d) * T(6) * y * z * w[12];
            g[2] += T(kC3d) * (T(6) * zz - T(3) * xx - T(3) * yy) * w[12];
            g[0] += -T(kC3c) * (T(4) * zz - T(3) * xx - yy) * w[13];
            g[1] += T(kC3c) * T(2) * x * y * w[13];
            g[2] += -T(kC3c) * T(8) * x * z * w[13];
            g[0] += T(kC3e) * T(2) * x * z * w[14];
            g[1] += -T(kC3e) * T(2) * y * z * w[14];
            g[2] += T(kC3e) * (xx - yy) * w[14];
            g[0] += -T(kC3a) * (T(3) * xx - T(3) * yy) * w[15];
            g[1] += T(kC3a) * T(6) * x * y * w[15];
        }
    }
}

// Rotation matrix (row-major) of the normalised quaternion (w, x, y, z).
template <typename T>
__device__ inline void quat_rot(T w, T x, T y, T z, T *Rm) {
    Rm[0] = T(1) - T(2) * (y * y + z * z);
    Rm[1] = T(2) * (x * y - w * z);
    Rm[2] = T(2) * (x * z + w * y);
    Rm[3] = T(2) * (x * y + w * z);
    Rm[4] = T(1) - T(2) * (x * x + z * z);
    Rm[5] = T(2) * (y * z - w * x);
    Rm[6] = T(2) * (x * z - w * y);
    Rm[7] = T(2) * (y * z + w * x);
    Rm[8] = T(1) - T(2) * (x * x + y * y);
}

// -0.5 / ln 2: alpha = sigma * exp(-q/2) = exp2(log2 sigma + kNegHalfLog2e * q)
constexpr float kNegHalfLog2e = -0.72134752044448170f;

// Opacity of a Gaussian record at a pixel centre (Eq. 4).  Forward and
// backward both call this, so their keep decisions agree bit for bit.
__device__ __forceinline__ float gauss_alpha(const GRec &g, float x, float y, float &dx, float &dy,
                                             float &q) {
    dx = x - g.px;
    dy = y - g.py;
    q = dx * (g.ca * dx + 2.f * g.cb * dy) + g.cc * dy * dy;
    // the hardware exp2 (v_exp_f32): exp2f adds only a denormal-range
    // wrapper, and alpha below alpha_min (1/255) is discarded anyway
    return __builtin_amdgcn_exp2f(fmaf(q, kNegHalfLog2e, g.lsig));
}

// A 2D Gaussian list entry at the camera ray (xr, yr, 1) of a pixel centre:
// whether it counts in pass 2 (the ray meets the plane in front of the near
// plane, alpha >= alpha_min, planar depth z < D_s + eps), with alpha and z.
// Pass 2 and the geometry channels both call this: their decisions agree
// bit for bit.
__device__ __forceinline__ bool g2_eval(const G2Ent &e, float xr, float yr, float zn, float amin, float ds,
                                        float &alpha, float &z) {
    const float c = fmaf(e.nx, xr, fmaf(e.ny, yr, e.nz));
    const float au = fmaf(e.Ux, xr, fmaf(e.Uy, yr, e.Uz));
    const float bv = fmaf(e.Vx, xr, fmaf(e.Vy, yr, e.Vz));
    const float ic = __builtin_amdgcn_rcpf(c);
    const float u = au * ic, v = bv * ic;
    alpha = e.sigma * __builtin_amdgcn_exp2f(fmaf(u, u, v * v) * kNegHalfLog2e);
    z = e.w * ic;
    return (c > 0.f) & (e.w >= zn * c) & (alpha >= amin) & (z < ds + e.eps);
}

__device__ __forceinline__ uint64_t umin64(uint64_t x, uint64_t y) { return x < y ? x : y; }

// Flattened tile index -> view (views are few: a scalar linear scan).
__device__ __forceinline__ int view_of_rtile(const ViewDev *views, int nv, int t) {
    int v = 0;
    while (v + 1 < nv && views[v + 1].rt_off <= t) ++v;
    return v;
}
__device__ __forceinline__ int view_of_stile(const ViewDev *views, int nv, int t) {
    int v = 0;
    while (v + 1 < nv && views[v + 1].st_off <= t) ++v;
    return v;
}

// ---------------------------------------------------------------------------
// launchers (one per kernel family; defined in the .hip files)

struct FrameArgs {
    const ViewDev *views;
    int n_views;
    int64_t n, m;
    int ks, kg;                   // SH coefficient rows of surfels, Gaussians
    ges_options opt;
    ges_surfels S;
    ges_gaussians G;
    unsigned char *ws;
    WsLayout L;                   // workspace layout (by value: kernels read it)
    int max_rt_per_view, max_st_per_view;
    // translucent surfels (the surfel optimisation stage): no occluders,
    // per-surfel opacity modulation w_mod, and the order adjustment
    int translucent, front_first;
    const float *w_mod;
};

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
// The frame's ges_run_status computed on the device into *out (workspace).
hipError_t launch_status(const WsHeader *h, int64_t s_cap, int64_t g_cap, int splatted, ges_run_status *out,
                         hipStream_t s);
// Fills up to four regions (word value val[r]) in one launch.
struct FillSet {
    uint32_t *p[4];
    int64_t n[4];
    uint32_t val[4];
    int count;
};
hipError_t launch_fill_set(const FillSet &f, hipStream_t s);
// Fills mult * (*count) words (at most max) with value; *count is read on the
// device when the kernel runs (a total an earlier kernel wrote).
hipError_t launch_fill_u32_counted(uint32_t *p, uint32_t value, const unsigned long long *count, int64_t mult,
                                   int64_t max, hipStream_t s);
// Exclusive scan: out[i] <- sum_{k<i} in[k * in_stride] for i < count; the
// total goes to out[count] and to *total64 (if not null).  In place when
// in == out and in_stride == 1.
hipError_t launch_scan_u32(const uint32_t *in, int64_t in_stride, uint32_t *out, int64_t count, uint32_t *tmp,
                           int64_t tmp_blocks, unsigned long long *total64, hipStream_t s);
// Two independent scans sharing their launches (each with its own tmp).
struct ScanJob {
    const uint32_t *in;
    int64_t stride;
    uint32_t *out;
    int64_t count;
    uint32_t *tmp;
    unsigned long long *total64;
};
hipError_t launch_scan2_u32(const ScanJob &j0, const ScanJob &j1, int64_t tmp_blocks, hipStream_t s);
int64_t scan_tmp_blocks(int64_t count);

// Gaussian and surfel projection in one launch.
hipError_t launch_project(const FrameArgs &a, hipStream_t s);
hipError_t launch_surfel_count(const FrameArgs &a, hipStream_t s);
hipError_t launch_surfel_fill(const FrameArgs &a, hipStream_t s);
// cus: compute units of the device (the persistent variant's grid).  sid and
// depth are per sample of the surfel grid.
hipError_t launch_raster(const FrameArgs &a, int32_t *sid, float *depth, int cus, hipStream_t s);
hipError_t launch_shade(const FrameArgs &a, hipStream_t s);
// sid / sdepth per sample; with 4 samples per pixel the pixel depth (mean of
// the hit samples) goes to depth, else sdepth is the depth map already.
hipError_t launch_resolve(const FrameArgs &a, const int32_t *sid, const float *sdepth, float *depth, float *color_s,
                          hipStream_t s);
hipError_t launch_gauss_count(const FrameArgs &a, hipStream_t s);
hipError_t launch_gauss_fill(const FrameArgs &a, hipStream_t s);
hipError_t launch_splat(const FrameArgs &a, const float *depth, const float *color_s, float *image,
                        float *accum, hipStream_t s);
hipError_t launch_bwd_tiles(const FrameArgs &a, const float *depth, const float *color_s, const float *accum,
                            const float *d_image, hipStream_t s);
hipError_t launch_bwd_surfel_tiles(const FrameArgs &a, const int32_t *sid, const float *accum,
                                   const float *d_image, hipStream_t s);
hipError_t launch_bwd_compact(const FrameArgs &a, const ges_gradients &g, hipStream_t s);
hipError_t launch_bwd_gaussians(const FrameArgs &a, const ges_gradients &g, int cus, hipStream_t s);
// Translucent surfels (ges_translucent.hip).
hipError_t launch_tblend(const FrameArgs &a, float *color, float *alpha, float *depth, int32_t *front, hipStream_t s);
hipError_t launch_tblend_bwd(const FrameArgs &a, const float *d_color, hipStream_t s);
hipError_t launch_tsurfels(const FrameArgs &a, float *g_mean, float *g_quat, float *g_scale, float *g_w, float *g_sh,
                           hipStream_t s);
hipError_t launch_bwd_surfels(const FrameArgs &a, const ges_gradients &g, hipStream_t s);
// Pruning scores: one view's covering counts folded into cover (cnt must
// read zero before and reads zero after); every view's contribution maxima
// folded into contrib (as float bits); keep flags.
hipError_t launch_score_surfel_view(const FrameArgs &a, int v, int ntiles, const int32_t *sid, uint32_t *cnt,
                                    int32_t *cover, int first_overwrite, hipStream_t s);
hipError_t launch_score_gauss(const FrameArgs &a, const float *depth, const float *accum, float *contrib,
                              hipStream_t s);
// Cameras of one launch of the Mip-GES filter-size kernel (passed by value).
constexpr int kMipCams = 16;
struct MipCams {
    int n;
    float R[kMipCams][9], t[kMipCams][3];
    float fx[kMipCams], fy[kMipCams], cx[kMipCams], cy[kMipCams], W[kMipCams], H[kMipCams], znear[kMipCams];
};
hipError_t launch_mip_filter3d(const float *mean, int64_t m, const ges_camera *cams, int n_views, float scale2,
                               float *out, hipStream_t s);

// Geometry channels (Eq. 10-12) over the frame's splat tiles.
hipError_t launch_geometry(const FrameArgs &a, const int32_t *sid, const float *depth, const float *accum,
                           const ges_geometry_out &out, hipStream_t s);
hipError_t launch_score_masks(int64_t n, int64_t m, const int32_t *cover, const float *contrib, int32_t cover_min,
                              float contrib_min, uint8_t *keep_s, uint8_t *keep_g, hipStream_t s);

}  // namespace ges
