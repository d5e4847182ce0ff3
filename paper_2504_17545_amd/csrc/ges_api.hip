// Host side of the C ABI declared in include/ges.h: argument validation,
// workspace layout, the per-frame launch sequence and status reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "ges_internal.h"

using namespace ges;

namespace {

thread_local std::string g_err;

ges_status fail(ges_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(GES_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

bool finite_pos(float x) { return isfinite(x) && x > 0.f; }

ges_status validate_cameras(const ges_camera *cams, int32_t n_views) {
    if (!cams) return fail(GES_ERR_ARG, "cams is NULL");
    if (n_views < 1 || n_views > kMaxViews) return fail(GES_ERR_ARG, "n_views=%d outside [1, %d]", n_views, kMaxViews);
    int64_t pix = 0;
    for (int v = 0; v < n_views; ++v) {
        const ges_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
            return fail(GES_ERR_ARG, "camera %d: size %dx%d outside [1, 16384]", v, c.width, c.height);
        if (!finite_pos(c.fx) || !finite_pos(c.fy))
            return fail(GES_ERR_ARG, "camera %d: focal lengths must be finite and > 0", v);
        if (!isfinite(c.cx) || !isfinite(c.cy)) return fail(GES_ERR_ARG, "camera %d: principal point not finite", v);
        if (!finite_pos(c.znear)) return fail(GES_ERR_ARG, "camera %d: znear must be finite and > 0", v);
        for (int k = 0; k < 9; ++k)
            if (!isfinite(c.R[k])) return fail(GES_ERR_ARG, "camera %d: R not finite", v);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.t[k]) || !isfinite(c.bg[k])) return fail(GES_ERR_ARG, "camera %d: t/bg not finite", v);
        pix += (int64_t)c.width * c.height;
    }
    if (pix >= (int64_t)1 << 31) return fail(GES_ERR_ARG, "total pixels %lld exceed 2^31", (long long)pix);
    return GES_OK;
}

ges_status validate_options(const ges_options *o) {
    if (!o) return fail(GES_ERR_ARG, "options is NULL");
    if (!finite_pos(o->surfel_radius)) return fail(GES_ERR_ARG, "surfel_radius must be > 0");
    if (!(o->alpha_min > 0.f && o->alpha_min < 1.f)) return fail(GES_ERR_ARG, "alpha_min must be in (0, 1)");
    if (!(isfinite(o->dilation) && o->dilation >= 0.f)) return fail(GES_ERR_ARG, "dilation must be >= 0");
    if (!finite_pos(o->w_s)) return fail(GES_ERR_ARG, "w_s must be > 0");
    if (!(isfinite(o->mip_2d) && o->mip_2d >= 0.f)) return fail(GES_ERR_ARG, "mip_2d must be finite and >= 0");
    if (!isfinite(o->eps_factor) || !isfinite(o->eps_const)) return fail(GES_ERR_ARG, "eps not finite");
    if (o->raster_tile != 8 && o->raster_tile != 16)
        return fail(GES_ERR_UNSUPPORTED, "raster_tile=%d (built: 8, 16)", o->raster_tile);
    const int tw = o->splat_tile_w, th = o->splat_tile_h;
    if (!((tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16)))
        return fail(GES_ERR_UNSUPPORTED, "splat tile %dx%d (built: 8x8, 16x8, 16x16)", tw, th);
    if (o->tile_queue < 0 || o->tile_queue > 32) return fail(GES_ERR_ARG, "tile_queue=%d outside [0, 32]", o->tile_queue);
    if (o->surfel_samples != 1 && o->surfel_samples != 4)
        return fail(GES_ERR_UNSUPPORTED, "surfel_samples=%d (built: 1, 4)", o->surfel_samples);
    if (o->surfel_pair_capacity < 0 || o->gauss_pair_capacity < 0) return fail(GES_ERR_ARG, "negative capacity");
    if (o->surfel_pair_capacity > 0x7fffffffLL || o->gauss_pair_capacity > 0x7fffffffLL)
        return fail(GES_ERR_ARG, "capacity above 2^31 - 1");
    return GES_OK;
}

int sh_rows(int degree) { return (degree + 1) * (degree + 1); }

ges_status validate_scene(const ges_surfels *S, const ges_gaussians *G) {
    if (!S || !G) return fail(GES_ERR_ARG, "surfels/gaussians descriptor is NULL");
    if (S->n < 0 || G->m < 0) return fail(GES_ERR_ARG, "negative primitive count");
    if (S->n > 0x7fffffffLL || G->m > 0x7fffffffLL) return fail(GES_ERR_ARG, "primitive count above 2^31 - 1");
    if (S->sh_degree < 0 || S->sh_degree > 3 || G->sh_degree < 0 || G->sh_degree > 3)
        return fail(GES_ERR_ARG, "sh_degree must be in [0, 3]");
    if (S->n > 0 && (!S->mean || !S->quat || !S->scale || !S->sh)) return fail(GES_ERR_ARG, "surfel array is NULL");
    if (G->m > 0 && (!G->mean || !G->quat || !G->scale || !G->opacity || !G->sh))
        return fail(GES_ERR_ARG, "Gaussian array is NULL");
    if (G->dims != 0 && G->dims != 2 && G->dims != 3) return fail(GES_ERR_ARG, "Gaussian dims must be 0, 2 or 3");
    return GES_OK;
}

// 2D Gaussians (2D-GES) render forward only, without the Mip-GES filters.
ges_status validate_gauss2d(const ges_gaussians *G, const ges_options *opt) {
    if (G->dims != 2) return GES_OK;
    if (G->filter3d) return fail(GES_ERR_UNSUPPORTED, "2D Gaussians with the Mip-GES 3D filter");
    if (opt->mip_2d > 0.f) return fail(GES_ERR_UNSUPPORTED, "2D Gaussians with the Mip-GES screen filter");
    return GES_OK;
}

// Tile counts and offsets of every view (host mirror of ViewDev).
void build_views(const ges_camera *cams, int32_t n_views, const ges_options *o, std::vector<ViewDev> &out,
                 int32_t &rtiles, int32_t &stiles, int64_t &pixels, int &max_rt, int &max_st) {
    out.resize(n_views);
    rtiles = stiles = 0;
    pixels = 0;
    int64_t samples = 0;
    const int f = o->surfel_samples == 4 ? 2 : 1;  // sample grid: f x f per pixel
    max_rt = max_st = 0;
    const int T = o->raster_tile, TW = o->splat_tile_w, TH = o->splat_tile_h;
    for (int v = 0; v < n_views; ++v) {
        const ges_camera &c = cams[v];
        ViewDev &V = out[v];
        memset(&V, 0, sizeof V);
        V.W = c.width;
        V.H = c.height;
        V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
        memcpy(V.R, c.R, sizeof V.R);
        memcpy(V.t, c.t, sizeof V.t);
        V.znear = c.znear;
        memcpy(V.bg, c.bg, sizeof V.bg);
        for (int k = 0; k < 3; ++k)
            V.o[k] = -(double)c.R[k] * c.t[0] - (double)c.R[3 + k] * c.t[1] - (double)c.R[6 + k] * c.t[2];
        V.limx = (float)(1.3 * (double)c.width / (2.0 * c.fx));
        V.limy = (float)(1.3 * (double)c.height / (2.0 * c.fy));
        V.sW = c.width * f;
        V.sH = c.height * f;
        V.sfx = c.fx * (float)f;
        V.sfy = c.fy * (float)f;
        V.scx = c.cx * (float)f;
        V.scy = c.cy * (float)f;
        V.s_off = samples;
        samples += (int64_t)V.sW * V.sH;
        V.rtx = (V.sW + T - 1) / T;
        V.rty = (V.sH + T - 1) / T;
        V.stx = (c.width + TW - 1) / TW;
        V.sty = (c.height + TH - 1) / TH;
        V.rt_off = rtiles;
        V.st_off = stiles;
        V.pix_off = pixels;
        rtiles += V.rtx * V.rty;
        stiles += V.stx * V.sty;
        pixels += (int64_t)c.width * c.height;
        max_rt = V.rtx * V.rty > max_rt ? V.rtx * V.rty : max_rt;
        max_st = V.stx * V.sty > max_st ? V.stx * V.sty : max_st;
    }
}

WsLayout make_layout(const std::vector<ViewDev> &views, int32_t rtiles, int32_t stiles, int64_t pixels, int64_t n,
                     int64_t m, const ges_options *o, bool translucent = false) {
    WsLayout L;
    memset(&L, 0, sizeof L);
    const int64_t nv = (int64_t)views.size();
    L.n = n;
    L.m = m;
    L.n_views = (int32_t)nv;
    L.pixels = pixels;
    L.samples = o->surfel_samples == 4 ? 4 * pixels : pixels;
    L.rtiles = rtiles;
    L.stiles = stiles;
    L.s_cap = o->surfel_pair_capacity > 0 ? o->surfel_pair_capacity : 12 * n * nv + rtiles + 1024;
    L.g_cap = o->gauss_pair_capacity > 0 ? o->gauss_pair_capacity : 8 * m * nv + stiles + 1024;
    if (L.s_cap > (int64_t)kCopyPosMask) L.s_cap = kCopyPosMask;  // slots hold a 29-bit position
    if (L.g_cap > 0x7fffffffLL) L.g_cap = 0x7fffffffLL;
    int64_t scan_max = (int64_t)rtiles * kCounterCopies + 1;
    if (stiles + 1 > scan_max) scan_max = stiles + 1;
    if (nv * m + 1 > scan_max) scan_max = nv * m + 1;
    if (nv * n + 1 > scan_max) scan_max = nv * n + 1;
    L.scan_blocks = scan_tmp_blocks(scan_max) + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + (bytes ? bytes : 1));
        return at;
    };
    L.header = take(sizeof(WsHeader));
    L.views = take(sizeof(ViewDev) * nv);
    L.grec = take(sizeof(G2Rec) * nv * m);  // 64 B: 2D Gaussians; 3D ones use 48 B of each
    L.gbox = take(sizeof(uint2) * nv * m);
    L.g_boff = take(sizeof(uint32_t) * (nv * m + 1));
    L.srec = take(sizeof(SRec) * nv * n);
    L.s_zmin = take(sizeof(float) * nv * n);
    L.sbox = take(sizeof(uint2) * nv * n);
    L.s_boff = take(sizeof(uint32_t) * (nv * n + 1));
    L.svis = take(align_up((size_t)(nv * n), 4));
    L.scol = take(sizeof(float) * 3 * nv * n);
    L.s_tcnt = take(sizeof(uint32_t) * kCounterStride * (size_t)rtiles * kCounterCopies);
    L.s_toff = take(sizeof(uint32_t) * ((size_t)rtiles * kCounterCopies + 1));
    L.s_tocc = take(sizeof(float) * rtiles);
    L.g_tcnt = take(sizeof(uint32_t) * kCounterStride * (size_t)stiles);
    L.g_toff = take(sizeof(uint32_t) * (stiles + 1));
    L.tile_maxd = take(sizeof(float) * stiles);
    L.s_ord = take(sizeof(TileOrd) * rtiles);
    L.g_ord = take(sizeof(TileOrd) * stiles);
    L.s_ents = take(sizeof(SEnt) * L.s_cap);
    L.s_slot = take(sizeof(uint32_t) * L.s_cap);
    L.g_ents = take(sizeof(GEnt) * L.g_cap);
    L.g_slot = take(sizeof(uint32_t) * L.g_cap);
    L.g_nkept = take(sizeof(uint32_t) * nv * m);
    L.g_act = take(sizeof(uint32_t) * m);
    L.g_aoff = take(sizeof(uint32_t) * (m + 1));
    L.g_alist = take(sizeof(uint32_t) * m);
    L.g_part = take(sizeof(float) * 9 * L.g_cap);
    L.s_part = take(sizeof(float) * 3 * L.s_cap);
    L.scan_tmp = take(sizeof(uint32_t) * L.scan_blocks);
    L.scan_tmp2 = take(sizeof(uint32_t) * L.scan_blocks);  // the second of two scans sharing launches
    L.s_cnt = take(sizeof(uint32_t) * n);
    L.status = take(sizeof(ges_run_status));
    L.s_depth = take(o->surfel_samples == 4 ? sizeof(float) * L.samples : 0);
    L.t_sorted = take(translucent ? sizeof(uint32_t) * L.s_cap : 0);
    L.t_state = take(translucent ? sizeof(float) * 3 * pixels : 0);
    L.t_part = take(translucent ? sizeof(float) * kTPartials * L.s_cap : 0);
    L.total = off;
    return L;
}

}  // namespace

struct ges_context {
    int device = 0;
    int cus = 256;  // compute units (the persistent raster's grid)
    int stage = 0;  // 0 none, 1 projected, 2 rastered, 3 splatted; kStageTranslucent: a translucent frame
    // translucent surfels (ges_translucent_render): the frame's mode and w
    int translucent = 0, front_first = 0;
    const float *w_mod = nullptr;
    ges_options opt;
    ges_surfels S;
    ges_gaussians G;
    std::vector<ViewDev> views;
    WsLayout L;
    unsigned char *ws = nullptr;
    // staging copies of the view table in pinned host memory, used in turn:
    // a frame's asynchronous copy reads its buffer while the host fills the
    // next frame's, so the host waits only if a buffer comes round again
    // before the copy that read it has run (a plan's graph uses buffer 0)
    static constexpr int kStaging = 4;
    ViewDev *pinned[kStaging] = {};
    hipEvent_t copied[kStaging] = {};
    bool copy_pending[kStaging] = {};
    int pinned_cap = 0;
    int next_staging = 0;
    bool capturing = false;  // a plan is recording this frame into a graph
    int max_rt = 0, max_st = 0;
    // second stream for the backward's independent surfel chain: the
    // backward forks onto it after an event on the caller's stream and joins
    // back before it returns (captured as a parallel graph branch by a plan)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_mid = nullptr;

    hipError_t ensure_aux() {
        if (aux) return hipSuccess;
        hipError_t e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_mid, hipEventDisableTiming);
        return e;
    }
    hipError_t fork(hipStream_t s) {
        hipError_t e = hipEventRecord(ev_fork, s);
        return e == hipSuccess ? hipStreamWaitEvent(aux, ev_fork, 0) : e;
    }
    hipError_t join(hipStream_t s) {
        hipError_t e = hipEventRecord(ev_join, aux);
        return e == hipSuccess ? hipStreamWaitEvent(s, ev_join, 0) : e;
    }
    // stage timing
    bool profile = false;
    struct Pending {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    double stage_ms[GES_STAGE_COUNT] = {};
    int64_t stage_n[GES_STAGE_COUNT] = {};

    hipEvent_t event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    FrameArgs args() const {
        FrameArgs a;
        a.views = reinterpret_cast<const ViewDev *>(ws + L.views);
        a.n_views = (int)views.size();
        a.n = S.n;
        a.m = G.m;
        a.ks = sh_rows(S.sh_degree);
        a.kg = sh_rows(G.sh_degree);
        a.opt = opt;
        a.S = S;
        a.G = G;
        a.ws = ws;
        a.L = L;
        a.max_rt_per_view = max_rt;
        a.max_st_per_view = max_st;
        a.translucent = translucent;
        a.front_first = front_first;
        a.w_mod = w_mod;
        return a;
    }
};

// Runs a launcher; with stage timing on, brackets it with two events.
#define TIMED(ctx, stage, stream, expr)                                          \
    do {                                                                         \
        hipEvent_t ea_ = nullptr, eb_ = nullptr;                                 \
        if ((ctx)->profile && !(ctx)->capturing) {                               \
            ea_ = (ctx)->event();                                                \
            eb_ = (ctx)->event();                                                \
            if (ea_) HIP_TRY(hipEventRecord(ea_, stream));                       \
        }                                                                        \
        HIP_TRY(expr);                                                           \
        if (ea_ && eb_) {                                                        \
            HIP_TRY(hipEventRecord(eb_, stream));                                \
            (ctx)->pending.push_back({(int)(stage), ea_, eb_});                  \
        }                                                                        \
    } while (0)

// Scratch of ges_scores_static: the per-surfel counters live in a device
// array of the library instead of the frame's workspace (one copy per
// device, held until the process ends).  Host code must use the address
// hipGetSymbolAddress returns on each device, never the array's name.
constexpr int64_t kStaticScoreWords = int64_t(1) << 22;  // surfels: 4,194,304 (16 MiB)
static __device__ __align__(256) uint32_t scratch[kStaticScoreWords];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// The pruning-score launch sequence; cnt: n words of scratch (zeroed here,
// left zeroed).
static ges_status run_scores(ges_context *ctx, const int32_t *sid, const float *depth, const float *accum,
                             int32_t cover_min, float contrib_min, int32_t accumulate, const ges_scores_out *out,
                             uint32_t *cnt, hipStream_t s) {
    const FrameArgs a = ctx->args();
    if (a.n > 0) {
        HIP_TRY(launch_fill_u32(cnt, 0u, a.n, s));
        for (int v = 0; v < (int)ctx->views.size(); ++v) {
            const ViewDev &V = ctx->views[v];
            HIP_TRY(launch_score_surfel_view(a, v, V.rtx * V.rty, sid, cnt, out->cover, v == 0 && !accumulate, s));
        }
    }
    if (a.m > 0) {
        if (!accumulate) HIP_TRY(launch_fill_u32((uint32_t *)out->contrib, 0u, a.m, s));
        HIP_TRY(launch_score_gauss(a, depth, accum, out->contrib, s));
    }
    HIP_TRY(launch_score_masks(a.n, a.m, out->cover, out->contrib, cover_min, contrib_min,
                               a.n > 0 ? out->keep_surfel : nullptr, a.m > 0 ? out->keep_gauss : nullptr, s));
    return GES_OK;
}

extern "C" {

void ges_options_default(ges_options *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->surfel_radius = (float)sqrt(2.0 * log(255.0));
    o->eps_factor = 5.0f;
    o->eps_const = -1.0f;
    o->alpha_min = 1.0f / 255.0f;
    o->dilation = 0.3f;
    o->w_s = 1.0f;
    o->raster_tile = 8;
    o->splat_tile_w = 16;
    o->splat_tile_h = 16;
    o->surfel_samples = 1;
}

const char *ges_last_error(void) { return g_err.c_str(); }

ges_status ges_context_create(ges_context **out, int device) {
    if (!out) return fail(GES_ERR_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(GES_ERR_HIP, "no HIP device %d (count %d)", device, count);
    ges_context *c = new ges_context();
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->cus = cus;
    ges_options_default(&c->opt);
    *out = c;
    return GES_OK;
}

ges_status ges_context_destroy(ges_context *ctx) {
    if (!ctx) return GES_OK;
    for (int k = 0; k < ges_context::kStaging; ++k) {
        if (ctx->copied[k]) {
            (void)hipEventSynchronize(ctx->copied[k]);
            (void)hipEventDestroy(ctx->copied[k]);
        }
        if (ctx->pinned[k]) (void)hipHostFree(ctx->pinned[k]);
    }
    for (auto &p : ctx->pending) {
        (void)hipEventSynchronize(p.b);
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->aux) {
        (void)hipStreamSynchronize(ctx->aux);
        (void)hipStreamDestroy(ctx->aux);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_mid) (void)hipEventDestroy(ctx->ev_mid);
    delete ctx;
    return GES_OK;
}

ges_status ges_total_pixels(const ges_camera *cams, int32_t n_views, int64_t *pixels) {
    if (!pixels) return fail(GES_ERR_ARG, "pixels is NULL");
    ges_status st = validate_cameras(cams, n_views);
    if (st) return st;
    int64_t p = 0;
    for (int v = 0; v < n_views; ++v) p += (int64_t)cams[v].width * cams[v].height;
    *pixels = p;
    return GES_OK;
}

ges_status ges_workspace_query(const ges_camera *cams, int32_t n_views, int64_t n, int64_t m, const ges_options *opt,
                               size_t *bytes) {
    if (!bytes) return fail(GES_ERR_ARG, "bytes is NULL");
    ges_status st = validate_cameras(cams, n_views);
    if (st) return st;
    if ((st = validate_options(opt))) return st;
    if (n < 0 || m < 0 || n > 0x7fffffffLL || m > 0x7fffffffLL) return fail(GES_ERR_ARG, "bad primitive counts");
    std::vector<ViewDev> views;
    int32_t rt, stl;
    int64_t pix;
    int a, b;
    build_views(cams, n_views, opt, views, rt, stl, pix, a, b);
    *bytes = make_layout(views, rt, stl, pix, n, m, opt).total;
    return GES_OK;
}

namespace {

constexpr int kStageTranslucent = 10;

// The frame's set-up, projection and surfel binning count (ges_project);
// with `translucent`, for translucent surfels (no occluders, w per surfel).
ges_status project_frame(ges_context *ctx, const ges_camera *cams, int32_t n_views, const ges_surfels *surfels,
                         const ges_gaussians *gaussians, const ges_options *opt, void *ws, size_t ws_bytes,
                         void *stream, bool translucent, const float *w_mod, int front_first) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    ges_status st;
    if ((st = validate_cameras(cams, n_views))) return st;
    if ((st = validate_options(opt))) return st;
    if ((st = validate_scene(surfels, gaussians))) return st;
    if ((st = validate_gauss2d(gaussians, opt))) return st;
    std::vector<ViewDev> views;
    int32_t rt, stl;
    int64_t pix;
    int max_rt, max_st;
    build_views(cams, n_views, opt, views, rt, stl, pix, max_rt, max_st);
    WsLayout L = make_layout(views, rt, stl, pix, surfels->n, gaussians->m, opt, translucent);
    if (!ws) return fail(GES_ERR_WORKSPACE, "workspace is NULL");
    if (ws_bytes < L.total)
        return fail(GES_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    if (((uintptr_t)ws & 255u) != 0) return fail(GES_ERR_WORKSPACE, "workspace must be 256-byte aligned");

    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    int slot = 0;
    if (ctx->capturing) {
        // nothing is uploaded under capture (the plan uploads the table);
        // the staging buffers were sized by the plan's trial frames
        if (ctx->pinned_cap < n_views) return fail(GES_ERR_STATE, "staging buffer not sized before capture");
    } else {
        slot = ctx->next_staging;
        ctx->next_staging = (slot + 1) % ges_context::kStaging;
        if (!ctx->copied[slot]) HIP_TRY(hipEventCreateWithFlags(&ctx->copied[slot], hipEventDisableTiming));
        if (ctx->copy_pending[slot]) {  // normally long done: the copy ran frames ago
            HIP_TRY(hipEventSynchronize(ctx->copied[slot]));
            ctx->copy_pending[slot] = false;
        }
    }
    if (ctx->pinned_cap < n_views) {
        for (int k = 0; k < ges_context::kStaging; ++k) {
            if (ctx->copy_pending[k]) {
                HIP_TRY(hipEventSynchronize(ctx->copied[k]));
                ctx->copy_pending[k] = false;
            }
            if (ctx->pinned[k]) HIP_TRY(hipHostFree(ctx->pinned[k]));
            ctx->pinned[k] = nullptr;
        }
        ctx->pinned_cap = 0;
        for (int k = 0; k < ges_context::kStaging; ++k)
            HIP_TRY(hipHostMalloc((void **)&ctx->pinned[k], sizeof(ViewDev) * n_views, hipHostMallocDefault));
        ctx->pinned_cap = n_views;
    }
    if (!ctx->capturing) memcpy(ctx->pinned[slot], views.data(), sizeof(ViewDev) * n_views);

    ctx->opt = *opt;
    ctx->S = *surfels;
    ctx->G = *gaussians;
    ctx->views = views;
    ctx->L = L;
    ctx->ws = (unsigned char *)ws;
    ctx->max_rt = max_rt;
    ctx->max_st = max_st;
    ctx->stage = 0;
    ctx->translucent = translucent ? 1 : 0;
    ctx->front_first = front_first ? 1 : 0;
    ctx->w_mod = w_mod;

    unsigned char *w = ctx->ws;
    // a plan's graph holds no copy of the view table: the plan uploads it
    // on its launch stream, before a replay, when the cameras change
    if (!ctx->capturing) {
        HIP_TRY(hipMemcpyAsync(w + L.views, ctx->pinned[slot], sizeof(ViewDev) * n_views, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ctx->copied[slot], s));
        ctx->copy_pending[slot] = true;
    }
    WsHeader *hdr = (WsHeader *)(w + L.header);
    {
        FillSet f{};
        f.p[0] = (uint32_t *)(w + L.header);
        f.n[0] = sizeof(WsHeader) / 4;
        f.p[1] = (uint32_t *)(w + L.s_tcnt);
        f.n[1] = (int64_t)rt * kCounterStride * kCounterCopies;
        f.p[2] = (uint32_t *)(w + L.svis);
        f.n[2] = (int64_t)align_up((size_t)(n_views * surfels->n), 4) / 4;
        f.p[3] = (uint32_t *)(w + L.s_tocc);  // +inf: no occluder yet
        f.n[3] = rt;
        f.val[3] = 0x7f800000u;
        f.count = 4;
        TIMED(ctx, GES_STAGE_CLEAR, s, launch_fill_set(f, s));
    }
    const FrameArgs a = ctx->args();
    // the two projections are independent: one launch does both, and one
    // pair of launches scans both slot-run counts into offsets
    TIMED(ctx, GES_STAGE_PROJECT, s, launch_project(a, s));
    uint32_t *gb = (uint32_t *)(w + L.g_boff), *sb = (uint32_t *)(w + L.s_boff);
    const ScanJob jg{gb, 1, gb, (int64_t)L.n_views * L.m, (uint32_t *)(w + L.scan_tmp2), &hdr->g_slots};
    const ScanJob js{sb, 1, sb, (int64_t)n_views * surfels->n, (uint32_t *)(w + L.scan_tmp), &hdr->s_slots};
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s, launch_scan2_u32(jg, js, L.scan_blocks, s));
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s, launch_surfel_count(a, s));
    ctx->stage = 1;
    return GES_OK;
}

}  // namespace

ges_status ges_project(ges_context *ctx, const ges_camera *cams, int32_t n_views, const ges_surfels *surfels,
                       const ges_gaussians *gaussians, const ges_options *opt, void *ws, size_t ws_bytes,
                       void *stream) {
    return project_frame(ctx, cams, n_views, surfels, gaussians, opt, ws, ws_bytes, stream, false, nullptr, 0);
}

ges_status ges_raster_surfels(ges_context *ctx, int32_t *surfel_id, float *depth, float *color_s, void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 1 || ctx->translucent) return fail(GES_ERR_STATE, "ges_raster_surfels before ges_project");
    if (!surfel_id || !depth || !color_s) return fail(GES_ERR_ARG, "output pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const WsLayout &L = ctx->L;
    unsigned char *w = ctx->ws;
    WsHeader *hdr = (WsHeader *)(w + L.header);
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s,
          launch_scan_u32((const uint32_t *)(w + L.s_tcnt), kCounterStride, (uint32_t *)(w + L.s_toff),
                          (int64_t)L.rtiles * kCounterCopies,
                          (uint32_t *)(w + L.scan_tmp), L.scan_blocks, &hdr->s_pairs, s));
    const FrameArgs a = ctx->args();
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s, launch_surfel_fill(a, s));
    // with 4 samples per pixel the sample depths go to the workspace and the
    // resolve writes the pixel depth
    float *sdepth = ctx->opt.surfel_samples == 4 ? (float *)(w + L.s_depth) : depth;
    TIMED(ctx, GES_STAGE_RASTER, s, launch_raster(a, surfel_id, sdepth, ctx->cus, s));
    TIMED(ctx, GES_STAGE_SHADE, s, launch_shade(a, s));
    TIMED(ctx, GES_STAGE_RESOLVE, s, launch_resolve(a, surfel_id, sdepth, depth, color_s, s));
    ctx->stage = 2;
    return GES_OK;
}

ges_status ges_splat_gaussians(ges_context *ctx, const float *depth, const float *color_s, float *image,
                               float *accum, void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 2 || ctx->translucent) return fail(GES_ERR_STATE, "ges_splat_gaussians before ges_raster_surfels");
    if (!depth || !color_s || !image || !accum) return fail(GES_ERR_ARG, "buffer pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const WsLayout &L = ctx->L;
    unsigned char *w = ctx->ws;
    WsHeader *hdr = (WsHeader *)(w + L.header);
    {
        FillSet f{};
        f.p[0] = (uint32_t *)(w + L.g_tcnt);
        f.n[0] = (int64_t)L.stiles * kCounterStride;
        f.p[1] = (uint32_t *)(w + L.g_act);
        f.n[1] = L.m;
        f.count = 2;
        TIMED(ctx, GES_STAGE_CLEAR, s, launch_fill_set(f, s));
    }
    const FrameArgs a = ctx->args();
    TIMED(ctx, GES_STAGE_GAUSS_BIN, s, launch_gauss_count(a, s));
    TIMED(ctx, GES_STAGE_GAUSS_BIN, s,
          launch_scan_u32((const uint32_t *)(w + L.g_tcnt), kCounterStride, (uint32_t *)(w + L.g_toff), L.stiles,
                          (uint32_t *)(w + L.scan_tmp), L.scan_blocks, &hdr->g_pairs, s));
    TIMED(ctx, GES_STAGE_GAUSS_BIN, s, launch_gauss_fill(a, s));
    TIMED(ctx, GES_STAGE_SPLAT, s, launch_splat(a, depth, color_s, image, accum, s));
    ctx->stage = 3;
    return GES_OK;
}

ges_status ges_backward(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *color_s,
                        const float *accum, const float *d_image, const ges_gradients *grads, void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 3 || ctx->translucent) return fail(GES_ERR_STATE, "ges_backward before ges_splat_gaussians");
    if (ctx->G.dims == 2) return fail(GES_ERR_UNSUPPORTED, "ges_backward of 2D Gaussians (forward only)");
    if (!surfel_id || !depth || !color_s || !accum || !d_image || !grads)
        return fail(GES_ERR_ARG, "buffer pointer is NULL");
    if (ctx->G.m > 0 && (!grads->mean || !grads->quat || !grads->scale || !grads->opacity || !grads->sh))
        return fail(GES_ERR_ARG, "Gaussian gradient pointer is NULL");
    if (ctx->S.n > 0 && !grads->surfel_sh) return fail(GES_ERR_ARG, "surfel gradient pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    const FrameArgs a = ctx->args();
    hipStream_t s = (hipStream_t)stream;
    // Two chains, both latency-bound, on two streams.  Second stream: the
    // Gaussian active-list scan and the gradient zeroing/compaction (they
    // need only the forward's flags), then the surfel chain.  Caller's
    // stream: the Gaussian tile partials, then -- once the compaction is
    // done -- the Gaussian chain rule.  The two read the same frame state and
    // write disjoint regions.
    const WsLayout &L = ctx->L;
    unsigned char *w = ctx->ws;
    WsHeader *hdr = (WsHeader *)(w + L.header);
    HIP_TRY(ctx->ensure_aux());
    HIP_TRY(ctx->fork(s));
    hipStream_t sa = ctx->aux;
    // the forward's active flags stay untouched (scanned into their own
    // array), so the backward can run again on the same frame
    TIMED(ctx, GES_STAGE_BWD_GAUSS, sa,
          launch_scan_u32((const uint32_t *)(w + L.g_act), 1, (uint32_t *)(w + L.g_aoff), L.m,
                          (uint32_t *)(w + L.scan_tmp), L.scan_blocks, &hdr->g_active, sa));
    TIMED(ctx, GES_STAGE_BWD_GAUSS, sa, launch_bwd_compact(a, *grads, sa));
    HIP_TRY(hipEventRecord(ctx->ev_mid, sa));
    if (ctx->S.n > 0) {
        // surfel partials: only (surfel, tile) pairs that show the surfel are
        // written, the other slots must read zero
        TIMED(ctx, GES_STAGE_BWD_SURFEL_TILES, sa,
              launch_fill_u32_counted((uint32_t *)(w + L.s_part), 0u, &hdr->s_slots, 3, 3 * L.s_cap, sa));
    }
    TIMED(ctx, GES_STAGE_BWD_SURFEL_TILES, sa, launch_bwd_surfel_tiles(a, surfel_id, accum, d_image, sa));
    TIMED(ctx, GES_STAGE_BWD_SURFEL, sa, launch_bwd_surfels(a, *grads, sa));
    TIMED(ctx, GES_STAGE_BWD_TILES, s, launch_bwd_tiles(a, depth, color_s, accum, d_image, s));
    HIP_TRY(hipStreamWaitEvent(s, ctx->ev_mid, 0));
    TIMED(ctx, GES_STAGE_BWD_GAUSS, s, launch_bwd_gaussians(a, *grads, ctx->cus, s));
    HIP_TRY(ctx->join(s));
    return GES_OK;
}

ges_status ges_scores(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                      int32_t cover_min, float contrib_min, int32_t accumulate, const ges_scores_out *out,
                      void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 3 || ctx->translucent) return fail(GES_ERR_STATE, "ges_scores before ges_splat_gaussians");
    if (ctx->G.dims == 2) return fail(GES_ERR_UNSUPPORTED, "ges_scores of 2D Gaussians");
    if (ctx->opt.surfel_samples != 1) return fail(GES_ERR_UNSUPPORTED, "ges_scores with surfel_samples != 1");
    if (!surfel_id || !depth || !accum || !out) return fail(GES_ERR_ARG, "buffer pointer is NULL");
    if (ctx->S.n > 0 && !out->cover) return fail(GES_ERR_ARG, "cover is NULL");
    if (ctx->G.m > 0 && !out->contrib) return fail(GES_ERR_ARG, "contrib is NULL");
    if (!isfinite(contrib_min)) return fail(GES_ERR_ARG, "contrib_min not finite");
    HIP_TRY(hipSetDevice(ctx->device));
    return run_scores(ctx, surfel_id, depth, accum, cover_min, contrib_min, accumulate, out,
                      (uint32_t *)(ctx->ws + ctx->L.s_cnt), (hipStream_t)stream);
}

ges_status ges_translucent_workspace_query(const ges_camera *cams, int32_t n_views, int64_t n_surfels,
                                           const ges_options *opt, size_t *bytes) {
    if (!bytes) return fail(GES_ERR_ARG, "bytes is NULL");
    ges_status st = validate_cameras(cams, n_views);
    if (st) return st;
    if ((st = validate_options(opt))) return st;
    if (n_surfels < 0 || n_surfels > 0x7fffffffLL) return fail(GES_ERR_ARG, "bad surfel count");
    std::vector<ViewDev> views;
    int32_t rt, stl;
    int64_t pix;
    int a, b;
    build_views(cams, n_views, opt, views, rt, stl, pix, a, b);
    *bytes = make_layout(views, rt, stl, pix, n_surfels, 0, opt, true).total;
    return GES_OK;
}

ges_status ges_translucent_render(ges_context *ctx, const ges_camera *cams, int32_t n_views,
                                  const ges_surfels *surfels, const float *w, int32_t front_first,
                                  const ges_options *opt, void *ws, size_t ws_bytes, const ges_translucent_out *out,
                                  void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (!surfels || !out) return fail(GES_ERR_ARG, "surfels/out is NULL");
    if (!out->color || !out->alpha || !out->depth || !out->front) return fail(GES_ERR_ARG, "output pointer is NULL");
    if (surfels->n > 0 && !w) return fail(GES_ERR_ARG, "w is NULL");
    if (opt && opt->surfel_samples != 1) return fail(GES_ERR_UNSUPPORTED, "translucent surfels with surfel_samples != 1");
    ges_gaussians none{};
    none.sh_degree = 0;
    ges_status st = project_frame(ctx, cams, n_views, surfels, &none, opt, ws, ws_bytes, stream, true, w,
                                  front_first);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const WsLayout &L = ctx->L;
    unsigned char *wsp = ctx->ws;
    WsHeader *hdr = (WsHeader *)(wsp + L.header);
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s,
          launch_scan_u32((const uint32_t *)(wsp + L.s_tcnt), kCounterStride, (uint32_t *)(wsp + L.s_toff),
                          (int64_t)L.rtiles * kCounterCopies, (uint32_t *)(wsp + L.scan_tmp), L.scan_blocks,
                          &hdr->s_pairs, s));
    const FrameArgs a = ctx->args();
    TIMED(ctx, GES_STAGE_SURFEL_BIN, s, launch_surfel_fill(a, s));
    TIMED(ctx, GES_STAGE_SHADE, s, launch_shade(a, s));
    TIMED(ctx, GES_STAGE_RASTER, s, launch_tblend(a, out->color, out->alpha, out->depth, out->front, s));
    ctx->stage = kStageTranslucent;
    return GES_OK;
}

ges_status ges_translucent_backward(ges_context *ctx, const float *d_color, const ges_surfel_gradients *grads,
                                    void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage != kStageTranslucent || !ctx->translucent)
        return fail(GES_ERR_STATE, "ges_translucent_backward before ges_translucent_render");
    if (!d_color || !grads) return fail(GES_ERR_ARG, "d_color/grads is NULL");
    if (ctx->S.n > 0 && (!grads->mean || !grads->quat || !grads->scale || !grads->w || !grads->sh))
        return fail(GES_ERR_ARG, "surfel gradient pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const FrameArgs a = ctx->args();
    TIMED(ctx, GES_STAGE_BWD_SURFEL_TILES, s, launch_tblend_bwd(a, d_color, s));
    TIMED(ctx, GES_STAGE_BWD_SURFEL, s,
          launch_tsurfels(a, grads->mean, grads->quat, grads->scale, grads->w, grads->sh, s));
    return GES_OK;
}

ges_status ges_mip_filter3d(const ges_camera *cams, int32_t n_views, const ges_gaussians *gaussians, float scale2,
                            float *out, void *stream) {
    ges_status st = validate_cameras(cams, n_views);
    if (st) return st;
    if (!gaussians) return fail(GES_ERR_ARG, "gaussians is NULL");
    if (gaussians->m < 0) return fail(GES_ERR_ARG, "negative Gaussian count");
    if (gaussians->m > 0 && (!gaussians->mean || !out)) return fail(GES_ERR_ARG, "mean/out is NULL");
    if (!(scale2 >= 0.f) || !isfinite(scale2)) return fail(GES_ERR_ARG, "scale2 must be finite and >= 0");
    HIP_TRY(launch_mip_filter3d(gaussians->mean, gaussians->m, cams, n_views, scale2, out, (hipStream_t)stream));
    return GES_OK;
}

ges_status ges_geometry(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                        const ges_geometry_out *out, void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 3 || ctx->translucent) return fail(GES_ERR_STATE, "ges_geometry before ges_splat_gaussians");
    if (ctx->opt.surfel_samples != 1) return fail(GES_ERR_UNSUPPORTED, "ges_geometry with surfel_samples != 1");
    if (!surfel_id || !depth || !accum || !out) return fail(GES_ERR_ARG, "buffer pointer is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    if (!out->normal_s && !out->depth_g && !out->normal_g && !out->depth_smooth && !out->normal_smooth)
        return GES_OK;
    HIP_TRY(launch_geometry(ctx->args(), surfel_id, depth, accum, *out, (hipStream_t)stream));
    return GES_OK;
}

ges_status ges_scores_static(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                             int32_t cover_min, float contrib_min, int32_t accumulate, const ges_scores_out *out,
                             void *stream) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    if (ctx->stage < 3 || ctx->translucent) return fail(GES_ERR_STATE, "ges_scores_static before ges_splat_gaussians");
    if (ctx->G.dims == 2) return fail(GES_ERR_UNSUPPORTED, "ges_scores_static of 2D Gaussians");
    if (ctx->opt.surfel_samples != 1) return fail(GES_ERR_UNSUPPORTED, "ges_scores_static with surfel_samples != 1");
    if (!surfel_id || !depth || !accum || !out) return fail(GES_ERR_ARG, "buffer pointer is NULL");
    if (ctx->S.n > 0 && !out->cover) return fail(GES_ERR_ARG, "cover is NULL");
    if (ctx->G.m > 0 && !out->contrib) return fail(GES_ERR_ARG, "contrib is NULL");
    if (!isfinite(contrib_min)) return fail(GES_ERR_ARG, "contrib_min not finite");
    if (ctx->S.n > kStaticScoreWords)
        return fail(GES_ERR_ARG, "ges_scores_static: %lld surfels exceed its scratch of %lld (use ges_scores)",
                    (long long)ctx->S.n, (long long)kStaticScoreWords);
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(GES_ERR_ARG, "device %d out of range", ctx->device);
    HIP_TRY(hipSetDevice(ctx->device));
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[ctx->device]) {
            // with this device current: its own copy of the array
            HIP_TRY(hipGetSymbolAddress(&g_scratch_ptr[ctx->device], HIP_SYMBOL(scratch)));
        }
        ptr = g_scratch_ptr[ctx->device];
    }
    return run_scores(ctx, surfel_id, depth, accum, cover_min, contrib_min, accumulate, out, (uint32_t *)ptr,
                      (hipStream_t)stream);
}

// Return code and message for a frame status read back from the device.
static ges_status status_result(const ges_context *ctx, const ges_run_status *out) {
    if (out->flags & (kFlagSurfelOverflow | kFlagGaussOverflow))
        return fail(GES_ERR_CAPACITY, "list capacity exceeded: surfel pairs %lld (cap %lld), Gaussian pairs %lld (cap %lld)",
                    (long long)out->surfel_pairs, (long long)ctx->L.s_cap, (long long)out->gauss_pairs,
                    (long long)ctx->L.g_cap);
    if (out->flags & kFlagColourRange)
        return fail(GES_ERR_CAPACITY, "a Gaussian colour reached the fixed-point range limit (127)");
    return GES_OK;
}

static ges_status enqueue_status(ges_context *ctx, hipStream_t s) {
    unsigned char *w = ctx->ws;
    HIP_TRY(launch_status((const WsHeader *)(w + ctx->L.header), ctx->L.s_cap, ctx->L.g_cap, ctx->stage >= 3 ? 1 : 0,
                          (ges_run_status *)(w + ctx->L.status), s));
    return GES_OK;
}

ges_status ges_poll_status(ges_context *ctx, void *stream, ges_run_status *out) {
    if (!ctx || !out) return fail(GES_ERR_ARG, "ctx/out is NULL");
    memset(out, 0, sizeof *out);
    if (ctx->stage < 1) return fail(GES_ERR_STATE, "no frame to poll");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ges_status st = enqueue_status(ctx, s);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(out, ctx->ws + ctx->L.status, sizeof *out, hipMemcpyDeviceToHost));
    return status_result(ctx, out);
}

ges_status ges_poll_status_async(ges_context *ctx, void *stream, ges_run_status *host_out) {
    if (!ctx || !host_out) return fail(GES_ERR_ARG, "ctx/host_out is NULL");
    if (ctx->stage < 1) return fail(GES_ERR_STATE, "no frame to poll");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    ges_status st = enqueue_status(ctx, s);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(host_out, ctx->ws + ctx->L.status, sizeof *host_out, hipMemcpyDeviceToHost, s));
    return GES_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plans: autotune, size, capture one frame into a graph, replay

struct ges_plan {
    int device = 0;
    ges_context *ctx = nullptr;
    std::vector<ges_camera> cams;
    ges_surfels S;
    ges_gaussians G;
    ges_options opt;
    ges_frame_buffers buf;
    bool backward = false;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};

namespace {

ges_status run_frame(ges_plan *p, hipStream_t s) {
    ges_status st;
    if ((st = ges_project(p->ctx, p->cams.data(), (int32_t)p->cams.size(), &p->S, &p->G, &p->opt, p->ws,
                          p->ws_bytes, s)))
        return st;
    if ((st = ges_raster_surfels(p->ctx, p->buf.surfel_id, p->buf.depth, p->buf.color_s, s))) return st;
    if ((st = ges_splat_gaussians(p->ctx, p->buf.depth, p->buf.color_s, p->buf.image, p->buf.accum, s))) return st;
    if (p->backward)
        if ((st = ges_backward(p->ctx, p->buf.surfel_id, p->buf.depth, p->buf.color_s, p->buf.accum,
                               p->buf.d_image, &p->buf.grads, s)))
            return st;
    return GES_OK;
}

ges_status plan_alloc(ges_plan *p) {
    if (p->ws) {
        HIP_TRY(hipFree(p->ws));
        p->ws = nullptr;
    }
    size_t bytes = 0;
    ges_status st = ges_workspace_query(p->cams.data(), (int32_t)p->cams.size(), p->S.n, p->G.m, &p->opt, &bytes);
    if (st) return st;
    HIP_TRY(hipMalloc(&p->ws, bytes));
    p->ws_bytes = bytes;
    return GES_OK;
}

// Runs checked frames until the list capacities fit (x1.25 headroom).
ges_status plan_size(ges_plan *p, hipStream_t s) {
    for (int attempt = 0; attempt < 6; ++attempt) {
        ges_status st = plan_alloc(p);
        if (st) return st;
        if ((st = run_frame(p, s))) return st;
        ges_run_status rs;
        st = ges_poll_status(p->ctx, s, &rs);
        const int64_t ns = rs.surfel_pairs > rs.surfel_slots ? rs.surfel_pairs : rs.surfel_slots;
        const int64_t ng = rs.gauss_pairs > rs.gauss_slots ? rs.gauss_pairs : rs.gauss_slots;
        if (st == GES_OK) {
            // keep headroom for later pose changes
            const int64_t want_s = ns + ns / 4 + 4096, want_g = ng + ng / 4 + 4096;
            if (p->opt.surfel_pair_capacity >= want_s && p->opt.gauss_pair_capacity >= want_g) return GES_OK;
            p->opt.surfel_pair_capacity = want_s < 0x7fffffffLL ? want_s : 0x7fffffffLL;
            p->opt.gauss_pair_capacity = want_g < 0x7fffffffLL ? want_g : 0x7fffffffLL;
            continue;
        }
        if (st != GES_ERR_CAPACITY || (rs.flags & kFlagColourRange)) return st;
        p->opt.surfel_pair_capacity = ns + ns / 4 + 4096 < 0x7fffffffLL ? ns + ns / 4 + 4096 : 0x7fffffffLL;
        p->opt.gauss_pair_capacity = ng + ng / 4 + 4096 < 0x7fffffffLL ? ng + ng / 4 + 4096 : 0x7fffffffLL;
    }
    return fail(GES_ERR_CAPACITY, "plan: list capacities did not converge");
}

std::string tune_key(const ges_plan *p) {
    hipDeviceProp_t prop;
    std::string dev = "gpu";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = prop.gcnArchName;
    std::string k = dev + "|";
    for (const auto &c : p->cams) k += std::to_string(c.width) + "x" + std::to_string(c.height) + ",";
    k += "|" + std::to_string(p->S.n) + "|" + std::to_string(p->G.m) + (p->backward ? "|bwd" : "|fwd");
    return k;
}

bool cache_lookup(const std::string &key, ges_options *o) {
    const char *path = getenv("GES_AUTOTUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string needle = "\"key\": \"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, needle.c_str())) continue;
        int rt, tw, th, tq = 0;
        const char *q = strstr(line, "\"raster_tile\":");
        const char *r = strstr(line, "\"splat_tile_w\":");
        const char *t = strstr(line, "\"splat_tile_h\":");
        const char *u = strstr(line, "\"tile_queue\":");
        if (q && r && t && sscanf(q, "\"raster_tile\": %d", &rt) == 1 && sscanf(r, "\"splat_tile_w\": %d", &tw) == 1 &&
            sscanf(t, "\"splat_tile_h\": %d", &th) == 1) {
            if (u) (void)sscanf(u, "\"tile_queue\": %d", &tq);
            o->raster_tile = rt;
            o->splat_tile_w = tw;
            o->splat_tile_h = th;
            o->tile_queue = tq;
            found = true;  // the last matching line wins
        }
    }
    fclose(f);
    return found && validate_options(o) == GES_OK;
}

void cache_store(const std::string &key, const ges_options &o, double ms) {
    const char *path = getenv("GES_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"key\": \"%s\", \"raster_tile\": %d, \"splat_tile_w\": %d, \"splat_tile_h\": %d, "
            "\"tile_queue\": %d, \"ms\": %.5f}\n",
            key.c_str(), o.raster_tile, o.splat_tile_w, o.splat_tile_h, o.tile_queue, ms);
    fclose(f);
}

// Mean ms of `reps` frames after `warm` untimed ones (HIP events on s).
ges_status time_frames(ges_plan *p, hipStream_t s, int warm, int reps, double *ms) {
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    ges_status st = GES_OK;
    for (int k = 0; k < warm && !st; ++k) st = run_frame(p, s);
    if (!st) (void)hipEventRecord(a, s);
    for (int k = 0; k < reps && !st; ++k) st = run_frame(p, s);
    if (!st) {
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, a, b);
        *ms = t / reps;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

void plan_free(ges_plan *p) {
    if (!p) return;
    if (p->pending && p->done) (void)hipEventSynchronize(p->done);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->ws) (void)hipFree(p->ws);
    if (p->ctx) ges_context_destroy(p->ctx);
    delete p;
}

}  // namespace

extern "C" {

ges_status ges_plan_create(ges_plan **out, int device, const ges_camera *cams, int32_t n_views,
                           const ges_surfels *surfels, const ges_gaussians *gaussians, const ges_options *opt,
                           const ges_frame_buffers *buffers, int flags, void *stream) {
    if (!out) return fail(GES_ERR_ARG, "out is NULL");
    *out = nullptr;
    ges_status st;
    if ((st = validate_cameras(cams, n_views))) return st;
    if ((st = validate_options(opt))) return st;
    if ((st = validate_scene(surfels, gaussians))) return st;
    if (!buffers || !buffers->surfel_id || !buffers->depth || !buffers->color_s || !buffers->image || !buffers->accum)
        return fail(GES_ERR_ARG, "plan output buffer is NULL");
    if ((st = validate_gauss2d(gaussians, opt))) return st;
    if (gaussians->dims == 2 && buffers->d_image)
        return fail(GES_ERR_UNSUPPORTED, "a backward plan of 2D Gaussians (forward only)");
    ges_plan *p = new ges_plan();
    p->device = device;
    if ((st = ges_context_create(&p->ctx, device))) {
        delete p;
        return st;
    }
    p->cams.assign(cams, cams + n_views);
    p->S = *surfels;
    p->G = *gaussians;
    p->opt = *opt;
    p->buf = *buffers;
    p->backward = buffers->d_image != nullptr;
    hipStream_t s = (hipStream_t)stream;
    auto bail = [&](ges_status e) {
        const std::string msg = g_err;
        plan_free(p);
        g_err = msg;
        return e;
    };
    if (hipSetDevice(device) != hipSuccess) return bail(fail(GES_ERR_HIP, "hipSetDevice(%d) failed", device));

    // candidate tile shapes
    std::vector<ges_options> cand;
    const std::string key = tune_key(p);
    ges_options cached = *opt;
    if ((flags & GES_PLAN_AUTOTUNE) && cache_lookup(key, &cached)) {
        cand.push_back(cached);
    } else if (flags & GES_PLAN_AUTOTUNE) {
        const int rts[2] = {8, 16};
        const int sts[3][2] = {{8, 8}, {16, 8}, {16, 16}};
        // pass 1 as one block per tile, or persistent at the occupancy the
        // raster reaches (8 blocks of 256 per CU at 16x16 tiles, 24 of 64 at 8x8)
        for (int r : rts)
            for (auto &t : sts)
                for (int tq : {0, r == 16 ? 8 : 24}) {
                    ges_options o = *opt;
                    o.raster_tile = r;
                    o.splat_tile_w = t[0];
                    o.splat_tile_h = t[1];
                    o.tile_queue = tq;
                    cand.push_back(o);
                }
    } else {
        cand.push_back(*opt);
    }
    double best_ms = 1e30;
    ges_options best = cand[0];
    if (cand.size() > 1) {
        for (const auto &c : cand) {
            p->opt = c;
            if ((st = plan_size(p, s))) return bail(st);
            double ms = 0;
            if ((st = time_frames(p, s, 2, 5, &ms))) return bail(st);
            if (ms < best_ms) {
                best_ms = ms;
                best = p->opt;
            }
        }
    }
    p->opt = best;
    if ((st = plan_size(p, s))) return bail(st);
    if (cand.size() > 1) cache_store(key, p->opt, best_ms);

    // capture the frame into a graph on a private stream (the context's
    // second stream exists before capture: its fork becomes a graph branch)
    if (p->ctx->ensure_aux() != hipSuccess) return bail(fail(GES_ERR_HIP, "stream creation failed"));
    if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(GES_ERR_HIP, "stream creation failed"));
    if (hipStreamSynchronize(s) != hipSuccess) return bail(fail(GES_ERR_HIP, "stream sync failed"));
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(GES_ERR_HIP, "hipStreamBeginCapture failed"));
    p->ctx->capturing = true;
    st = run_frame(p, p->cap_stream);
    p->ctx->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return bail(st);
    }
    if (ce != hipSuccess || !g) return bail(fail(GES_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ce)));
    p->graph = g;
    const hipError_t ie = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) return bail(fail(GES_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ie)));
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess)
        return bail(fail(GES_ERR_HIP, "event creation failed"));
    // the view table the replays read (the graph does not copy it)
    memcpy(p->ctx->pinned[0], p->ctx->views.data(), sizeof(ViewDev) * p->ctx->views.size());
    if (hipMemcpyAsync(p->ctx->ws + p->ctx->L.views, p->ctx->pinned[0], sizeof(ViewDev) * p->ctx->views.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(GES_ERR_HIP, "view table upload failed"));
    *out = p;
    return GES_OK;
}

ges_status ges_plan_launch(ges_plan *p, const ges_camera *cams, void *stream) {
    if (!p) return fail(GES_ERR_ARG, "plan is NULL");
    HIP_TRY(hipSetDevice(p->device));
    if (cams) {
        const int nv = (int)p->cams.size();
        ges_status st = validate_cameras(cams, nv);
        if (st) return st;
        for (int v = 0; v < nv; ++v)
            if (cams[v].width != p->cams[v].width || cams[v].height != p->cams[v].height)
                return fail(GES_ERR_ARG, "plan view %d: size %dx%d differs from %dx%d", v, cams[v].width,
                            cams[v].height, p->cams[v].width, p->cams[v].height);
        std::vector<ViewDev> views;
        int32_t rt, stl;
        int64_t pix;
        int a, b;
        build_views(cams, nv, &p->opt, views, rt, stl, pix, a, b);
        // upload through the context's staging buffers, used in turn (the
        // host waits only if a buffer's earlier upload has not run yet); the
        // upload runs in stream order, after any replay still running here
        ges_context *ctx = p->ctx;
        const int slot = ctx->next_staging;
        ctx->next_staging = (slot + 1) % ges_context::kStaging;
        if (!ctx->copied[slot]) HIP_TRY(hipEventCreateWithFlags(&ctx->copied[slot], hipEventDisableTiming));
        if (ctx->copy_pending[slot]) {
            HIP_TRY(hipEventSynchronize(ctx->copied[slot]));
            ctx->copy_pending[slot] = false;
        }
        memcpy(ctx->pinned[slot], views.data(), sizeof(ViewDev) * nv);
        HIP_TRY(hipMemcpyAsync(ctx->ws + ctx->L.views, ctx->pinned[slot], sizeof(ViewDev) * nv,
                               hipMemcpyHostToDevice, (hipStream_t)stream));
        HIP_TRY(hipEventRecord(ctx->copied[slot], (hipStream_t)stream));
        ctx->copy_pending[slot] = true;
        p->cams.assign(cams, cams + nv);
        p->ctx->views = views;
    }
    HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
    HIP_TRY(hipEventRecord(p->done, (hipStream_t)stream));
    p->pending = true;
    return GES_OK;
}

ges_status ges_plan_options(const ges_plan *p, ges_options *out) {
    if (!p || !out) return fail(GES_ERR_ARG, "plan/out is NULL");
    *out = p->opt;
    return GES_OK;
}

ges_status ges_plan_poll(ges_plan *p, void *stream, ges_run_status *out) {
    if (!p) return fail(GES_ERR_ARG, "plan is NULL");
    return ges_poll_status(p->ctx, stream, out);
}

ges_status ges_plan_destroy(ges_plan *p) {
    plan_free(p);
    return GES_OK;
}

ges_status ges_profile_enable(ges_context *ctx, int enable) {
    if (!ctx) return fail(GES_ERR_ARG, "ctx is NULL");
    ctx->profile = enable != 0;
    return GES_OK;
}

ges_status ges_profile_read(ges_context *ctx, double *ms, int64_t *launches, int reset) {
    if (!ctx || !ms) return fail(GES_ERR_ARG, "ctx/ms is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    for (auto &p : ctx->pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, p.a, p.b));
        ctx->stage_ms[p.stage] += t;
        ctx->stage_n[p.stage] += 1;
        ctx->free_events.push_back(p.a);
        ctx->free_events.push_back(p.b);
    }
    ctx->pending.clear();
    for (int k = 0; k < GES_STAGE_COUNT; ++k) {
        ms[k] = ctx->stage_ms[k];
        if (launches) launches[k] = ctx->stage_n[k];
        if (reset) {
            ctx->stage_ms[k] = 0.0;
            ctx->stage_n[k] = 0;
        }
    }
    return GES_OK;
}

}  // extern "C"
