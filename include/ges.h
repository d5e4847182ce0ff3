/*
 * ges.h -- C ABI of the MI355X (gfx950) render library for Gaussian-enhanced
 * surfels (Ye, Shao, Zhou, "When Gaussian Meets Surfel: Ultra-fast
 * High-fidelity Radiance Field Rendering", ACM TOG 44(4), 2025).
 *
 * The library computes the paper's two-pass, sorting-free render and its
 * gradient:
 *   pass 1 (Sec. 3): opaque 2D surfels, z-buffered, give the surfel id map,
 *          the depth map D_s and the colour map C_s (Eq. 1 colours);
 *   pass 2 (Sec. 3, Eq. 2-4): 3D Gaussians are splatted, depth-tested per
 *          pixel against D_s + eps_i (eps_i = 5/3 sum s, Sec. 5) and
 *          accumulated order-independently into C_G, W_G;
 *   composite (Eq. 5): C = (W_s C_s + C_G) / (W_s + W_G), W_s = 1;
 *   backward: gradients of a loss w.r.t. the parameters the joint stage of
 *          Sec. 4.2 optimises (Gaussian p, r, s, sigma, SH; surfel SH).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every pointer argument named as device memory is a device pointer
 *   owned by the caller (the library never allocates or frees it).  Host
 *   structs are read during the call only.  All arrays are float32,
 *   structure-of-arrays with the primitive index fastest: a "[3][n]" array
 *   holds x[0..n), y[0..n), z[0..n) back to back.
 * Views.  A call renders n_views cameras at once.  Per-pixel outputs are the
 *   views' images concatenated in view order; within a view a "[c][H][W]"
 *   image is row-major with channels outermost.  P_v = W_v * H_v.
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Every call
 *   only enqueues work on it and returns; nothing synchronises except
 *   ges_poll_status.  One context serves one stream at a time.
 * Errors.  No call aborts or throws.  A non-zero ges_status is returned and
 *   ges_last_error() describes it (thread-local, valid until the next call on
 *   that thread).  Argument errors are detected on the host before anything
 *   is enqueued.  Capacity overflow of the per-tile lists is detected on the
 *   device: the launch's outputs are then invalid and ges_poll_status reports
 *   GES_ERR_CAPACITY with the sizes needed.
 * Order of calls per frame: ges_project -> ges_raster_surfels ->
 *   ges_splat_gaussians -> (optionally) ges_backward, all with the same
 *   context and workspace; the workspace must stay untouched in between.
 */
#ifndef GES_H
#define GES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ges_status {
    GES_OK = 0,
    GES_ERR_ARG = 1,          /* invalid argument (host check)                  */
    GES_ERR_WORKSPACE = 2,    /* workspace missing or smaller than required     */
    GES_ERR_CAPACITY = 3,     /* per-tile list capacity exceeded (device check) */
    GES_ERR_HIP = 4,          /* a HIP runtime call failed                      */
    GES_ERR_UNSUPPORTED = 5,  /* option value not built into this library       */
    GES_ERR_STATE = 6         /* entry points called out of order               */
} ges_status;

/* Pinhole camera.  World -> camera x_c = R x_w + t (R row-major), OpenCV axes
 * (x right, y down, z forward).  Pixel (i, j) has its centre at
 * (i + 0.5, j + 0.5) and images the camera-space ray ((i+.5-cx)/fx,
 * (j+.5-cy)/fy, 1).  Depth is camera-space z.  znear > 0 culls Gaussian
 * centres with z <= znear and surfel hits with z < znear.  bg is the colour
 * C_s of pixels no surfel covers.  1 <= width, height <= 16384. */
typedef struct ges_camera {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float znear;
    float bg[3];
} ges_camera;

/* Surfels S = {p, r, s, SH} (Sec. 3): a disc of radius
 * options.surfel_radius on the local XY plane, scaled by s = (s_u, s_v),
 * rotated by the quaternion r (w,x,y,z; normalised inside) and translated
 * to p.  Device arrays: mean [3][n], quat [4][n], scale [2][n] (> 0),
 * sh [n][K][3] with K = (sh_degree + 1)^2, 0 <= sh_degree <= 3 (degree 0 is
 * the paper's "RGB surfels" ablation).  n == 0 is legal (pointers unused).
 * The SH is per surfel (its 3K coefficients contiguous): colour is
 * evaluated only for surfels that win a pixel, a small fraction of them in
 * a dense scene, and a surfel-major layout reads only their coefficients. */
typedef struct ges_surfels {
    int64_t n;
    int32_t sh_degree;
    int32_t reserved;
    const float *mean, *quat, *scale, *sh;
} ges_surfels;

/* 3D Gaussians G = {p, sigma, r, s, SH} (Sec. 3).  Device arrays:
 * mean [3][m], quat [4][m] (w,x,y,z), scale [3][m] (> 0), opacity [m]
 * (sigma in (0, 1]), sh [m][K][3].  Parameters are activated values: no
 * exp/sigmoid is applied inside.  m == 0 is legal.  The SH is per Gaussian,
 * as for surfels: colour is evaluated only for Gaussians that keep a list
 * entry after the depth cull, and the backward reads the coefficients of
 * those Gaussians only. */
typedef struct ges_gaussians {
    int64_t m;
    int32_t sh_degree;
    int32_t dims;           /* 0 or 3: 3D Gaussians, scale [3][m] (Sec. 3).
                               2: the 2D Gaussians of 2D-GES (Sec. 6.4),
                               scale [2][m]: planar splats whose rotation's
                               third axis is the normal; alpha = opacity
                               exp(-(u^2 + v^2)/2) at the pixel ray's hit on
                               the plane ((u, v) in units of the scales),
                               the depth test on that hit's camera depth
                               (planar depth) with eps = eps_factor / 2 x
                               (s_u + s_v); D_G and N_G of ges_geometry take
                               the planar depth and the normal.  Forward
                               only: ges_backward, ges_scores(_static) and
                               backward plans return GES_ERR_UNSUPPORTED, as
                               do filter3d and mip_2d                        */
    const float *mean, *quat, *scale, *opacity, *sh;
    const float *filter3d;  /* [m] or NULL: Mip-GES world-space filter (Sec.
                               6.1): Sigma3 + filter3d_i I, opacity times
                               sqrt(det Sigma3 / det(Sigma3 + filter3d_i I));
                               a fixed input (no gradient), e.g. from
                               ges_mip_filter3d */
} ges_gaussians;

/* Render options.  ges_options_default fills the paper's values. */
typedef struct ges_options {
    float surfel_radius;  /* opaque disc radius in scaled units: sqrt(2 ln 255)
                             (Sec. 4.1, after Eq. 7)                          */
    float eps_factor;     /* eps_i = eps_factor / 3 * sum_j s_ij (Sec. 5: 5)  */
    float eps_const;      /* >= 0: use this eps for every Gaussian instead
                             (the eps = 0 and eps = 0.1 ablations, Table 5)   */
    float alpha_min;      /* alpha below this is zero (Sec. 3 after Eq. 4)    */
    float dilation;       /* added to the projected 2D covariance (0.3)       */
    float w_s;            /* surfel weight W_s of Eq. 5 (1)                   */
    int32_t raster_tile;  /* square surfel raster tile edge: 8 or 16          */
    int32_t splat_tile_w; /* Gaussian splat tile: 8x8, 16x8 or 16x16          */
    int32_t splat_tile_h;
    int32_t tile_queue;   /* 0: pass 1 launches one block per raster tile;
                             k in 1..32: a persistent pass 1 of k blocks per
                             CU taking tiles from per-XCD work queues (same
                             results; a tuning choice)                        */
    int64_t surfel_pair_capacity;  /* (surfel, tile) list entries; 0 = auto;
                                      at most 2^29 - 1 (larger is clamped)  */
    int64_t gauss_pair_capacity;   /* (Gaussian, tile) list entries; 0 = auto */
    int32_t surfel_samples;        /* 1, or 4: pass 1 supersampled 2x2 (Sec. 5,
                                      the 4x surfel sampling of Mip-GES): the
                                      surfel id map has one entry per sample,
                                      C_s is the samples' mean colour and D_s
                                      the mean depth of the samples that hit */
    float mip_2d;                  /* > 0: Mip-GES screen-space filter (Sec.
                                      6.1): Sigma2 + mip_2d I in place of the
                                      dilation, opacity times sqrt(det Sigma2 /
                                      det(Sigma2 + mip_2d I)); 0: dilation     */
} ges_options;

/* Device-side status of the last frame, filled by ges_poll_status. */
typedef struct ges_run_status {
    uint32_t flags;               /* bit 0: surfel list overflow, bit 1:
                                     Gaussian list overflow, bit 2: a colour
                                     exceeded the fixed-point range (>= 127),
                                     bit 3: a translucent tile list exceeded
                                     the blend's sort capacity */
    uint32_t reserved;
    int64_t surfel_pairs;         /* (surfel, raster tile) list entries       */
    int64_t gauss_pairs;          /* (Gaussian, splat tile) list entries      */
    int64_t surfel_slots;         /* raster tiles inside the surfel boxes     */
    int64_t gauss_slots;          /* splat tiles inside the Gaussian boxes    */
    int64_t surfel_box_pixels;    /* pixels of the surfel entries' boxes
                                     clipped to their tiles, over the entries
                                     pass 1 evaluated (the ones its occlusion
                                     cull kept; 0 before rasterisation)      */
    int64_t gauss_box_pixels;     /* the same for the kept Gaussian entries
                                     (0 before ges_splat_gaussians)          */
    int64_t visible_surfels;      /* surfels that won at least one pixel,
                                     summed over views (0 before
                                     ges_raster_surfels)                     */
    int64_t active_gaussians;     /* Gaussians with a list entry in some view
                                     (set by ges_backward, 0 before it)      */
    /* a capacity option must be at least max(pairs, slots) of its kind */
} ges_run_status;

typedef struct ges_context ges_context;

/* Fills *opt with the defaults above (raster 8x8, splat 16x16). */
void ges_options_default(ges_options *opt);

/* Creates a context on HIP device `device`.  The context holds host-side
 * state of one frame (cameras, scene descriptors, workspace layout); it
 * allocates no device memory.  Returns GES_ERR_HIP if the device does not
 * exist. */
ges_status ges_context_create(ges_context **out, int device);
ges_status ges_context_destroy(ges_context *ctx);

/* Bytes of device workspace a frame with these cameras, primitive counts and
 * options needs (forward and backward).  Host only; touches no device.
 * cams: host array of n_views cameras (1 <= n_views <= 1024). */
ges_status ges_workspace_query(const ges_camera *cams, int32_t n_views, int64_t n, int64_t m,
                               const ges_options *opt, size_t *bytes);

/* Number of pixels of the views (sum of width*height), for sizing outputs. */
ges_status ges_total_pixels(const ges_camera *cams, int32_t n_views, int64_t *pixels);

/* ges_project -- per-primitive set-up of one frame (all views).
 * Gaussians (Eq. 4 and the text after it): camera-space centre, culling at
 *   znear, projected covariance J W Sigma W^T J^T + dilation I with the
 *   3DGS Jacobian (x/z, y/z clamped to 1.3 x the half field of view),
 *   projected centre p_hat, centre depth d_i, eps_i, SH colour in the
 *   direction centre -> camera (Eq. 1), and the pixel bounding box of the
 *   ellipse alpha >= alpha_min.
 * Surfels (Sec. 3): camera-space disc frame, the exact bounding box of the
 *   projected disc, and the count of raster tiles it touches.
 * The scene arrays are read here and again by ges_backward: they must stay
 * valid and unchanged until the frame's last call.  `ws` is a device buffer
 * of at least ges_workspace_query bytes, owned by the caller.  cams and opt
 * are host pointers copied into the context. */
ges_status ges_project(ges_context *ctx, const ges_camera *cams, int32_t n_views,
                       const ges_surfels *surfels, const ges_gaussians *gaussians,
                       const ges_options *opt, void *ws, size_t ws_bytes, void *stream);

/* ges_raster_surfels -- pass 1 (Sec. 3): software z-buffer of the opaque
 * surfels.  Each pixel shows the nearest surfel whose disc (u^2 + v^2 <= R^2,
 * inclusive) its ray hits at z >= znear; an exact depth tie goes to the
 * smaller surfel index.  Outputs (device, caller-owned, concatenated views):
 *   surfel_id [sum P_v] int32, -1 where no surfel;
 *   depth     [sum P_v] float, D_s, +inf where no surfel;
 *   color_s   [sum 3 P_v] float, per view [3][H][W], C_s (bg where none).
 * With options.surfel_samples = 4 every pixel (i, j) is sampled at
 * (i + 1/4 + a/2, j + 1/4 + b/2), a, b in {0, 1} -- the pixel centres of the
 * view at twice its resolution -- and surfel_id holds [sum 4 P_v] entries,
 * per view a (2H) x (2W) grid in which sample (a, b) of pixel (i, j) is
 * entry (2j + b) * 2W + 2i + a; depth and color_s stay per pixel: the mean
 * depth of the samples that hit a surfel (+inf if none) and the mean of the
 * samples' colours. */
ges_status ges_raster_surfels(ges_context *ctx, int32_t *surfel_id, float *depth,
                              float *color_s, void *stream);

/* ges_splat_gaussians -- pass 2 and composite (Eq. 2-5).  Reads depth and
 * color_s written by ges_raster_surfels.  A Gaussian counts at a pixel iff
 * alpha >= alpha_min and d_i < D_s + eps_i.  C_G and W_G are summed in 2^-24
 * fixed point, so the result does not depend on the order of the Gaussian
 * array.  Outputs (device, caller-owned):
 *   image [sum 3 P_v] float, per view [3][H][W], C of Eq. 5;
 *   accum [sum 4 P_v] float, per view [4][H][W]: C_G (3 channels), W_G. */
ges_status ges_splat_gaussians(ges_context *ctx, const float *depth, const float *color_s,
                               float *image, float *accum, void *stream);

/* Gradient outputs of ges_backward (device, caller-owned, overwritten, summed
 * over the frame's views): layouts equal to the parameter arrays. */
typedef struct ges_gradients {
    float *mean;      /* [3][m] */
    float *quat;      /* [4][m] w.r.t. the unnormalised quaternion */
    float *scale;     /* [3][m] */
    float *opacity;   /* [m]    */
    float *sh;        /* [m][K][3] */
    float *surfel_sh; /* [n][K_s][3]; zero for surfels visible in no view */
} ges_gradients;

/* ges_backward -- gradient of L given dL/dC (d_image, same layout as image).
 * Differentiates Eq. 1-5 w.r.t. the Gaussian mean, quaternion, scale,
 * opacity and SH and the surfel SH.  The depth-test indicator, eps, the alpha
 * threshold, the SH clamp at zero and the surfel geometry carry no gradient.
 * Per-pixel terms are recomputed from the frame's saved state (surfel_id,
 * depth, color_s, accum) and summed per Gaussian and per surfel in a fixed
 * order (or exactly, in integers): the result is bitwise reproducible and
 * independent of the order of the Gaussian array.  It changes none of the
 * frame's state: it may be called again on the same frame (for another
 * d_image), with the same result for the same d_image.  Gradients are
 * written with non-temporal stores. */
ges_status ges_backward(ges_context *ctx, const int32_t *surfel_id, const float *depth,
                        const float *color_s, const float *accum, const float *d_image,
                        const ges_gradients *grads, void *stream);

/* ges_mip_filter3d -- per-Gaussian variance of the Mip-GES world-space
 * filter (Sec. 6.1, after Mip-Splatting): scale2 x (z / f_x)^2 of the
 * nearest of the n_views cameras (host array) whose image [0, W] x [0, H]
 * holds the Gaussian's projected centre with z > znear; 0 if none does
 * (0.2 is Mip-Splatting's scale2).  Reads gaussians->mean; writes out [m]
 * (device).  Asynchronous on `stream`; needs no context or workspace. */
ges_status ges_mip_filter3d(const ges_camera *cams, int32_t n_views, const ges_gaussians *gaussians, float scale2,
                            float *out, void *stream);

/* Outputs of ges_scores (device, caller-owned). */
typedef struct ges_scores_out {
    int32_t *cover;        /* [n] covering score n_i (required if n > 0)      */
    float *contrib;        /* [m] contribution score (required if m > 0)      */
    uint8_t *keep_surfel;  /* [n] or NULL: 1 iff cover[i] >= cover_min       */
    uint8_t *keep_gauss;   /* [m] or NULL: 1 iff contrib[i] >= contrib_min   */
} ges_scores_out;

/* ges_scores -- pruning scores of the rendered frame (all its views).
 * Surfels (Sec. 4.1, surfel pruning): n_{i,j} is the number of pixels of
 *   view j whose frontmost surfel is i, i.e. the pixels of surfel_id equal
 *   to i; cover[i] = max over the frame's views of n_{i,j} (an exact count).
 * Gaussians (Sec. 4.2, Eq. 9): s_{i,j} is the largest, over the pixels of
 *   view j where Gaussian i counts in pass 2 (alpha >= alpha_min and
 *   d_i < D_s + eps_i, the same FP32 decisions as ges_splat_gaussians), of
 *   c_{i,j} alpha / (W_s + W_G), with c_{i,j} the largest channel of its
 *   colour in view j and W_G from accum; 0 if it counts nowhere.
 *   contrib[i] = max over the frame's views of s_{i,j}.
 * The paper prunes surfels with n_i < n_thr (16 real, 4 synthetic scenes)
 *   and Gaussians with max_j s_{i,j} < 0.02; keep_* flag the complement.
 * accumulate != 0 folds this frame into the values already in cover and
 *   contrib (maximum), so the scores of many training views can be taken
 *   one frame at a time; 0 overwrites them.  The keep flags are computed
 *   from the folded values.
 * Inputs surfel_id, depth, accum are the frame's outputs of
 *   ges_raster_surfels and ges_splat_gaussians (unchanged since).  Maxima
 *   and integer sums do not depend on evaluation order: results are exact
 *   and reproducible.  Uses n words of the frame's workspace as scratch and
 *   changes nothing a later ges_backward reads.  Asynchronous on `stream`. */
ges_status ges_scores(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                      int32_t cover_min, float contrib_min, int32_t accumulate, const ges_scores_out *out,
                      void *stream);

/* ges_scores_static -- ges_scores for callers that cannot allocate device
 * memory (code under graph capture, serving loops that forbid allocation):
 * the same kernels and results, with the per-surfel counters in a device
 * array of the library (16 MiB per device, kept until the process ends)
 * instead of the frame's workspace.  Allocates nothing.  At most 4,194,304
 * surfels (n above that: GES_ERR_ARG, nothing enqueued).  Every call on a
 * device shares that device's array, left zeroed by each call: calls that
 * overlap on one device (on different streams, or from several threads)
 * race and their results are undefined.  Same arguments and ordering rules
 * as ges_scores. */
ges_status ges_scores_static(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                             int32_t cover_min, float contrib_min, int32_t accumulate, const ges_scores_out *out,
                             void *stream);

/* ------------------------------------------------------------------------
 * Translucent surfels of the surfel optimisation stage (Sec. 4.1, Eq. 6-7).
 * A surfel's opacity at the point (x, y) of its local plane (the disc's
 * coordinates scaled by s, as for the opaque pass) is alpha = min(1, w G),
 * G = exp(-(x^2 + y^2) / 2), zero where min(alpha, G) < 1/255; the surfels
 * that reach a pixel are alpha-blended front to back in the order of their
 * centre depth (camera z of the centre; smaller index on a tie), and with
 * front_first the pixel's nearest surfel with alpha > 0 (depth of the ray's
 * intersection; smaller index on a tie) is blended first, the others keeping
 * their order (the adjustment the paper applies once w > 30).  At w = 255
 * with front_first the colour is the opaque pass's C_s.
 * ------------------------------------------------------------------------ */

/* Outputs of ges_translucent_render (device, caller-owned, [c][H][W] planes
 * per view, views concatenated). */
typedef struct ges_translucent_out {
    float *color;    /* [sum 3 P_v] blended colour plus T_end times bg        */
    float *alpha;    /* [sum P_v]   1 - T_end                                 */
    float *depth;    /* [sum P_v]   sum_k alpha_k T_k z_k (not normalised)   */
    int32_t *front;  /* [sum P_v]   the surfel blended first with front_first, */
                     /*             else -1                                    */
} ges_translucent_out;

/* Gradients of ges_translucent_backward (device, caller-owned, written
 * whole): shaped like the surfel arrays; w like the w input. */
typedef struct ges_surfel_gradients {
    float *mean, *quat, *scale, *w, *sh;
} ges_surfel_gradients;

/* Workspace bytes of ges_translucent_render for these cameras and surfels. */
ges_status ges_translucent_workspace_query(const ges_camera *cams, int32_t n_views, int64_t n_surfels,
                                           const ges_options *opt, size_t *bytes);

/* Renders translucent surfels (w: [n] device, the opacity modulation of
 * each surfel, >= 0).  Uses the surfel binning of ges_project (raster
 * tiles; no occluders) and one blend kernel per raster tile that sorts the
 * tile's list in LDS (at most 2048 entries per tile: a longer list sets
 * status flag bit 3 and its tail is ignored).  options: surfel_samples must
 * be 1.  The context then holds a translucent frame (the opaque calls and
 * ges_backward refuse it).  Asynchronous on `stream`; errors as for
 * ges_project. */
ges_status ges_translucent_render(ges_context *ctx, const ges_camera *cams, int32_t n_views,
                                  const ges_surfels *surfels, const float *w, int32_t front_first,
                                  const ges_options *opt, void *ws, size_t ws_bytes, const ges_translucent_out *out,
                                  void *stream);

/* Gradients of sum_pixels d_color . color ([sum 3 P_v] device) with respect
 * to the surfels' mean, quat, scale, w and SH, for the last translucent
 * frame.  The sums are taken in fixed orders (reproducible).  Asynchronous on
 * `stream`; GES_ERR_STATE without a translucent frame. */
ges_status ges_translucent_backward(ges_context *ctx, const float *d_color, const ges_surfel_gradients *grads,
                                    void *stream);

/* Outputs of ges_geometry (device, caller-owned; any may be NULL).  Per
 * view [c][H][W] planes, views concatenated, like the image. */
typedef struct ges_geometry_out {
    float *normal_s;       /* [sum 3 P_v] N_s: the frontmost surfel's unit
                              normal, world space, facing the camera; 0 where
                              no surfel covers the pixel                       */
    float *depth_g;        /* [sum P_v]   D_G (Eq. 10)                         */
    float *normal_g;       /* [sum 3 P_v] N_G (Eq. 11)                         */
    float *depth_smooth;   /* [sum P_v]   D_smooth (Eq. 12)                    */
    float *normal_smooth;  /* [sum 3 P_v] N_smooth (Eq. 12)                    */
} ges_geometry_out;

/* ges_geometry -- geometry channels of the rendered frame (Sec. 6.4, the
 * depth and normal smoothing of 2D-GES, Eq. 10-12), for 3D Gaussians:
 *   D_G = sum of d_i alpha_i and N_G = sum of n_i alpha_i over the Gaussians
 *   that count at the pixel in pass 2 (the same FP32 alpha threshold and
 *   depth test as ges_splat_gaussians), with d_i the centre depth (camera
 *   z) and n_i the shortest axis (world space, facing the camera);
 *   D_smooth = (D_s W_s + D_G) / (W_s + W_G), N_smooth = (N_s W_s + N_G) /
 *   (W_s + W_G), with D_s W_s and N_s read as 0 where no surfel covers the
 *   pixel.
 * The sums are taken in 2^-24 fixed point: independent of the order of the
 * Gaussian array.  Inputs are the frame's outputs (unchanged since);
 * nothing of the frame's state is modified.  Asynchronous on `stream`. */
ges_status ges_geometry(ges_context *ctx, const int32_t *surfel_id, const float *depth, const float *accum,
                        const ges_geometry_out *out, void *stream);

/* Synchronises `stream` and reports the device-side status of the last
 * frame.  Returns GES_ERR_CAPACITY if a list overflowed (then raise the
 * capacities to at least the reported pair counts and render again). */
ges_status ges_poll_status(ges_context *ctx, void *stream, ges_run_status *out);

/* ges_poll_status without waiting: enqueues on `stream` the assembly of the
 * frame's status and its copy into *host_out, and returns.  host_out must be
 * pinned host memory (hipHostMalloc) that stays valid until the copy has run
 * (an event recorded on `stream` after this call tells when); its contents
 * are then what ges_poll_status would report (flags bit 0/1: list overflow,
 * bit 2: colour range), and the frame's outputs are invalid if any flag is
 * set.  For loops that must not synchronise every frame: check the status
 * of frame k once a later frame's work has been enqueued. */
ges_status ges_poll_status_async(ges_context *ctx, void *stream, ges_run_status *host_out);

/* Message of the last failed call on this thread ("" if none). */
const char *ges_last_error(void);

/* Stage timing.  When enabled, every kernel launch of the entry points above
 * is bracketed by a pair of hipEvents recorded on the call's stream; the
 * elapsed times are summed per stage.  Off by default (no events recorded). */
typedef enum ges_stage {
    GES_STAGE_PROJECT = 0,        /* Gaussian projection + surfel set-up (one
                                     launch)                                   */
    GES_STAGE_SURFEL_BIN,         /* slot scans, count, tile-offset scan, fill */
    GES_STAGE_RASTER,             /* pass-1 z-buffer                           */
    GES_STAGE_SHADE,              /* SH colour of visible surfels              */
    GES_STAGE_RESOLVE,            /* C_s per pixel + per-tile max depth        */
    GES_STAGE_GAUSS_BIN,          /* Gaussian count, scans, list fill          */
    GES_STAGE_SPLAT,              /* pass 2 + composite                        */
    GES_STAGE_BWD_TILES,          /* per-tile partials                         */
    GES_STAGE_BWD_GAUSS,          /* per-Gaussian chain rule                   */
    GES_STAGE_BWD_SURFEL,         /* per-surfel SH gradient                    */
    GES_STAGE_BWD_SURFEL_TILES,   /* per-tile surfel colour partials           */
    GES_STAGE_CLEAR,              /* counter / flag clears                     */
    GES_STAGE_COUNT
} ges_stage;

/* ------------------------------------------------------------------------
 * Plans: many views, forward (+ backward) as one replayable graph.
 *
 * Multi-view optimisation (Sec. 4) renders many calibrated views per step.
 * A plan fixes the views' sizes, the scene arrays, the output buffers and
 * the options, runs the tile-shape autotuner if asked, sizes the per-tile
 * lists from a checked trial frame (with 25% headroom), and captures the
 * whole frame -- every stage of every view -- into one hipGraph.  Each
 * stage is one launch over the flattened (view, tile) or (view, primitive)
 * index space of all views, so views of different resolution share every
 * launch.  ges_plan_launch replays the graph; camera poses and intrinsics
 * may change between launches, image sizes may not.
 * ------------------------------------------------------------------------ */
typedef struct ges_plan ges_plan;

/* Device buffers a plan writes and reads (caller-owned, fixed for the plan's
 * life).  d_image == NULL makes a forward-only plan. */
typedef struct ges_frame_buffers {
    int32_t *surfel_id;
    float *depth, *color_s, *image, *accum;
    const float *d_image;
    ges_gradients grads;
} ges_frame_buffers;

#define GES_PLAN_AUTOTUNE 1  /* time every built tile shape, keep the fastest */

/* Builds a plan on `device` (runs trial frames on `stream` and waits for
 * them).  The plan allocates its own workspace once, here.  With
 * GES_PLAN_AUTOTUNE the candidate launch shapes (raster tile 8/16 x splat
 * 8x8, 16x8, 16x16 x pass 1 per tile or persistent) are timed on these
 * inputs, and the list capacities come from a checked trial frame; if the
 * environment variable
 * GES_AUTOTUNE_CACHE names a file, results are read from and appended to it
 * (JSON lines keyed by device name, view sizes and primitive counts). */
ges_status ges_plan_create(ges_plan **out, int device, const ges_camera *cams, int32_t n_views,
                           const ges_surfels *surfels, const ges_gaussians *gaussians,
                           const ges_options *opt, const ges_frame_buffers *buffers, int flags,
                           void *stream);

/* Replays the frame on `stream`.  cams: NULL (the cameras of the previous
 * launch, or of the plan's creation, are kept), or n_views cameras with the
 * plan's image sizes (new poses/intrinsics; host array, copied: the view
 * table is uploaded on `stream` ahead of the replay, through pinned staging
 * buffers used in turn, so the call waits only if a staging buffer's upload
 * from four launches back has not run yet). */
ges_status ges_plan_launch(ges_plan *plan, const ges_camera *cams, void *stream);

/* Options the plan runs with (tile shapes, capacities). */
ges_status ges_plan_options(const ges_plan *plan, ges_options *out);

/* Synchronises `stream` and reports the last replay's device status. */
ges_status ges_plan_poll(ges_plan *plan, void *stream, ges_run_status *out);

ges_status ges_plan_destroy(ges_plan *plan);

/* Turns stage timing on (enable != 0) or off for this context. */
ges_status ges_profile_enable(ges_context *ctx, int enable);

/* Waits for the recorded events and writes, per stage, the summed elapsed
 * milliseconds (ms[GES_STAGE_COUNT], host) and the number of timed launches
 * (launches[GES_STAGE_COUNT], host; may be NULL).  reset != 0 clears the
 * sums afterwards. */
ges_status ges_profile_read(ges_context *ctx, double *ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* GES_H */
