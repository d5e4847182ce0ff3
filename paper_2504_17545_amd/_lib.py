"""ctypes binding of libges.so (include/ges.h): same names, argument marshalling only.

Every step of the render runs in the library's HIP kernels.  This module
loads the in-tree library and raises if it is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libges.so")

GES_OK, GES_ERR_ARG, GES_ERR_WORKSPACE, GES_ERR_CAPACITY, GES_ERR_HIP, GES_ERR_UNSUPPORTED, GES_ERR_STATE = range(7)
STATUS_NAMES = {0: "GES_OK", 1: "GES_ERR_ARG", 2: "GES_ERR_WORKSPACE", 3: "GES_ERR_CAPACITY",
                4: "GES_ERR_HIP", 5: "GES_ERR_UNSUPPORTED", 6: "GES_ERR_STATE"}
FLAG_SURFEL_OVERFLOW, FLAG_GAUSS_OVERFLOW, FLAG_COLOUR_RANGE = 1, 2, 4


class GESError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ges_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("znear", C.c_float), ("bg", C.c_float * 3)]


class ges_surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("scale", C.c_void_p), ("sh", C.c_void_p)]


class ges_gaussians(C.Structure):
    _fields_ = [("m", C.c_int64), ("sh_degree", C.c_int32), ("dims", C.c_int32),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("scale", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("filter3d", C.c_void_p)]


class ges_options(C.Structure):
    _fields_ = [("surfel_radius", C.c_float), ("eps_factor", C.c_float), ("eps_const", C.c_float),
                ("alpha_min", C.c_float), ("dilation", C.c_float), ("w_s", C.c_float),
                ("raster_tile", C.c_int32), ("splat_tile_w", C.c_int32), ("splat_tile_h", C.c_int32),
                ("tile_queue", C.c_int32), ("surfel_pair_capacity", C.c_int64),
                ("gauss_pair_capacity", C.c_int64), ("surfel_samples", C.c_int32), ("mip_2d", C.c_float)]


class ges_run_status(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("reserved", C.c_uint32), ("surfel_pairs", C.c_int64),
                ("gauss_pairs", C.c_int64), ("surfel_slots", C.c_int64), ("gauss_slots", C.c_int64),
                ("surfel_box_pixels", C.c_int64), ("gauss_box_pixels", C.c_int64),
                ("visible_surfels", C.c_int64), ("active_gaussians", C.c_int64)]

    @property
    def surfel_capacity(self) -> int:
        return max(self.surfel_pairs, self.surfel_slots)

    @property
    def gauss_capacity(self) -> int:
        return max(self.gauss_pairs, self.gauss_slots)


class ges_gradients(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("scale", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p), ("surfel_sh", C.c_void_p)]


class ges_scores_out(C.Structure):
    _fields_ = [("cover", C.c_void_p), ("contrib", C.c_void_p), ("keep_surfel", C.c_void_p),
                ("keep_gauss", C.c_void_p)]


class ges_geometry_out(C.Structure):
    _fields_ = [("normal_s", C.c_void_p), ("depth_g", C.c_void_p), ("normal_g", C.c_void_p),
                ("depth_smooth", C.c_void_p), ("normal_smooth", C.c_void_p)]


class ges_translucent_out(C.Structure):
    _fields_ = [("color", C.c_void_p), ("alpha", C.c_void_p), ("depth", C.c_void_p), ("front", C.c_void_p)]


class ges_surfel_gradients(C.Structure):
    _fields_ = [("mean", C.c_void_p), ("quat", C.c_void_p), ("scale", C.c_void_p), ("w", C.c_void_p),
                ("sh", C.c_void_p)]


class ges_frame_buffers(C.Structure):
    _fields_ = [("surfel_id", C.c_void_p), ("depth", C.c_void_p), ("color_s", C.c_void_p),
                ("image", C.c_void_p), ("accum", C.c_void_p), ("d_image", C.c_void_p),
                ("grads", ges_gradients)]


GES_PLAN_AUTOTUNE = 1

# (name, restype, argtypes) of every exported entry point
SIGNATURES = {
    "ges_options_default": (None, [C.POINTER(ges_options)]),
    "ges_context_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "ges_context_destroy": (C.c_int, [C.c_void_p]),
    "ges_workspace_query": (C.c_int, [C.POINTER(ges_camera), C.c_int32, C.c_int64, C.c_int64,
                                      C.POINTER(ges_options), C.POINTER(C.c_size_t)]),
    "ges_total_pixels": (C.c_int, [C.POINTER(ges_camera), C.c_int32, C.POINTER(C.c_int64)]),
    "ges_project": (C.c_int, [C.c_void_p, C.POINTER(ges_camera), C.c_int32, C.POINTER(ges_surfels),
                              C.POINTER(ges_gaussians), C.POINTER(ges_options), C.c_void_p, C.c_size_t,
                              C.c_void_p]),
    "ges_raster_surfels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ges_splat_gaussians": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "ges_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(ges_gradients), C.c_void_p]),
    "ges_scores": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_int32,
                             C.POINTER(ges_scores_out), C.c_void_p]),
    "ges_scores_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                    C.c_int32, C.POINTER(ges_scores_out), C.c_void_p]),
    "ges_mip_filter3d": (C.c_int, [C.POINTER(ges_camera), C.c_int32, C.POINTER(ges_gaussians), C.c_float,
                                   C.c_void_p, C.c_void_p]),
    "ges_geometry": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(ges_geometry_out),
                               C.c_void_p]),
    "ges_translucent_workspace_query": (C.c_int, [C.POINTER(ges_camera), C.c_int32, C.c_int64,
                                                  C.POINTER(ges_options), C.POINTER(C.c_size_t)]),
    "ges_translucent_render": (C.c_int, [C.c_void_p, C.POINTER(ges_camera), C.c_int32, C.POINTER(ges_surfels),
                                         C.c_void_p, C.c_int32, C.POINTER(ges_options), C.c_void_p, C.c_size_t,
                                         C.POINTER(ges_translucent_out), C.c_void_p]),
    "ges_translucent_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(ges_surfel_gradients), C.c_void_p]),
    "ges_poll_status": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(ges_run_status)]),
    "ges_poll_status_async": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ges_last_error": (C.c_char_p, []),
    "ges_plan_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(ges_camera), C.c_int32,
                                  C.POINTER(ges_surfels), C.POINTER(ges_gaussians), C.POINTER(ges_options),
                                  C.POINTER(ges_frame_buffers), C.c_int, C.c_void_p]),
    "ges_plan_launch": (C.c_int, [C.c_void_p, C.POINTER(ges_camera), C.c_void_p]),
    "ges_plan_options": (C.c_int, [C.c_void_p, C.POINTER(ges_options)]),
    "ges_plan_poll": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(ges_run_status)]),
    "ges_plan_destroy": (C.c_int, [C.c_void_p]),
    "ges_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "ges_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
}

STAGES = ["project", "surfel_bin", "raster", "shade", "resolve", "gauss_bin",
          "splat", "bwd_tiles", "bwd_gauss", "bwd_surfel", "bwd_surfel_tiles", "clear"]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing at {LIB_PATH}: run "
                               "`python -m paper_2504_17545_amd.build` (no CPU fallback exists)")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status: int):
    if status != GES_OK:
        raise GESError(status, lib().ges_last_error().decode())


# ----------------------------------------------------------------------------
# marshalling helpers


def make_camera(cam) -> ges_camera:
    """ges_camera from any object with width, height, fx, fy, cx, cy, R (3x3),
    t (3), znear, bg attributes."""
    c = ges_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, dtype=np.float64).reshape(9)
    t = np.asarray(cam.t, dtype=np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
        c.bg[k] = float(cam.bg[k])
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def camera_array(cams: Sequence) -> C.Array:
    arr = (ges_camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = cam if isinstance(cam, ges_camera) else make_camera(cam)
    return arr


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def sh_degree_of(sh) -> int:
    k = int(sh.shape[0])
    d = int(round(k ** 0.5)) - 1
    if (d + 1) ** 2 != k:
        raise ValueError(f"SH rows {k} is not a square")
    return d


def make_surfels(mean, quat, scale, sh) -> ges_surfels:
    """Surfel descriptor; sh is [n][K][3] (per surfel, see include/ges.h)."""
    s = ges_surfels()
    s.n = int(mean.shape[1])
    if sh.dim() != 3 or int(sh.shape[0]) != s.n or int(sh.shape[2]) != 3:
        raise ValueError(f"surfel sh must be [n][K][3] with n={s.n}, got {tuple(sh.shape)}")
    s.sh_degree = sh_degree_of(sh.permute(1, 2, 0))
    s.mean, s.quat, s.scale, s.sh = _ptr(mean), _ptr(quat), _ptr(scale), _ptr(sh)
    return s


def make_gaussians(mean, quat, scale, opacity, sh, filter3d=None) -> ges_gaussians:
    """Gaussian descriptor; sh is [m][K][3] (per Gaussian, see include/ges.h);
    filter3d [m] optional (Mip-GES world-space filter variances).  A scale of
    two rows ([2][m]) marks the 2D Gaussians of 2D-GES (dims = 2)."""
    g = ges_gaussians()
    g.m = int(mean.shape[1])
    g.dims = 2 if int(scale.shape[0]) == 2 else 3
    if sh.dim() != 3 or int(sh.shape[0]) != g.m or int(sh.shape[2]) != 3:
        raise ValueError(f"Gaussian sh must be [m][K][3] with m={g.m}, got {tuple(sh.shape)}")
    g.sh_degree = sh_degree_of(sh.permute(1, 2, 0))
    g.mean, g.quat, g.scale, g.opacity, g.sh = _ptr(mean), _ptr(quat), _ptr(scale), _ptr(opacity), _ptr(sh)
    if filter3d is not None:
        if int(filter3d.numel()) != g.m:
            raise ValueError(f"filter3d must hold m={g.m} values")
        g.filter3d = _ptr(filter3d)
    return g


def options(**kw) -> ges_options:
    o = ges_options()
    lib().ges_options_default(C.byref(o))
    for k, v in kw.items():
        if k == "splat_tile":
            o.splat_tile_w, o.splat_tile_h = int(v[0]), int(v[1])
            continue
        if not hasattr(o, k):
            raise AttributeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(lib().ges_context_create(C.byref(h), int(device)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().ges_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ges_workspace_query(cams, n: int, m: int, opt: ges_options) -> int:
    arr = camera_array(cams)
    out = C.c_size_t()
    _check(lib().ges_workspace_query(arr, len(cams), int(n), int(m), C.byref(opt), C.byref(out)))
    return int(out.value)


def ges_total_pixels(cams) -> int:
    arr = camera_array(cams)
    out = C.c_int64()
    _check(lib().ges_total_pixels(arr, len(cams), C.byref(out)))
    return int(out.value)


def ges_project(ctx: Context, cams, surfels: ges_surfels, gaussians: ges_gaussians, opt: ges_options,
                ws_ptr: int, ws_bytes: int, stream: int):
    arr = camera_array(cams)
    _check(lib().ges_project(ctx.handle, arr, len(cams), C.byref(surfels), C.byref(gaussians),
                             C.byref(opt), C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.c_void_p(stream)))


def ges_raster_surfels(ctx: Context, surfel_id, depth, color_s, stream: int):
    _check(lib().ges_raster_surfels(ctx.handle, _ptr(surfel_id), _ptr(depth), _ptr(color_s),
                                    C.c_void_p(stream)))


def ges_splat_gaussians(ctx: Context, depth, color_s, image, accum, stream: int):
    _check(lib().ges_splat_gaussians(ctx.handle, _ptr(depth), _ptr(color_s), _ptr(image), _ptr(accum),
                                     C.c_void_p(stream)))


def ges_backward(ctx: Context, surfel_id, depth, color_s, accum, d_image, grads: ges_gradients,
                 stream: int):
    _check(lib().ges_backward(ctx.handle, _ptr(surfel_id), _ptr(depth), _ptr(color_s), _ptr(accum),
                              _ptr(d_image), C.byref(grads), C.c_void_p(stream)))


def ges_scores(ctx: Context, surfel_id, depth, accum, cover_min: int, contrib_min: float, accumulate: bool,
               cover, contrib, keep_surfel, keep_gauss, stream: int):
    out = ges_scores_out(_ptr(cover), _ptr(contrib), _ptr(keep_surfel), _ptr(keep_gauss))
    _check(lib().ges_scores(ctx.handle, _ptr(surfel_id), _ptr(depth), _ptr(accum), int(cover_min),
                            float(contrib_min), int(bool(accumulate)), C.byref(out), C.c_void_p(stream)))


def ges_scores_static(ctx: Context, surfel_id, depth, accum, cover_min: int, contrib_min: float, accumulate: bool,
                      cover, contrib, keep_surfel, keep_gauss, stream: int):
    out = ges_scores_out(_ptr(cover), _ptr(contrib), _ptr(keep_surfel), _ptr(keep_gauss))
    _check(lib().ges_scores_static(ctx.handle, _ptr(surfel_id), _ptr(depth), _ptr(accum), int(cover_min),
                                   float(contrib_min), int(bool(accumulate)), C.byref(out), C.c_void_p(stream)))


def ges_mip_filter3d(cams, gaussians: ges_gaussians, scale2: float, out, stream: int):
    arr = camera_array(cams)
    _check(lib().ges_mip_filter3d(arr, len(cams), C.byref(gaussians), float(scale2), _ptr(out),
                                  C.c_void_p(stream)))


def ges_geometry(ctx: Context, surfel_id, depth, accum, normal_s, depth_g, normal_g, depth_smooth, normal_smooth,
                 stream: int):
    out = ges_geometry_out(_ptr(normal_s), _ptr(depth_g), _ptr(normal_g), _ptr(depth_smooth), _ptr(normal_smooth))
    _check(lib().ges_geometry(ctx.handle, _ptr(surfel_id), _ptr(depth), _ptr(accum), C.byref(out),
                              C.c_void_p(stream)))


def ges_translucent_workspace_query(cams, n: int, opt: ges_options) -> int:
    arr = camera_array(cams)
    out = C.c_size_t()
    _check(lib().ges_translucent_workspace_query(arr, len(cams), int(n), C.byref(opt), C.byref(out)))
    return int(out.value)


def ges_translucent_render(ctx: Context, cams, surfels: ges_surfels, w, front_first: bool, opt: ges_options,
                           ws_ptr: int, ws_bytes: int, color, alpha, depth, front, stream: int):
    arr = camera_array(cams)
    out = ges_translucent_out(_ptr(color), _ptr(alpha), _ptr(depth), _ptr(front))
    _check(lib().ges_translucent_render(ctx.handle, arr, len(cams), C.byref(surfels), _ptr(w), int(bool(front_first)),
                                        C.byref(opt), C.c_void_p(ws_ptr), C.c_size_t(ws_bytes), C.byref(out),
                                        C.c_void_p(stream)))


def ges_translucent_backward(ctx: Context, d_color, g_mean, g_quat, g_scale, g_w, g_sh, stream: int):
    g = ges_surfel_gradients(_ptr(g_mean), _ptr(g_quat), _ptr(g_scale), _ptr(g_w), _ptr(g_sh))
    _check(lib().ges_translucent_backward(ctx.handle, _ptr(d_color), C.byref(g), C.c_void_p(stream)))


FLAG_SORT_OVERFLOW = 8


def ges_poll_status(ctx: Context, stream: int, raise_on_error: bool = True) -> ges_run_status:
    st = ges_run_status()
    rc = lib().ges_poll_status(ctx.handle, C.c_void_p(stream), C.byref(st))
    if rc != GES_OK and (raise_on_error or rc != GES_ERR_CAPACITY):
        _check(rc)
    return st


def ges_poll_status_async(ctx: Context, stream: int, host_out_ptr: int):
    """Enqueue the frame's status copy into pinned host memory at host_out_ptr
    (sizeof(ges_run_status) bytes); read it once the stream has passed this
    point."""
    _check(lib().ges_poll_status_async(ctx.handle, C.c_void_p(stream), C.c_void_p(host_out_ptr)))


def status_result(st: ges_run_status):
    """GES_OK, or the status code ges_poll_status would return for st."""
    if st.flags & (FLAG_SURFEL_OVERFLOW | FLAG_GAUSS_OVERFLOW | FLAG_COLOUR_RANGE):
        return GES_ERR_CAPACITY
    return GES_OK


class Plan:
    """Handle of a ges_plan (graph-captured multi-view frame)."""

    def __init__(self, device: int, cams, surfels: ges_surfels, gaussians: ges_gaussians, opt: ges_options,
                 buffers: ges_frame_buffers, flags: int, stream: int):
        h = C.c_void_p()
        arr = camera_array(cams)
        _check(lib().ges_plan_create(C.byref(h), int(device), arr, len(cams), C.byref(surfels),
                                     C.byref(gaussians), C.byref(opt), C.byref(buffers), int(flags),
                                     C.c_void_p(stream)))
        self.handle = h
        self.n_views = len(cams)

    def launch(self, stream: int, cams=None):
        arr = camera_array(cams) if cams is not None else None
        _check(lib().ges_plan_launch(self.handle, arr, C.c_void_p(stream)))

    def options(self) -> ges_options:
        o = ges_options()
        _check(lib().ges_plan_options(self.handle, C.byref(o)))
        return o

    def poll(self, stream: int, raise_on_error: bool = True) -> ges_run_status:
        st = ges_run_status()
        rc = lib().ges_plan_poll(self.handle, C.c_void_p(stream), C.byref(st))
        if rc != GES_OK and (raise_on_error or rc != GES_ERR_CAPACITY):
            _check(rc)
        return st

    def close(self):
        if self.handle:
            lib().ges_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ges_profile_enable(ctx: Context, enable: bool = True):
    _check(lib().ges_profile_enable(ctx.handle, int(bool(enable))))


def ges_profile_read(ctx: Context, reset: bool = True):
    """{stage: (total ms, timed launches)} since the last reset."""
    ms = (C.c_double * len(STAGES))()
    n = (C.c_int64 * len(STAGES))()
    _check(lib().ges_profile_read(ctx.handle, ms, n, int(bool(reset))))
    return {name: (ms[k], n[k]) for k, name in enumerate(STAGES)}


def exported_symbols() -> Iterable[str]:
    return SIGNATURES.keys()
