"""torch-facing wrapper of the C ABI: device buffers, streams, autograd.

PyTorch only provides device memory and the stream here; every stage of the
render and of its gradient runs in libges.so's HIP kernels.

Scene tensors are float32, contiguous, on the same CUDA (HIP) device,
structure-of-arrays with the primitive index last, except the SH, which is
per primitive (only the surfels that win a pixel and the Gaussians that keep
a list entry are shaded, and only their coefficients are read):
  surfels:   mean [3,N], quat [4,N] (w,x,y,z), scale [2,N], sh [N,K,3] (per surfel)
  gaussians: mean [3,M], quat [4,M], scale [3,M] (or [2,M]: the 2D Gaussians of
             2D-GES, forward only), opacity [M], sh [M,K,3] (per Gaussian)
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import torch

from . import _lib

SURFEL_KEYS = ("mean", "quat", "scale", "sh")
GAUSS_KEYS = ("mean", "quat", "scale", "opacity", "sh")


def _dev_tensor(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    return t.contiguous()


class _Slot:
    """A library context and its device workspace, reused by successive
    frames of one Renderer: a frame holds its slot until it is released
    (after its backward, or when it is garbage-collected), and a later frame
    takes it over with no context creation and, while the workspace is large
    enough, no allocation."""

    def __init__(self, device):
        self.ctx = _lib.Context(device.index if device.index is not None else torch.cuda.current_device())
        self.ws: Optional[torch.Tensor] = None
        self.released: Optional[torch.cuda.Event] = None  # work of the last frame on this slot

    def workspace(self, nbytes: int, device) -> torch.Tensor:
        if self.ws is None or self.ws.numel() < nbytes + 256:
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        return self.ws


@dataclasses.dataclass
class Frame:
    """Outputs and saved state of one rendered frame (all views)."""
    image: torch.Tensor      # [sum 3 P_v]
    accum: torch.Tensor      # [sum 4 P_v]  C_G (3), W_G
    surfel_id: torch.Tensor  # [sum P_v] int32
    depth: torch.Tensor      # [sum P_v]
    color_s: torch.Tensor    # [sum 3 P_v]
    cams: list
    offsets: List[int]       # first pixel of each view
    ctx: _lib.Context
    workspace: torch.Tensor
    ws_ptr: int
    ws_bytes: int
    opt: _lib.ges_options
    surfels: Dict[str, torch.Tensor]
    gaussians: Dict[str, torch.Tensor]
    status: Optional[_lib.ges_run_status] = None
    slot: Optional[_Slot] = None
    pool: Optional[list] = None

    def release(self):
        """Hand the frame's context and workspace back to its renderer (the
        frame can no longer be scored or differentiated).  Stream-ordered:
        the next frame on the slot waits for this one's queued work."""
        if self.slot is not None and self.pool is not None:
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(self.image.device))
            self.slot.released = ev
            self.pool.append(self.slot)
        self.slot = None
        self.pool = None
        self.ctx = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def view(self, name: str, v: int) -> torch.Tensor:
        """Per-view image of output `name` shaped [c, H, W] (or [H, W]); the
        surfel id map with 4 samples per pixel is [2H, 2W]."""
        cam = self.cams[v]
        W, H = int(cam.width), int(cam.height)
        off = self.offsets[v]
        t = getattr(self, name)
        ch = {"image": 3, "color_s": 3, "accum": 4, "surfel_id": 1, "depth": 1}[name]
        if name == "surfel_id" and t.numel() == 4 * self.depth.numel():  # sample grid
            return t[4 * off: 4 * (off + W * H)].view(2 * H, 2 * W)
        blk = t[ch * off: ch * (off + W * H)]
        return blk.view(H, W) if ch == 1 else blk.view(ch, H, W)


class Renderer:
    """Owns the options; renders frames and their gradients on one device."""

    def __init__(self, device: Optional[torch.device] = None, **opts):
        self.device = torch.device(device or "cuda")
        self.opts = dict(opts)
        self._pool: List[_Slot] = []          # released slots, reused by later frames
        self._caps = None                     # list capacities learned by a checked frame
        self._pending: List[tuple] = []       # (event, pinned status, frame label) of lazily checked frames

    def options(self, **over) -> _lib.ges_options:
        kw = dict(self.opts)
        kw.update(over)
        return _lib.options(**kw)

    def render(self, surfels: Dict[str, torch.Tensor], gaussians: Dict[str, torch.Tensor], cams: Sequence,
               check=True, max_retries: int = 3, **over) -> Frame:
        """Forward of every view in `cams`.

        check=True waits for the frame and re-renders with larger list
        capacities if the device reported an overflow (a frame that
        overflowed is never returned).  check="lazy" does not wait: the
        first lazy frame is checked as above and its list sizes (+25%) are
        kept; later frames reuse them and enqueue an asynchronous status copy,
        and every later call raises GESError if an earlier lazy frame's copy
        has arrived with an overflow flag (see `check_pending`).
        check=False does neither."""
        S = {k: _dev_tensor(surfels[k], f"surfels.{k}") for k in SURFEL_KEYS}
        G = {k: _dev_tensor(gaussians[k], f"gaussians.{k}") for k in GAUSS_KEYS}
        if gaussians.get("filter3d") is not None:
            G["filter3d"] = _dev_tensor(gaussians["filter3d"], "gaussians.filter3d")
        opt = self.options(**over)
        if check == "lazy":
            self.check_pending(wait=False)
            if self._caps is not None:
                opt.surfel_pair_capacity, opt.gauss_pair_capacity = self._caps
                frame = self._render_once(S, G, list(cams), opt)
                pinned = torch.empty(C.sizeof(_lib.ges_run_status), dtype=torch.uint8, pin_memory=True)
                stream = torch.cuda.current_stream(self.device)
                _lib.ges_poll_status_async(frame.ctx, stream.cuda_stream, pinned.data_ptr())
                ev = torch.cuda.Event()
                ev.record(stream)
                self._pending.append((ev, pinned))
                return frame
            frame = self.render(S, G, cams, True, max_retries, **over)
            st = frame.status
            self._caps = (int(max(st.surfel_capacity, 1) * 1.25) + 4096,
                          int(max(st.gauss_capacity, 1) * 1.25) + 4096)
            return frame
        for _ in range(max_retries + 1):
            frame = self._render_once(S, G, list(cams), opt)
            if not check:
                return frame
            st = _lib.ges_poll_status(frame.ctx, torch.cuda.current_stream(self.device).cuda_stream,
                                      raise_on_error=False)
            frame.status = st
            if st.flags & _lib.FLAG_COLOUR_RANGE:
                raise _lib.GESError(_lib.GES_ERR_CAPACITY, "Gaussian colour outside the fixed-point range")
            over_s = st.flags & _lib.FLAG_SURFEL_OVERFLOW
            over_g = st.flags & _lib.FLAG_GAUSS_OVERFLOW
            if not (over_s or over_g):
                return frame
            if over_s:
                opt.surfel_pair_capacity = int(st.surfel_capacity * 1.25) + 1024
            if over_g:
                opt.gauss_pair_capacity = int(st.gauss_capacity * 1.25) + 1024
        raise _lib.GESError(_lib.GES_ERR_CAPACITY, "list capacity still exceeded after retries")

    def check_pending(self, wait: bool = False):
        """Examine the status copies of lazily checked frames that have
        arrived (all of them with wait=True); raise GESError if one reports
        an overflow or a colour out of range, after raising the learned list
        sizes so that the next frame fits."""
        keep = []
        bad = None
        for ev, pinned in self._pending:
            if not (wait or ev.query()):
                keep.append((ev, pinned))
                continue
            ev.synchronize()
            st = _lib.ges_run_status.from_buffer_copy(bytes(pinned.numpy()))
            if _lib.status_result(st) != _lib.GES_OK and bad is None:
                bad = st
        self._pending = keep
        if bad is not None:
            if self._caps is not None:
                self._caps = (max(self._caps[0], int(bad.surfel_capacity * 1.25) + 4096),
                              max(self._caps[1], int(bad.gauss_capacity * 1.25) + 4096))
            raise _lib.GESError(_lib.GES_ERR_CAPACITY,
                                f"an earlier lazily checked frame overflowed (flags {bad.flags}); "
                                "its outputs were invalid; list sizes raised for later frames")

    def _acquire(self) -> _Slot:
        if self._pool:
            slot = self._pool.pop()
            if slot.released is not None:
                torch.cuda.current_stream(self.device).wait_event(slot.released)
                slot.released = None
            return slot
        return _Slot(self.device)

    def _render_once(self, S, G, cams, opt) -> Frame:
        dev = self.device
        n, m = int(S["mean"].shape[1]), int(G["mean"].shape[1])
        ws_bytes = _lib.ges_workspace_query(cams, n, m, opt)
        slot = self._acquire()
        ws = slot.workspace(ws_bytes, dev)
        base = ws.data_ptr()
        ws_ptr = (base + 255) // 256 * 256
        P = _lib.ges_total_pixels(cams)
        offsets, acc = [], 0
        for c in cams:
            offsets.append(acc)
            acc += int(c.width) * int(c.height)
        sid = torch.empty(P * int(opt.surfel_samples or 1), dtype=torch.int32, device=dev)  # per sample
        depth = torch.empty(P, dtype=torch.float32, device=dev)
        color_s = torch.empty(3 * P, dtype=torch.float32, device=dev)
        image = torch.empty(3 * P, dtype=torch.float32, device=dev)
        accum = torch.empty(4 * P, dtype=torch.float32, device=dev)
        ctx = slot.ctx
        stream = torch.cuda.current_stream(dev).cuda_stream
        sd = _lib.make_surfels(S["mean"], S["quat"], S["scale"], S["sh"])
        gd = _lib.make_gaussians(G["mean"], G["quat"], G["scale"], G["opacity"], G["sh"], G.get("filter3d"))
        _lib.ges_project(ctx, cams, sd, gd, opt, ws_ptr, ws_bytes, stream)
        _lib.ges_raster_surfels(ctx, sid, depth, color_s, stream)
        _lib.ges_splat_gaussians(ctx, depth, color_s, image, accum, stream)
        return Frame(image, accum, sid, depth, color_s, cams, offsets, ctx, ws, ws_ptr, ws_bytes, opt, S, G,
                     slot=slot, pool=self._pool)

    def backward(self, frame: Frame, d_image: torch.Tensor) -> Dict[str, torch.Tensor]:
        """Gradients of sum(d_image * image) w.r.t. the Gaussian parameters
        and the surfel SH (summed over the frame's views)."""
        if frame.ctx is None:
            raise ValueError("frame was released: render it again")
        d_image = _dev_tensor(d_image.reshape(-1), "d_image")
        if d_image.numel() != frame.image.numel():
            raise ValueError("d_image must match the image size")
        G, S = frame.gaussians, frame.surfels
        out = {k: torch.empty_like(G[k]) for k in GAUSS_KEYS}
        out["surfel_sh"] = torch.empty_like(S["sh"])
        gr = _lib.ges_gradients()
        gr.mean, gr.quat, gr.scale = out["mean"].data_ptr(), out["quat"].data_ptr(), out["scale"].data_ptr()
        gr.opacity, gr.sh, gr.surfel_sh = out["opacity"].data_ptr(), out["sh"].data_ptr(), out["surfel_sh"].data_ptr()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.ges_backward(frame.ctx, frame.surfel_id, frame.depth, frame.color_s, frame.accum, d_image, gr, stream)
        return out


    def scores(self, frame: Frame, cover_min: int = 16, contrib_min: float = 0.02,
               into: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """Pruning scores of the frame's views (ges_scores): `cover` [N] int32
        (max over views of the frontmost-pixel count), `contrib` [M] float
        (max over views of Eq. 9's contribution), and the keep flags
        `keep_surfel` / `keep_gauss` (uint8) at the given thresholds.  With
        `into` (a previous result), this frame's scores are folded into it
        by maximum."""
        if frame.ctx is None:
            raise ValueError("frame was released: render it again")
        n, m = int(frame.surfels["mean"].shape[1]), int(frame.gaussians["mean"].shape[1])
        dev = frame.image.device
        out = into if into is not None else dict(
            cover=torch.empty(n, dtype=torch.int32, device=dev),
            contrib=torch.empty(m, dtype=torch.float32, device=dev),
            keep_surfel=torch.empty(n, dtype=torch.uint8, device=dev),
            keep_gauss=torch.empty(m, dtype=torch.uint8, device=dev))
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _lib.ges_scores(frame.ctx, frame.surfel_id, frame.depth, frame.accum, cover_min, contrib_min,
                        into is not None, out["cover"], out["contrib"], out["keep_surfel"], out["keep_gauss"],
                        stream)
        return out


    def geometry(self, frame: Frame) -> Dict[str, torch.Tensor]:
        """Geometry channels of the frame (ges_geometry, Eq. 10-12):
        normal_s, normal_g, normal_smooth [sum 3 P_v] and depth_g,
        depth_smooth [sum P_v], per view [c][H][W]."""
        if frame.ctx is None:
            raise ValueError("frame was released: render it again")
        P = frame.depth.numel()
        dev = frame.image.device
        out = dict(normal_s=torch.empty(3 * P, device=dev), depth_g=torch.empty(P, device=dev),
                   normal_g=torch.empty(3 * P, device=dev), depth_smooth=torch.empty(P, device=dev),
                   normal_smooth=torch.empty(3 * P, device=dev))
        _lib.ges_geometry(frame.ctx, frame.surfel_id, frame.depth, frame.accum, out["normal_s"], out["depth_g"],
                          out["normal_g"], out["depth_smooth"], out["normal_smooth"],
                          torch.cuda.current_stream(self.device).cuda_stream)
        return out


class PlannedFrame:
    """A ges_plan with its torch buffers: many views, forward (+ backward),
    captured once into a graph and replayed by `launch`.

    Write the upstream gradient into `d_image` (in place) before a launch;
    after it, `image`, `accum`, ... and `grads` hold the frame's results.
    Camera poses/intrinsics may change per launch, image sizes may not."""

    def __init__(self, surfels: Dict[str, torch.Tensor], gaussians: Dict[str, torch.Tensor], cams: Sequence,
                 backward: bool = True, autotune: bool = False, device: Optional[torch.device] = None, **opts):
        dev = torch.device(device or "cuda")
        self.device = dev
        self.cams = list(cams)
        S = {k: _dev_tensor(surfels[k], f"surfels.{k}") for k in SURFEL_KEYS}
        G = {k: _dev_tensor(gaussians[k], f"gaussians.{k}") for k in GAUSS_KEYS}
        if gaussians.get("filter3d") is not None:
            G["filter3d"] = _dev_tensor(gaussians["filter3d"], "gaussians.filter3d")
        self.surfels, self.gaussians = S, G
        P = _lib.ges_total_pixels(self.cams)
        self.offsets, acc = [], 0
        for c in self.cams:
            self.offsets.append(acc)
            acc += int(c.width) * int(c.height)
        samples = int(opts.get("surfel_samples", 1))
        self.surfel_id = torch.empty(P * samples, dtype=torch.int32, device=dev)  # per sample
        self.depth = torch.empty(P, dtype=torch.float32, device=dev)
        self.color_s = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.image = torch.empty(3 * P, dtype=torch.float32, device=dev)
        self.accum = torch.empty(4 * P, dtype=torch.float32, device=dev)
        buf = _lib.ges_frame_buffers()
        buf.surfel_id, buf.depth, buf.color_s = (self.surfel_id.data_ptr(), self.depth.data_ptr(),
                                                 self.color_s.data_ptr())
        buf.image, buf.accum = self.image.data_ptr(), self.accum.data_ptr()
        self.grads = None
        self.d_image = None
        if backward:
            self.d_image = torch.zeros(3 * P, dtype=torch.float32, device=dev)
            self.grads = {k: torch.zeros_like(G[k]) for k in GAUSS_KEYS}
            self.grads["surfel_sh"] = torch.zeros_like(S["sh"])
            buf.d_image = self.d_image.data_ptr()
            for k in GAUSS_KEYS:
                setattr(buf.grads, k, self.grads[k].data_ptr())
            buf.grads.surfel_sh = self.grads["surfel_sh"].data_ptr()
        self._buf = buf
        sd = _lib.make_surfels(S["mean"], S["quat"], S["scale"], S["sh"])
        gd = _lib.make_gaussians(G["mean"], G["quat"], G["scale"], G["opacity"], G["sh"], G.get("filter3d"))
        opt = _lib.options(**opts)
        stream = torch.cuda.current_stream(dev).cuda_stream
        self.plan = _lib.Plan(dev.index if dev.index is not None else torch.cuda.current_device(), self.cams,
                              sd, gd, opt, buf, _lib.GES_PLAN_AUTOTUNE if autotune else 0, stream)

    def launch(self, cams: Optional[Sequence] = None):
        if cams is not None:
            self.cams = list(cams)
        self.plan.launch(torch.cuda.current_stream(self.device).cuda_stream, cams)

    def options(self) -> _lib.ges_options:
        return self.plan.options()

    def poll(self, raise_on_error: bool = True) -> _lib.ges_run_status:
        return self.plan.poll(torch.cuda.current_stream(self.device).cuda_stream, raise_on_error)

    def view(self, name: str, v: int) -> torch.Tensor:
        return Frame.view(self, name, v)  # same layout helper

    def close(self):
        self.plan.close()


class _GESFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g_mean, g_quat, g_scale, g_opacity, g_sh, s_sh, s_mean, s_quat, s_scale, renderer, cams):
        S = dict(mean=s_mean, quat=s_quat, scale=s_scale, sh=s_sh)
        G = dict(mean=g_mean, quat=g_quat, scale=g_scale, opacity=g_opacity, sh=g_sh)
        frame = renderer.render(S, G, cams, check="lazy")
        ctx.frame = frame
        ctx.renderer = renderer
        return frame.image

    @staticmethod
    def backward(ctx, d_image):
        g = ctx.renderer.backward(ctx.frame, d_image.contiguous())
        ctx.frame.release()  # its context and workspace serve the next frame
        ctx.frame = None
        return g["mean"], g["quat"], g["scale"], g["opacity"], g["sh"], g["surfel_sh"], None, None, None, None, None


def render_differentiable(renderer: Renderer, surfels: Dict[str, torch.Tensor],
                          gaussians: Dict[str, torch.Tensor], cams: Sequence) -> torch.Tensor:
    """Image [sum 3 P_v] whose backward runs ges_backward (Gaussian
    parameters and surfel SH receive gradients; surfel geometry is fixed).

    No host synchronisation per frame: frames are checked lazily (see
    Renderer.render), and each frame's context and workspace go back to the
    renderer after its backward for the next frame to reuse."""
    return _GESFunction.apply(gaussians["mean"], gaussians["quat"], gaussians["scale"], gaussians["opacity"],
                              gaussians["sh"], surfels["sh"], surfels["mean"].detach(), surfels["quat"].detach(),
                              surfels["scale"].detach(), renderer, list(cams))
