"""Translucent surfels of the surfel optimisation stage (Sec. 4.1, Eq. 6-7)
through ges_translucent_render / ges_translucent_backward: torch buffers and
streams around the C ABI, nothing more (every step runs in the HIP library).
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import torch

from . import _lib
from .render import SURFEL_KEYS, _dev_tensor


class TranslucentFrame:
    """Outputs of one translucent render: colour [3 * P], alpha, depth, front
    [P] ([c][H][W] planes per view, views concatenated)."""

    def __init__(self, ctx, cams, color, alpha, depth, front, surfels, w, ws):
        self.ctx, self.cams = ctx, cams
        self.color, self.alpha, self.depth, self.front = color, alpha, depth, front
        self.surfels, self.w, self._ws = surfels, w, ws
        self.status = None

    def view(self, name: str, v: int) -> torch.Tensor:
        """Output `name` of view v as [c][H][W] (or [H][W]): each view's
        planes are one block, views concatenated."""
        off = sum(int(c.width) * int(c.height) for c in self.cams[:v])
        c = self.cams[v]
        H, W = int(c.height), int(c.width)
        t = getattr(self, name)
        ch = 3 if name == "color" else 1
        blk = t[ch * off: ch * (off + H * W)]
        return blk.view(H, W) if ch == 1 else blk.view(ch, H, W)


class TranslucentRenderer:
    """Renders translucent surfels and their gradients on one device."""

    def __init__(self, device: Optional[torch.device] = None, **opts):
        self.device = torch.device(device or "cuda")
        self.opts = dict(opts)

    def render(self, surfels: Dict[str, torch.Tensor], w: torch.Tensor, cams: Sequence, front_first: bool = False,
               check: bool = True, max_retries: int = 3) -> TranslucentFrame:
        S = {k: _dev_tensor(surfels[k], f"surfels.{k}") for k in SURFEL_KEYS}
        w = _dev_tensor(w, "w")
        cams = list(cams)
        opt = _lib.options(**self.opts)
        sd = _lib.make_surfels(S["mean"], S["quat"], S["scale"], S["sh"])
        P = _lib.ges_total_pixels(cams)
        dev = self.device
        for _ in range(max_retries + 1):
            ws_bytes = _lib.ges_translucent_workspace_query(cams, sd.n, opt)
            ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
            ws_ptr = (ws.data_ptr() + 255) // 256 * 256
            ctx = _lib.Context(dev.index or 0)
            color = torch.empty(3 * P, dtype=torch.float32, device=dev)
            alpha = torch.empty(P, dtype=torch.float32, device=dev)
            depth = torch.empty(P, dtype=torch.float32, device=dev)
            front = torch.empty(P, dtype=torch.int32, device=dev)
            stream = torch.cuda.current_stream(dev).cuda_stream
            _lib.ges_translucent_render(ctx, cams, sd, w, front_first, opt, ws_ptr, ws_bytes, color, alpha, depth,
                                        front, stream)
            f = TranslucentFrame(ctx, cams, color, alpha, depth, front, S, w, ws)
            if not check:
                return f
            st = _lib.ges_poll_status(ctx, stream, raise_on_error=False)
            f.status = st
            if st.flags & _lib.FLAG_SORT_OVERFLOW:
                raise _lib.GESError(_lib.GES_ERR_CAPACITY, "a tile's translucent list exceeds the sort capacity")
            if not st.flags & _lib.FLAG_SURFEL_OVERFLOW:
                return f
            opt.surfel_pair_capacity = int(max(st.surfel_capacity, 1) * 1.25) + 4096
        raise _lib.GESError(_lib.GES_ERR_CAPACITY, "list capacity not found")

    def backward(self, frame: TranslucentFrame, d_color: torch.Tensor) -> Dict[str, torch.Tensor]:
        """d(sum d_color * color) / d(surfel mean, quat, scale, w, sh)."""
        d_color = _dev_tensor(d_color, "d_color")
        S = frame.surfels
        g = {k: torch.empty_like(S[k]) for k in SURFEL_KEYS}
        g["w"] = torch.empty_like(frame.w)
        _lib.ges_translucent_backward(frame.ctx, d_color, g["mean"], g["quat"], g["scale"], g["w"], g["sh"],
                                      torch.cuda.current_stream(self.device).cuda_stream)
        return g
