"""FP64 CPU oracle of 2D-GES's second pass (Sec. 6.4): 2D Gaussians in place
of the 3D ones.  TEST INFRASTRUCTURE ONLY (see the package notes).

A 2D Gaussian is a planar splat: centre p, rotation r whose first two axes
t_u, t_v span its plane and whose third is its normal, scales (s_u, s_v),
maximum opacity sigma and SH colour.  At a pixel the camera ray through the
pixel centre meets the splat's plane at the camera depth

    z = (n . mu) / (n . r)           (mu: the centre, r = (x', y', 1): the ray),

the planar depth that replaces the centre depth of the 3D Gaussian (Sec.
6.4); its local coordinates there are u = (X - mu) . t_u / s_u, v alike
(X = z r), and

    alpha = sigma exp(-(u^2 + v^2) / 2),   zero below 1/255 (as Eq. 4).

It counts at the pixel iff its planar depth passes the pass-2 test
z < D_s + eps with eps = (5/D) sum_j s_j, D = 2 (Sec. 5), and the hit is in
front of the near plane (z >= znear) and not edge-on -- the surfel rules.
Then (Eq. 2-3, 5 unchanged) C_G = sum alpha c, W_G = sum alpha and
C = (C_s W_s + C_G) / (W_s + W_G); the geometry channels (Eq. 10-12) take
d_i = the planar depth at the pixel and n_i = the splat's normal, world
space, turned to face the camera.

The surfel pass is `render.py`'s, unchanged (a render of the scene without
Gaussians gives C_s, D_s and its bookkeeping).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from .render import (DT, Cam, Options, _degree, _t, facing, quat_to_rot, render, surfel_frames,
                     view_directions)
from .sh import sh_colour


def gauss2d_frames(G, cam: Cam) -> Dict[str, torch.Tensor]:
    """Camera-space centre, unit axes and normal, eps, opacity and colour of
    every 2D Gaussian (scale [2][M]) in this view."""
    mean = _t(G.mean)
    mu = (cam.R @ mean).T + cam.t                    # [M, 3]
    A = cam.R @ quat_to_rot(_t(G.quat))              # [M, 3, 3]
    scale = _t(G.scale)                              # [2, M]
    assert scale.shape[0] == 2 or scale.shape[1] == 0, "2D Gaussians have two scales"
    return dict(mu=mu, tu=A[:, :, 0], tv=A[:, :, 1], n=A[:, :, 2], scale=scale.T,
                opacity=_t(G.opacity),
                colour=sh_colour(_t(G.sh), view_directions(mean, cam), _degree(_t(G.sh))),
                normal_world=facing(quat_to_rot(_t(G.quat))[:, :, 2], cam.o[None, :] - mean.T))


def eps_2d(G, opts: Options) -> torch.Tensor:
    """eps_i = (5/D) sum_j s_ij with D = 2 (Sec. 5); the constant-eps option
    as for 3D Gaussians."""
    s = _t(G.scale)
    if opts.eps_const >= 0:
        return torch.full((s.shape[1],), opts.eps_const, dtype=DT)
    return opts.eps_factor / 2.0 * s.sum(0)


def splat_hits(fr, cam: Cam, pix: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Per (pixel, splat): the planar depth z where the pixel's ray meets the
    splat's plane, alpha there, and whether the hit counts geometrically
    (not edge-on, z >= znear).  [P, M] each."""
    r = cam.rays(pix)                                  # [P, 3]
    mu, tu, tv, n, sc = fr["mu"], fr["tu"], fr["tv"], fr["n"], fr["scale"]
    nr = r @ n.T                                       # [P, M]
    nmu = (n * mu).sum(-1)                             # [M]
    rnorm = torch.linalg.norm(r, dim=-1, keepdim=True)
    edge = nr.abs() <= 1e-12 * rnorm
    z = nmu[None, :] / torch.where(edge, torch.ones_like(nr), nr)
    u = (z * (r @ tu.T) - (mu * tu).sum(-1)[None, :]) / sc[:, 0][None, :]
    v = (z * (r @ tv.T) - (mu * tv).sum(-1)[None, :]) / sc[:, 1][None, :]
    alpha = fr["opacity"][None, :] * torch.exp(-0.5 * (u * u + v * v))
    return dict(z=z, alpha=alpha, front=(~edge) & (z >= cam.znear), edge=edge)


def depth_test(z: torch.Tensor, fr, depth_s: torch.Tensor, eps: torch.Tensor) -> torch.Tensor:
    """The pass-2 depth test with the planar depth: z < D_s + eps."""
    return z < depth_s[:, None] + eps[None, :]


def gauss2d_pass(fr, eps, cam: Cam, pix: torch.Tensor, depth_s: torch.Tensor, opts: Options):
    """C_G [3,P], W_G [P], D_G [P], N_G [3,P] of the pixels `pix`, with the
    pairs' weights w [P,M] and planar depths z [P,M], and the margins of the
    discrete decisions for comparisons with FP32 evaluations:
      alpha_margin  min |ln(alpha / alpha_min)| over pairs in front of the
                    near plane whose depth test passes or nearly passes;
      depth_margin  min |z - D_s - eps| / (D_s + eps) over pairs with alpha
                    at or near the threshold;
      near_margin   min |z - znear| / znear over pairs with alpha near or
                    above the threshold."""
    P, M = pix.shape[0], fr["mu"].shape[0]
    if M == 0:
        z0 = torch.zeros(P, dtype=DT)
        inf = torch.full((P,), math.inf, dtype=DT)
        return dict(cg=torch.zeros(3, P, dtype=DT), wg=z0, dg=z0.clone(), ng=torch.zeros(3, P, dtype=DT),
                    w=torch.zeros(P, 0, dtype=DT), z=torch.zeros(P, 0, dtype=DT), alpha_margin=inf,
                    depth_margin=inf.clone(), near_margin=inf.clone(), count=torch.zeros(P, dtype=torch.long))
    h = splat_hits(fr, cam, pix)
    z, alpha, edge = h["z"], h["alpha"], h["edge"]
    keep = h["front"] & depth_test(z, fr, depth_s, eps) & (alpha >= opts.alpha_min)
    w = torch.where(keep, alpha, torch.zeros_like(alpha))
    cg = fr["colour"] @ w.T
    wg = w.sum(1)
    dg = (w * z).sum(1)
    ng = (w @ fr["normal_world"]).T
    with torch.no_grad():
        lim = depth_s[:, None] + eps[None, :]
        lm = (torch.log(alpha.clamp_min(1e-300)) - math.log(opts.alpha_min)).abs()
        near_ok = (~edge) & (z >= cam.znear * (1 - 1e-4))
        alpha_margin = torch.where(near_ok & (z < lim * (1 + 1e-4)), lm, torch.full_like(lm, math.inf)).min(1).values
        dm = (z - lim).abs() / lim.abs()
        dm = torch.where(torch.isfinite(lim), dm, torch.full_like(dm, math.inf))
        around = alpha >= opts.alpha_min * (1 - 1e-4)
        depth_margin = torch.where(near_ok & around, dm, torch.full_like(dm, math.inf)).min(1).values
        nm = (z - cam.znear).abs() / cam.znear
        near_margin = torch.where((~edge) & around, nm, torch.full_like(nm, math.inf)).min(1).values
    return dict(cg=cg, wg=wg, dg=dg, ng=ng, w=w, z=z, alpha_margin=alpha_margin, depth_margin=depth_margin,
                near_margin=near_margin, count=keep.sum(1))


def render_2dges(scene, cam_idx=0, pix=None, opts: Optional[Options] = None, chunk_elems=2_000_000):
    """2D-GES render of the pixels `pix` (default: whole image) of camera
    `cam_idx`, scene.gaussians being 2D Gaussians (scale [2][M]).  Returns
    the surfel pass's outputs and bookkeeping (`render.py`), C_G, W_G, the
    image, the geometry channels N_s, D_G, N_G, D_smooth, N_smooth (as
    `render.geometry`, with the planar depth and splat normal) and the
    pass-2 margins (alpha_margin, depth_margin, near_margin)."""
    opts = opts or Options()
    cam = Cam(scene.cameras[cam_idx])
    if pix is None:
        pix = torch.arange(cam.W * cam.H)
    pix = torch.as_tensor(pix, dtype=torch.long)
    S, G = scene.surfels, scene.gaussians
    no_g = type(G)(G.mean[:, :0], G.quat[:, :0], np.zeros((3, 0)), G.opacity[:0], G.sh[..., :0])
    with torch.no_grad():
        sp = render(type(scene)(S, no_g, scene.cameras), cam_idx, pix, opts)
        fr = gauss2d_frames(G, cam)
        eps = eps_2d(G, opts)
        P = pix.shape[0]
        acc = dict(cg=torch.zeros(3, P, dtype=DT), wg=torch.zeros(P, dtype=DT), dg=torch.zeros(P, dtype=DT),
                   ng=torch.zeros(3, P, dtype=DT), alpha_margin=torch.full((P,), math.inf, dtype=DT),
                   depth_margin=torch.full((P,), math.inf, dtype=DT),
                   near_margin=torch.full((P,), math.inf, dtype=DT), count=torch.zeros(P, dtype=torch.long))
        step = max(1, chunk_elems // max(G.m, 1))
        for s0 in range(0, P, step):
            sl = slice(s0, s0 + step)
            gp = gauss2d_pass(fr, eps, cam, pix[sl], sp["depth"][sl], opts)
            for k in acc:
                if acc[k].dim() == 2:
                    acc[k][:, sl] = gp[k]
                else:
                    acc[k][sl] = gp[k]
        ids = sp["id"]
        if S.n:
            ns = facing(surfel_frames(S, cam)["n"] @ cam.R, cam.o[None, :] - _t(S.mean).T)
            Ns = torch.where(ids[None, :] >= 0, ns[ids.clamp_min(0)].T, torch.zeros(3, P, dtype=DT))
            Ds = torch.where(ids >= 0, sp["depth"], torch.zeros_like(sp["depth"]))
        else:
            Ns = torch.zeros(3, P, dtype=DT)
            Ds = torch.zeros(P, dtype=DT)
        den = opts.w_s + acc["wg"]
        out = dict(sp)
        out.update(cg=acc["cg"], wg=acc["wg"], image=(opts.w_s * sp["color_s"] + acc["cg"]) / den,
                   alpha_margin=acc["alpha_margin"], depth_margin=acc["depth_margin"],
                   near_margin_g=acc["near_margin"], count=acc["count"], normal_s=Ns, depth_g=acc["dg"],
                   normal_g=acc["ng"], depth_smooth=(Ds * opts.w_s + acc["dg"]) / den,
                   normal_smooth=(Ns * opts.w_s + acc["ng"]) / den)
    return out
