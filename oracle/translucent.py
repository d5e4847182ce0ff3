"""FP64 CPU oracle of the translucent-surfel render of the surfel optimisation
stage (Sec. 4.1, Eq. 6-7): TEST INFRASTRUCTURE ONLY (see the package notes).

A surfel is the disc of `render.py` -- centre p, rotation r, scales s, local
coordinates (x, y) scaled by s -- carrying an opacity that grows from a 2D
Gaussian into an opaque disc with the modulating parameter w:

    G(x, y) = exp(-(x^2 + y^2) / 2),   alpha = min(1, w G),
    alpha = 0 where min(alpha, G) < 1/255 (Eq. 6-7 and the text after them).

(x, y) are the local coordinates of the point where the pixel ray meets the
surfel's plane, the same intersection the opaque pass uses (G >= 1/255 is
exactly the opaque disc of radius sqrt(2 ln 255)).  The pixel colour is the
front-to-back alpha blend

    C = sum_k alpha_k T_k c_k + T_end bg,   T_1 = 1, T_{k+1} = T_k (1 - alpha_k)

over the surfels in the order of their centre depth (camera z of the centre,
smaller index first on a tie: the order a per-tile sort by centre depth
gives, since every surfel that reaches a pixel is in its tile's list).  With
`front_first` (the order adjustment used once w is large), the surfel with
the smallest depth at the pixel itself (camera z of the intersection point,
smaller index first on a tie) among those with alpha > 0 is blended first
and the others keep their order.  Alpha of the pixel is 1 - T_end and its
depth the blended sum_k alpha_k T_k z_k.  c_k is the surfel colour of Eq. 1.
Rays that meet a surfel's plane behind the near plane, or edge-on, do not
see it.

Gradients are torch autograd of this definition (the 1/255 rule and the
ordering are indicators; the clamp at 1 passes gradient only below 1).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from .render import DT, Cam, Options, _degree, _t, quat_to_rot, view_directions
from .sh import sh_colour

ALPHA_MIN = 1.0 / 255.0
U32 = 2.0 ** -24            # FP32 unit roundoff
SURFEL_KEYS = ("mean", "quat", "scale", "w", "sh")


def _frames(leaves, cam: Cam):
    mean, quat, scale, w, sh = (leaves[k] for k in SURFEL_KEYS)
    mu = (cam.R @ mean).T + cam.t                  # [N, 3]
    A = cam.R @ quat_to_rot(quat)                  # [N, 3, 3]
    col = sh_colour(sh, view_directions(mean, cam), _degree(sh))
    return dict(mu=mu, tu=A[:, :, 0], tv=A[:, :, 1], n=A[:, :, 2], scale=scale.T, w=w, colour=col)


def surfel_alphas(f, cam: Cam, pix: torch.Tensor):
    """Per (pixel, surfel): alpha (Eq. 6-7 with the 1/255 rule), the depth z
    of the ray's intersection with the surfel plane, and the margins of the
    discrete decisions: |ln(G / alpha_min)| and |ln(w G / alpha_min)| (the
    1/255 rule; +inf where the surfel is not in front), |ln(w G)| (the clamp
    at 1); and `dev`, a first-order bound on the deviation of an FP32
    evaluation of a kept alpha, alpha (dq / 2 + 4 u), from the roundings of
    q = u^2 + v^2 when u c is evaluated as U.r with the plane folded into
    U = (w t_u - (mu.t_u) n) / s_u: the pixel ray (x', y') = ((px + 1/2 -
    cx) / fx, ...) rounded twice (2 u |x'|, through the exact dq/dx'); U
    rounded 4 times relative to its two terms and U.r twice relative to its
    products -- 6 u (|n.mu||r.t_u| + |mu.t_u||n.r|) / (s_u |n.r|) in u,
    likewise v, the large terms that cancel down to u c for rays near a
    small, distant disc; n.r twice (2 u |r| / |n.r| relative) -- u the FP32
    unit roundoff; the exp2 and the reciprocal add 4 u."""
    r = cam.rays(pix)                                              # [P, 3]
    mu, tu, tv, n, sc = f["mu"], f["tu"], f["tv"], f["n"], f["scale"]
    nr = r @ n.T                                                   # [P, N]
    nmu = (n * mu).sum(-1)
    rnorm = torch.linalg.norm(r, dim=-1, keepdim=True)
    edge = nr.abs() <= 1e-12 * rnorm
    z = nmu / torch.where(edge, torch.ones_like(nr), nr)
    u = (z * (r @ tu.T) - (mu * tu).sum(-1)) / sc[:, 0]
    v = (z * (r @ tv.T) - (mu * tv).sum(-1)) / sc[:, 1]
    q = u * u + v * v
    G = torch.exp(-0.5 * q)
    wG = f["w"][None, :] * G
    a = torch.minimum(wG, torch.ones_like(wG))
    front = (~edge) & (z >= cam.znear)
    keep = front & (torch.minimum(a, G) >= ALPHA_MIN)
    alpha = torch.where(keep, a, torch.zeros_like(a))
    with torch.no_grad():
        inf = torch.full_like(q, math.inf)
        m_g = torch.where(front, (-0.5 * q - math.log(ALPHA_MIN)).abs(), inf)
        m_a = torch.where(front, (torch.log(wG.clamp_min(1e-300)) - math.log(ALPHA_MIN)).abs(), inf)
        m_c = torch.where(keep, torch.log(wG.clamp_min(1e-300)).abs(), inf)
        anr = nr.abs().clamp_min(1e-300)
        amu = nmu.abs()[None, :]
        rtu, rtv = r @ tu.T, r @ tv.T                               # [P, N]
        # dq/dr = 2 u du/dr + 2 v dv/dr, du/dr = (z / s_u)(t_u - (r.t_u) n / (n.r))
        zr = z / torch.where(edge, torch.ones_like(nr), nr)         # z / (n.r)
        dq = 0
        for c in range(2):                                         # x', y' (the ray's third component is 1)
            du = (z * tu[:, c][None, :] - zr * rtu * n[:, c][None, :]) / sc[:, 0][None, :]
            dv = (z * tv[:, c][None, :] - zr * rtv * n[:, c][None, :]) / sc[:, 1][None, :]
            dq = dq + (2 * u * du + 2 * v * dv).abs() * 2 * U32 * r[:, c].abs()[:, None]
        Au = amu * rtu.abs() + (mu * tu).sum(-1).abs()[None, :] * anr
        Av = amu * rtv.abs() + (mu * tv).sum(-1).abs()[None, :] * anr
        d_rec = 6 * U32 * (2 * u.abs() * Au / (sc[:, 0][None, :] * anr) + 2 * v.abs() * Av / (sc[:, 1][None, :] * anr))
        d_c = 2 * q * 2 * U32 * rnorm / anr
        dev = torch.where(keep, a * ((dq + d_rec + d_c) / 2 + 4 * U32), torch.zeros_like(a))
    return alpha, z, dict(g=m_g, a=m_a, clamp=m_c, dev=dev)


def translucent_render(scene, w, cam_idx=0, pix=None, front_first=False, leaves=None,
                       chunk_elems=4_000_000) -> Dict[str, torch.Tensor]:
    """Colour [3,P], alpha [P], blended depth [P], the front-first surfel [P]
    (-1: none or not front_first) and decision margins of the pixels `pix`
    (flat indices; default the whole image) of camera `cam_idx`.  w: the
    per-surfel opacity modulation [N].  `leaves` optionally passes autograd
    leaves for SURFEL_KEYS (see `translucent_gradients`).

    Margins (FP32 bookkeeping for the parity tests): `rule` the smallest
    1/255-rule margin over the surfels in front of the pixel, `clamp` the
    smallest |ln(w G)| over those kept, `front_gap` the relative depth gap
    between the two nearest kept surfels (+inf with fewer than two),
    `order_gap` the smallest relative gap between the centre depths of two
    kept surfels adjacent in the blend order (+inf with fewer than two):
    below the rounding of a centre depth the order is a near-tie;
    `alpha_dev` the sum over kept surfels of their FP32 alpha bound (see
    `surfel_alphas`): the colour of an FP32 blend can stray by up to
    2 max|c| alpha_dev, its alpha by alpha_dev."""
    cam = Cam(scene.cameras[cam_idx])
    if pix is None:
        pix = torch.arange(cam.W * cam.H)
    pix = torch.as_tensor(pix, dtype=torch.long)
    S = scene.surfels
    if leaves is None:
        leaves = dict(mean=_t(S.mean), quat=_t(S.quat), scale=_t(S.scale), w=_t(w), sh=_t(S.sh))
    f = _frames(leaves, cam)
    N = f["mu"].shape[0]
    order = torch.argsort(f["mu"][:, 2].detach(), stable=True)    # centre depth, smaller index first
    col = f["colour"][:, order]                                    # [3, N]
    cz = f["mu"][:, 2].detach()[order]                             # centre depths in blend order
    bg = cam.bg
    step = max(1, chunk_elems // max(N, 1))
    outs = []
    for s0 in range(0, pix.shape[0], step):
        p = pix[s0:s0 + step]
        P = p.shape[0]
        if N == 0:
            outs.append(dict(color=bg[:, None].expand(3, P).clone(), alpha=torch.zeros(P, dtype=DT),
                             depth=torch.zeros(P, dtype=DT), front=torch.full((P,), -1, dtype=torch.long),
                             rule=torch.full((P,), math.inf, dtype=DT),
                             clamp=torch.full((P,), math.inf, dtype=DT),
                             front_gap=torch.full((P,), math.inf, dtype=DT),
                             order_gap=torch.full((P,), math.inf, dtype=DT),
                             alpha_dev=torch.zeros(P, dtype=DT)))
            continue
        alpha, z, m = surfel_alphas(f, cam, p)
        a_s, z_s = alpha[:, order], z[:, order]                    # blend order
        with torch.no_grad():
            kept = a_s > 0
            zk = torch.where(kept, z_s, torch.full_like(z_s, math.inf))
            # nearest kept surfel at the pixel: smallest z, then smallest index
            zmin = zk.min(1).values
            has = torch.isfinite(zmin)
            cand = kept & (zk == zmin[:, None])
            ids = torch.where(cand, order[None, :].expand(P, N), torch.full_like(zk, N, dtype=torch.long))
            fid = ids.min(1).values
            fpos = torch.argmax((order[None, :] == fid[:, None]).to(torch.int8), dim=1)
            if N >= 2:
                z2 = torch.topk(zk, 2, dim=1, largest=False).values[:, 1]
                fgap = torch.where(torch.isfinite(z2), (z2 - zmin) / zmin, torch.full_like(z2, math.inf))
            else:
                fgap = torch.full((P,), math.inf, dtype=DT)
            # the previous kept place before each place, and the relative
            # centre-depth gap to it at kept places
            ar = torch.arange(N)[None, :].expand(P, N)
            kidx = torch.where(kept, ar, torch.full_like(ar, -1))
            prev = torch.cummax(torch.cat([torch.full((P, 1), -1, dtype=torch.long), kidx[:, :-1]], 1), 1).values
            gaps = (cz[None, :] - cz[prev.clamp_min(0)]).abs() / cz.abs()[None, :]
            ogap = torch.where(kept & (prev >= 0), gaps, torch.full_like(gaps, math.inf)).min(1).values
        if front_first:
            sel = torch.zeros_like(a_s, dtype=torch.bool)
            sel[torch.arange(P)[has], fpos[has]] = True
            a_f = (a_s * sel).sum(1)
            c_f = (col[:, None, :] * sel[None, :, :]).sum(2)       # [3, P]
            z_f = (z_s * sel).sum(1)
            a_r = torch.where(sel, torch.zeros_like(a_s), a_s)
        else:
            a_f = torch.zeros(P, dtype=DT)
            c_f = torch.zeros(3, P, dtype=DT)
            z_f = torch.zeros(P, dtype=DT)
            a_r = a_s
        one = torch.ones(P, 1, dtype=DT)
        T = torch.cumprod(torch.cat([one, 1 - a_r], 1), 1)         # [P, N+1]: T before each, then T_end
        wgt = a_r * T[:, :-1]
        rest_c = wgt @ col.T + T[:, -1:] * bg[None, :]             # [P, 3]
        rest_d = (wgt * torch.where(a_r > 0, z_s, torch.zeros_like(z_s))).sum(1)
        color = a_f[None, :] * c_f + (1 - a_f)[None, :] * rest_c.T
        Tend = (1 - a_f) * T[:, -1]
        depth = a_f * z_f + (1 - a_f) * rest_d
        outs.append(dict(color=color, alpha=1 - Tend, depth=depth,
                         front=torch.where(has & torch.tensor(front_first), fid, torch.full_like(fid, -1)),
                         rule=torch.minimum(m["g"], m["a"]).min(1).values,
                         clamp=m["clamp"].min(1).values, front_gap=fgap, order_gap=ogap,
                         alpha_dev=m["dev"].sum(1)))
    out = {}
    for k in outs[0]:
        out[k] = torch.cat([o[k] for o in outs], 1 if outs[0][k].dim() == 2 else 0)
    out["pix"] = pix
    out["surfel_colour"] = f["colour"]
    return out


def translucent_gradients(scene, w, dL_dC: np.ndarray, pix, cam_idx=0, front_first=False,
                          chunk_elems=2_000_000) -> Dict[str, np.ndarray]:
    """d(sum dL_dC * C)/d(surfel mean, quat, scale, w, sh) by autograd of the
    definition above.  dL_dC: [3, P] at the pixels `pix`."""
    S = scene.surfels
    leaves = dict(mean=_t(S.mean, True), quat=_t(S.quat, True), scale=_t(S.scale, True),
                  w=_t(w, True), sh=_t(S.sh, True))
    pix = torch.as_tensor(pix, dtype=torch.long)
    g = _t(dL_dC).reshape(3, -1)
    step = max(1, chunk_elems // max(S.n, 1))
    for s0 in range(0, pix.shape[0], step):
        out = translucent_render(scene, w, cam_idx, pix[s0:s0 + step], front_first, leaves=leaves)
        loss = (out["color"] * g[:, s0:s0 + step]).sum()
        if loss.requires_grad:
            loss.backward()
    return {k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape)) for k, v in leaves.items()}


def translucent_fd(scene, w, dL_dC: np.ndarray, pix, which, cam_idx=0, front_first=False, rel_h=1e-6):
    """Central differences of sum dL_dC * C for (group, flat index) pairs of
    SURFEL_KEYS, at h and h/4 (NaN where the two disagree: the step crossed a
    discontinuity)."""
    import copy
    pix = torch.as_tensor(pix, dtype=torch.long)
    g = _t(dL_dC).reshape(3, -1)
    base = dict(mean=scene.surfels.mean, quat=scene.surfels.quat, scale=scene.surfels.scale, w=w,
                sh=scene.surfels.sh)
    base64 = {k: np.asarray(v, dtype=np.float64) for k, v in base.items()}

    def loss_at(group, flat, delta):
        arrs = {k: v.copy() for k, v in base64.items()}
        arrs[group].reshape(-1)[flat] += delta
        sc = copy.copy(scene)
        sc.surfels = copy.copy(scene.surfels)
        for k in ("mean", "quat", "scale", "sh"):
            setattr(sc.surfels, k, arrs[k])
        with torch.no_grad():
            out = translucent_render(sc, arrs["w"], cam_idx, pix, front_first)
        return float((out["color"] * g).sum())

    res = np.empty(len(which))
    for i, (group, flat) in enumerate(which):
        x = base64[group].reshape(-1)[flat]
        h = rel_h * max(1.0, abs(x))
        f1 = (loss_at(group, flat, h) - loss_at(group, flat, -h)) / (2 * h)
        f2 = (loss_at(group, flat, h / 4) - loss_at(group, flat, -h / 4)) / (h / 2)
        scale = max(abs(f1), abs(f2), 1e-12)
        res[i] = f1 if abs(f1 - f2) <= 1e-4 * scale + 1e-9 else np.nan
    return res
