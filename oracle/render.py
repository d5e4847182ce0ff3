"""FP64 CPU oracle of the Gaussian-enhanced-surfel two-pass render.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the HIP product path
never does, and this module imports nothing from it.

It is the plain per-pixel definition of the method, evaluated by brute force
(every pixel against every primitive), in float64 with torch CPU ops:

* Surfels (Sec. 3): a disc of radius R_s on the local XY plane, placed by
  scale s (2D), rotation r and translation p.  Pass 1 is a z-buffer: each
  pixel shows the nearest surfel whose disc its ray hits; D_s is that depth
  and C_s that surfel's colour.  The opaque disc radius is sqrt(2 ln 255)
  (the radius where the opacity-modulated surfel of Sec. 4.1, Eq. 6-7 at
  w = 255 stops being opaque).
* Colour (Eq. 1): the SH colour in the direction from the primitive centre to
  the camera, offset by 1/2 and clamped at 0 (see `sh.py`).
* Gaussians (Eq. 2-4): alpha = sigma exp(-q/2) with q the Mahalanobis
  distance under the projected covariance, set to zero below 1/255; a
  Gaussian counts at a pixel only if its centre depth d_i < D_s + eps_i with
  eps_i = (5/D) sum_j s_ij, D = 3 (Sec. 5).  C_G = sum alpha c, W_G = sum alpha.
* Composite (Eq. 5): C = (C_s W_s + C_G) / (W_s + W_G), W_s = 1.

Readings of points the paper leaves open are listed in the design notes; the
ones that change numbers are: pixel centres at +1/2, camera-space z as depth,
near plane 0.2 (surfel hits and Gaussian centres), 3DGS's projected
covariance (1.3 x half-fov clamp of x/z, y/z in the Jacobian, +0.3 I
dilation), strict depth test, inclusive disc rim and alpha threshold, smallest
index wins an exact depth tie, uncovered pixels show the background colour.

Gradients are torch autograd of this same definition (indicator functions,
the alpha threshold and the SH clamp contribute zero derivative, exactly as
autograd treats them); they are pinned to FP64 central differences in the
tests.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np
import torch

from .sh import sh_colour

DT = torch.float64
SURFEL_RADIUS = math.sqrt(2.0 * math.log(255.0))


@dataclasses.dataclass
class Options:
    surfel_radius: float = SURFEL_RADIUS
    eps_factor: float = 5.0      # eps_i = eps_factor / 3 * (s1 + s2 + s3)
    eps_const: float = -1.0      # >= 0: constant eps for every Gaussian
    alpha_min: float = 1.0 / 255.0
    dilation: float = 0.3
    w_s: float = 1.0
    surfel_samples: int = 1      # 1, or 4: the surfel pass supersampled 2x2 (Sec. 5)
    mip_2d: float = 0.0          # > 0: Mip-GES screen-space filter variance (replaces `dilation`)


# ----------------------------------------------------------------------------
# helpers


def _t(a, requires_grad=False):
    t = torch.as_tensor(np.asarray(a), dtype=DT).clone()
    if requires_grad:
        t.requires_grad_(True)
    return t


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrices [n,3,3] of quaternions q [4][n] (w,x,y,z), normalised first."""
    q = q / torch.linalg.norm(q, dim=0, keepdim=True)
    w, x, y, z = q[0], q[1], q[2], q[3]
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=-1)
    return r.reshape(-1, 3, 3)


class Cam:
    """float64 view of a synth.Camera."""

    def __init__(self, cam):
        self.W, self.H = int(cam.width), int(cam.height)
        self.fx, self.fy = float(cam.fx), float(cam.fy)
        self.cx, self.cy = float(cam.cx), float(cam.cy)
        self.R = _t(cam.R).reshape(3, 3)
        self.t = _t(cam.t).reshape(3)
        self.znear = float(cam.znear)
        self.bg = _t(cam.bg).reshape(3)
        self.o = -self.R.T @ self.t  # camera centre in world space

    def rays(self, pix: torch.Tensor, offset=(0.0, 0.0)) -> torch.Tensor:
        """Camera-space rays (x', y', 1) through pixel centres, pix = flat
        index; `offset` moves the point inside the pixel (sample positions)."""
        px = (pix % self.W).to(DT) + 0.5 + offset[0]
        py = torch.div(pix, self.W, rounding_mode="floor").to(DT) + 0.5 + offset[1]
        return torch.stack([(px - self.cx) / self.fx, (py - self.cy) / self.fy,
                            torch.ones_like(px)], dim=-1)

    def centres(self, pix: torch.Tensor) -> torch.Tensor:
        px = (pix % self.W).to(DT) + 0.5
        py = torch.div(pix, self.W, rounding_mode="floor").to(DT) + 0.5
        return torch.stack([px, py], dim=-1)


def _degree(sh) -> int:
    return int(round(math.sqrt(sh.shape[0]))) - 1


# ----------------------------------------------------------------------------
# per-primitive quantities of one view


def surfel_frames(S, cam: Cam, sh=None) -> Dict[str, torch.Tensor]:
    """Camera-space centre, unit tangent axes and normal of every surfel, and
    its colour in this view (Eq. 1).  `sh` overrides S.sh (autograd leaf)."""
    mean = _t(S.mean)                       # [3, N]
    mu = (cam.R @ mean).T + cam.t           # [N, 3]
    A = cam.R @ quat_to_rot(_t(S.quat))     # [N, 3, 3]
    sh = _t(S.sh) if sh is None else sh
    d = view_directions(mean, cam)
    return dict(mu=mu, tu=A[:, :, 0], tv=A[:, :, 1], n=A[:, :, 2],
                scale=_t(S.scale).T, colour=sh_colour(sh, d, _degree(sh)))


def view_directions(mean: torch.Tensor, cam: Cam) -> torch.Tensor:
    """Unit directions [n, 3] from each primitive centre (mean [3][n], world)
    to the camera centre o (Sec. 3, the text after Eq. 1; reading R6)."""
    d = cam.o[:, None] - mean
    return (d / torch.linalg.norm(d, dim=0, keepdim=True)).T


def ewa_jacobian(mu: torch.Tensor, cam: Cam) -> torch.Tensor:
    """Jacobian [M, 2, 3] of the perspective map (x, y, z) -> (fx x/z + cx,
    fy y/z + cy) at the camera-space centres mu [M, 3], the local affine
    approximation of the projected covariance (Eq. 4; reading R10: x/z and
    y/z are first clamped to 1.3 x the tangent of the half field of view)."""
    z = mu[:, 2]
    limx = 1.3 * cam.W / (2.0 * cam.fx)
    limy = 1.3 * cam.H / (2.0 * cam.fy)
    xc = torch.clamp(mu[:, 0] / z, -limx, limx) * z
    yc = torch.clamp(mu[:, 1] / z, -limy, limy) * z
    zero = torch.zeros_like(z)
    return torch.stack([
        torch.stack([cam.fx / z, zero, -cam.fx * xc / (z * z)], dim=-1),
        torch.stack([zero, cam.fy / z, -cam.fy * yc / (z * z)], dim=-1)], dim=1)


def projected_covariance(J: torch.Tensor, Rcam: torch.Tensor, sig3: torch.Tensor,
                         dilation: float) -> torch.Tensor:
    """Screen-space covariance [M, 2, 2] = J W Sigma3 W^T J^T + dilation I
    (Eq. 4's Sigma; W = the world-to-camera rotation; reading R11)."""
    T = J @ Rcam
    return T @ sig3 @ T.transpose(1, 2) + dilation * torch.eye(2, dtype=DT)


def filter_compensation(det_before: torch.Tensor, det_after: torch.Tensor) -> torch.Tensor:
    """Opacity factor that keeps a Gaussian's integral when a low-pass filter
    widens its covariance: the Gaussian's normaliser goes with sqrt(det)."""
    return torch.sqrt(det_before / det_after)


def gaussian_projection(G, cam: Cam, opts: Options, params=None) -> Dict[str, torch.Tensor]:
    """Projected centre, conic, depth, eps, opacity and colour of every
    Gaussian in this view (Eq. 4 and the text after it; Sec. 5 for eps).

    `params` optionally supplies autograd leaves (mean, quat, scale, opacity,
    sh) in the same layouts as the Gaussians arrays."""
    if params is None:
        params = dict(mean=_t(G.mean), quat=_t(G.quat), scale=_t(G.scale),
                      opacity=_t(G.opacity), sh=_t(G.sh))
    mean, quat, scale = params["mean"], params["quat"], params["scale"]
    mu = (cam.R @ mean).T + cam.t                     # [M, 3]
    valid = mu[:, 2] > cam.znear
    Rq = quat_to_rot(quat)
    Msc = Rq * scale.T[:, None, :]                    # Rq diag(s)
    sig3 = Msc @ Msc.transpose(1, 2)                  # world covariance
    z = mu[:, 2]
    opac = params["opacity"]
    if G.filter3d is not None:
        # Mip-GES world-space filter: Sigma3 + v I, opacity scaled so that the
        # Gaussian's integral is kept: sqrt(det Sigma3 / det(Sigma3 + v I))
        v = _t(G.filter3d)
        sig3 = sig3 + v[:, None, None] * torch.eye(3, dtype=DT)
        s2 = scale * scale
        opac = opac * filter_compensation(s2.prod(0), (s2 + v[None, :]).prod(0))
    if opts.mip_2d > 0:
        # Mip-GES screen-space filter: Sigma2 + e I in place of the dilation,
        # opacity scaled by sqrt(det Sigma2 / det(Sigma2 + e I))
        base = projected_covariance(ewa_jacobian(mu, cam), cam.R, sig3, 0.0)
        sig2 = base + opts.mip_2d * torch.eye(2, dtype=DT)
        opac = opac * filter_compensation(torch.linalg.det(base), torch.linalg.det(sig2))
    else:
        sig2 = projected_covariance(ewa_jacobian(mu, cam), cam.R, sig3, opts.dilation)
    det = sig2[:, 0, 0] * sig2[:, 1, 1] - sig2[:, 0, 1] * sig2[:, 1, 0]
    conic = torch.stack([sig2[:, 1, 1] / det, -sig2[:, 0, 1] / det,
                         sig2[:, 0, 0] / det], dim=-1)   # (a, b, c) of the inverse
    phat = torch.stack([cam.fx * mu[:, 0] / z + cam.cx,
                        cam.fy * mu[:, 1] / z + cam.cy], dim=-1)
    if opts.eps_const >= 0:
        eps = torch.full_like(z, opts.eps_const)
    else:
        eps = opts.eps_factor / 3.0 * scale.sum(dim=0)
    colour = sh_colour(params["sh"], view_directions(mean, cam), _degree(params["sh"]))
    return dict(mu=mu, valid=valid, phat=phat, conic=conic, cov2=sig2, depth=z,
                eps=eps, opacity=opac, colour=colour)


# ----------------------------------------------------------------------------
# pass 1: surfels


# 2x2 supersampling of the surfel pass (Sec. 5: the pass rendered at twice
# the resolution and downsampled): sample (a, b) of pixel (i, j) sits at
# (i + 1/4 + a/2, j + 1/4 + b/2), the pixel centre (2i + a + 1/2, 2j + b + 1/2)
# of the doubled image; order (0,0), (1,0), (0,1), (1,1).
SAMPLE_OFFSETS = ((-0.25, -0.25), (0.25, -0.25), (-0.25, 0.25), (0.25, 0.25))


def surfel_pass(frames, cam: Cam, pix: torch.Tensor, opts: Options, tie_rel=1e-5,
                band_rel=1e-4, offset=(0.0, 0.0)):
    """Nearest surfel hit for each pixel in `pix` (brute force over surfels).

    Returns depth D_s (+inf if none), id (-1 if none), the number of surfels
    whose hit depth lies within `tie_rel` (relative) of D_s (1 = unique), a
    padded list of those candidate ids, the relative gap (z2 - D_s) / D_s from
    the nearest hit to the next one (+inf with fewer than two hits), and
    margins of the discrete decisions
    that could change the winner (for tolerance bookkeeping in tests):
      rim:   min |u^2+v^2-R^2|/R^2 over surfels with depth <= D_s(1+band_rel)
      near:  min |z - znear|/znear over those surfels hitting within the rim.
    The same margins divided by the condition number of the decision (how
    much a relative perturbation of size e of the inputs -- centre, frame,
    ray -- can move the decided quantity, in units of e), for comparisons
    with an evaluation in lower precision:
      gap_k:  gap / (kz_1 + kz_2), kz = |mu|/|n.mu| + |r|/|n.r| for the
              nearest and the next hit (the relative condition of z =
              n.mu / n.r); +inf with fewer than two hits;
      rim_k:  min over the same surfels of the rim margin / k_rim, with
              k_rim = 2 (|u|/R T_u + |v|/R T_v) + 2 |r|/|n.r| and
              T_u = (|n.mu||r.t_u| + |mu.t_u||n.r|) / (s_u R |n.r|) the size
              of the terms that cancel in u (likewise v);
      near_k: min of near / kz;
      kz_win: kz of the winning surfel (0 where none).
    """
    r = cam.rays(pix, offset)                             # [P, 3]
    mu, tu, tv, n, sc = (frames[k] for k in ("mu", "tu", "tv", "n", "scale"))
    N = mu.shape[0]
    P = r.shape[0]
    if N == 0:
        inf = torch.full((P,), math.inf, dtype=DT)
        return dict(depth=inf, id=torch.full((P,), -1, dtype=torch.long),
                    ties=torch.zeros(P, dtype=torch.long), gap=inf.clone(),
                    cands=torch.full((P, 1), -1, dtype=torch.long),
                    rim=torch.full((P,), math.inf, dtype=DT),
                    near=torch.full((P,), math.inf, dtype=DT), gap_k=inf.clone(),
                    rim_k=inf.clone(), near_k=inf.clone(), kz_win=torch.zeros(P, dtype=DT))
    R2 = opts.surfel_radius ** 2
    nr = r @ n.T                                          # n . r
    nmu = (n * mu).sum(-1)                                # n . mu
    rnorm = torch.linalg.norm(r, dim=-1, keepdim=True)
    edge = nr.abs() <= 1e-12 * rnorm
    z = nmu / torch.where(edge, torch.ones_like(nr), nr)  # hit depth along the ray
    # (X - mu) . t = z (r . t) - mu . t  with X = z r
    u = (z * (r @ tu.T) - (mu * tu).sum(-1)) / sc[:, 0]
    v = (z * (r @ tv.T) - (mu * tv).sum(-1)) / sc[:, 1]
    rho = u * u + v * v
    front = (~edge) & (z >= cam.znear)
    hit = front & (rho <= R2)
    zh = torch.where(hit, z, torch.full_like(z, math.inf))
    depth, idx = zh.min(dim=1)                            # first index on exact ties
    none = torch.isinf(depth)
    idx = torch.where(none, torch.full_like(idx, -1), idx)
    tie_mask = hit & (zh <= depth[:, None] * (1 + tie_rel))
    ties = tie_mask.sum(1)
    # relative gap from the nearest hit to the next one (inf with < 2 hits)
    if N >= 2:
        z2 = torch.topk(zh, 2, dim=1, largest=False).values[:, 1]
        gap = torch.where(torch.isinf(z2), torch.full_like(z2, math.inf), (z2 - depth) / depth)
    else:
        gap = torch.full((P,), math.inf, dtype=DT)
    # condition numbers of the decisions (bookkeeping only)
    anr = nr.abs().clamp_min(1e-300)
    anmu = nmu.abs().clamp_min(1e-300)
    kz = torch.linalg.norm(mu, dim=-1)[None, :] / anmu[None, :] + rnorm / anr      # [P, N]
    kz_win = torch.where(none, torch.zeros_like(depth), torch.gather(kz, 1, idx.clamp_min(0)[:, None])[:, 0])
    if N >= 2:
        top2 = torch.topk(zh, 2, dim=1, largest=False).indices
        ksum = torch.gather(kz, 1, top2).sum(1)
        gap_k = torch.where(torch.isinf(gap), gap, gap / ksum)
    else:
        gap_k = gap.clone()
    R = math.sqrt(R2)
    Tu = (anmu[None, :] * (r @ tu.T).abs() + (mu * tu).sum(-1).abs()[None, :] * anr) / (sc[:, 0][None, :] * R * anr)
    Tv = (anmu[None, :] * (r @ tv.T).abs() + (mu * tv).sum(-1).abs()[None, :] * anr) / (sc[:, 1][None, :] * R * anr)
    k_rim = 2 * (u.abs() / R * Tu + v.abs() / R * Tv) + 2 * rnorm / anr
    kmax = max(1, int(ties.max()))
    order = torch.argsort((~tie_mask).to(torch.int8), dim=1, stable=True)[:, :kmax]
    cands = torch.where(torch.gather(tie_mask, 1, order), order,
                        torch.full_like(order, -1))
    relevant = (~edge) & (z >= cam.znear * (1 - band_rel)) & (
        z <= torch.where(none, torch.full_like(depth, math.inf), depth * (1 + band_rel))[:, None])
    rim_m = torch.where(relevant, (rho - R2).abs() / R2, torch.full_like(z, math.inf))
    rim = rim_m.min(1).values
    rim_k = (rim_m / k_rim).min(1).values
    near_rel = (~edge) & (rho <= R2 * (1 + band_rel))
    near_m = torch.where(near_rel, (z - cam.znear).abs() / cam.znear, torch.full_like(z, math.inf))
    near = near_m.min(1).values
    near_k = (near_m / kz).min(1).values
    return dict(depth=depth, id=idx, ties=ties, gap=gap, cands=cands, rim=rim, near=near, gap_k=gap_k,
                rim_k=rim_k, near_k=near_k, kz_win=kz_win)


# ----------------------------------------------------------------------------
# pass 2: Gaussians


def gaussian_pass(proj, cam: Cam, pix: torch.Tensor, depth_s: torch.Tensor, opts: Options,
                  band_rel=1e-4, kz_win=None, band=None):
    """C_G, W_G (Eq. 2-3) for each pixel in `pix`, with margins of the alpha
    threshold (|alpha/alpha_min - 1|) and of the depth test
    (|d - D_s - eps| / (D_s + eps)) over the Gaussians near those decisions.

    Bookkeeping for lower-precision comparisons: the same margins divided by
    their condition numbers (see `surfel_pass`):
      alpha_k: |ln(alpha / alpha_min)| / k_a, with k_a = |ln sigma| +
               q/2 (1 + cond(Sigma_2)) + |Sigma_2^-1 d| (|p_hat| + |x|) the
               sensitivity of ln alpha to relative perturbations of sigma,
               of the conic and of the pixel and projected-centre
               coordinates (taken as absolute positions);
      depth_k: k_d = (D_s kz_win + |mu| + eps + d) / (D_s + eps), with
               kz_win the winning surfel's depth condition (`kz_win`).
    With `band`, also the [P, M] masks `pair_band` (either scaled margin of
    the pair below `band`) and `reach` (alpha >= alpha_min, or in band)."""
    P = pix.shape[0]
    M = proj["depth"].shape[0]
    if M == 0:
        zero = torch.zeros((P,), dtype=DT)
        inf = torch.full((P,), math.inf, dtype=DT)
        return dict(cg=torch.zeros((3, P), dtype=DT), wg=zero, alpha_margin=inf,
                    depth_margin=inf, count=torch.zeros(P, dtype=torch.long),
                    alpha_k=inf.clone(), depth_k=inf.clone())
    x = cam.centres(pix)                                   # [P, 2]
    dx = x[:, None, 0] - proj["phat"][None, :, 0]
    dy = x[:, None, 1] - proj["phat"][None, :, 1]
    a, b, c = proj["conic"][:, 0], proj["conic"][:, 1], proj["conic"][:, 2]
    q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
    alpha = proj["opacity"] * torch.exp(-0.5 * q)
    with torch.no_grad():
        lim = depth_s[:, None] + proj["eps"][None, :]
        depth_ok = proj["depth"][None, :] < lim
        valid = proj["valid"][None, :]
        keep = valid & depth_ok & (alpha >= opts.alpha_min)
        am = (alpha / opts.alpha_min - 1).abs()
        alpha_margin = torch.where(valid & (proj["depth"][None, :] < lim * (1 + band_rel)), am,
                                   torch.full_like(am, math.inf)).min(1).values
        dm = (proj["depth"][None, :] - lim).abs() / lim.abs()
        dm = torch.where(torch.isfinite(lim), dm, torch.full_like(dm, math.inf))
        dmm = torch.where(valid & (alpha >= opts.alpha_min * (1 - band_rel)), dm, torch.full_like(dm, math.inf))
        depth_margin = dmm.min(1).values
        count = keep.sum(1)
        # condition numbers (bookkeeping only)
        cov = proj["cov2"]
        tr = cov[:, 0, 0] + cov[:, 1, 1]
        det = cov[:, 0, 0] * cov[:, 1, 1] - cov[:, 0, 1] * cov[:, 1, 0]
        disc = torch.sqrt(torch.clamp_min(tr * tr / 4 - det, 0))
        cond = (tr / 2 + disc) / torch.clamp_min(tr / 2 - disc, 1e-300)
        gx, gy = a * dx + b * dy, b * dx + c * dy
        pos = (gx.abs() * (proj["phat"][None, :, 0].abs() + x[:, None, 0].abs())
               + gy.abs() * (proj["phat"][None, :, 1].abs() + x[:, None, 1].abs()))
        k_a = torch.log(proj["opacity"]).abs()[None, :] + 0.5 * q * (1 + cond[None, :]) + pos
        lm = (torch.log(proj["opacity"])[None, :] - 0.5 * q - math.log(opts.alpha_min)).abs()  # |ln(alpha/alpha_min)|
        alpha_k = torch.where(valid & (proj["depth"][None, :] < lim * (1 + band_rel)), lm / k_a,
                              torch.full_like(am, math.inf)).min(1).values
        kzw = torch.zeros_like(depth_s) if kz_win is None else kz_win
        ds_f = torch.where(torch.isfinite(depth_s), depth_s, torch.zeros_like(depth_s))
        k_d = (ds_f[:, None] * kzw[:, None] + torch.linalg.norm(proj["mu"], dim=-1)[None, :]
               + proj["eps"][None, :] + proj["depth"][None, :].abs()) / lim.abs()
        depth_k = (dmm / k_d).min(1).values
        extra = {}
        if band is not None:
            a_band = valid & (lm / k_a < band)
            reach = (valid & (alpha >= opts.alpha_min)) | a_band
            extra = dict(pair_band=a_band | (reach & (dm / k_d < band)), reach=reach)
    w = torch.where(keep, alpha, torch.zeros_like(alpha))  # [P, M]
    cg = proj["colour"] @ w.T                              # [3, P]
    wg = w.sum(1)
    return dict(cg=cg, wg=wg, alpha_margin=alpha_margin, depth_margin=depth_margin,
                count=count, w=w, alpha_k=alpha_k, depth_k=depth_k, **extra)


# ----------------------------------------------------------------------------
# full render


def render(scene, cam_idx=0, pix=None, opts: Optional[Options] = None, chunk_elems=4_000_000,
           gauss=None, surfel_sh=None):
    """Render the pixels `pix` (flat indices; default: whole image) of camera
    `cam_idx`.  Returns float64 tensors: image [3,P], C_s [3,P], D_s [P],
    id [P], C_G [3,P], W_G [P], ties [P], cands [P,k] and decision margins.

    With opts.surfel_samples = 4 the surfel pass is evaluated at the four
    sample points of each pixel (SAMPLE_OFFSETS): C_s is the mean of the
    samples' colours (the background for a sample no surfel covers) and D_s
    the mean depth of the samples that hit a surfel (+inf if none), the
    D_s pass 2 tests against.  sample_id / sample_depth [4,P] hold the
    samples' own results; id, cands and ties refer to sample 0 and the
    margins to the worst sample.

    `gauss` / `surfel_sh` optionally pass autograd leaves (see `gradients`)."""
    opts = opts or Options()
    cam = Cam(scene.cameras[cam_idx])
    if pix is None:
        pix = torch.arange(cam.W * cam.H)
    pix = torch.as_tensor(pix, dtype=torch.long)
    S, G = scene.surfels, scene.gaussians
    frames = surfel_frames(S, cam, sh=surfel_sh)
    proj = gaussian_projection(G, cam, opts, params=gauss)
    width = max(S.n, G.m, 1)
    step = max(1, chunk_elems // width)
    outs = []
    offsets = SAMPLE_OFFSETS if opts.surfel_samples == 4 else ((0.0, 0.0),)
    for s0 in range(0, pix.shape[0], step):
        p = pix[s0:s0 + step]
        with torch.no_grad():
            sps = [surfel_pass({k: v.detach() for k, v in frames.items()}, cam, p, opts, offset=o)
                   for o in offsets]
        bgp = cam.bg[:, None].expand(3, p.shape[0])
        css = []
        for sp in sps:
            ids = sp["id"]
            css.append(bgp if S.n == 0 else
                       torch.where(ids[None, :] >= 0, frames["colour"][:, ids.clamp_min(0)], bgp))
        cs = sum(css) / len(css)                           # the samples' mean colour
        if len(sps) == 1:
            sp = sps[0]
            depth = sp["depth"]
        else:
            # the samples' mean depth over those that hit a surfel (+inf if none)
            with torch.no_grad():
                dz = torch.stack([x["depth"] for x in sps])
                hit = torch.isfinite(dz)
                nh = hit.sum(0)
                depth = torch.where(nh > 0, torch.where(hit, dz, torch.zeros_like(dz)).sum(0) / nh.clamp_min(1),
                                    torch.full_like(dz[0], math.inf))
            sp = dict(id=sps[0]["id"], ties=torch.stack([x["ties"] for x in sps]).max(0).values,
                      gap=torch.stack([x["gap"] for x in sps]).min(0).values,
                      cands=sps[0]["cands"],
                      rim=torch.stack([x["rim"] for x in sps]).min(0).values,
                      near=torch.stack([x["near"] for x in sps]).min(0).values,
                      gap_k=torch.stack([x["gap_k"] for x in sps]).min(0).values,
                      rim_k=torch.stack([x["rim_k"] for x in sps]).min(0).values,
                      near_k=torch.stack([x["near_k"] for x in sps]).min(0).values,
                      kz_win=torch.stack([x["kz_win"] for x in sps]).max(0).values)
        gp = gaussian_pass(proj, cam, p, depth, opts, kz_win=sp["kz_win"])
        img = (opts.w_s * cs + gp["cg"]) / (opts.w_s + gp["wg"])
        o = dict(image=img, color_s=cs, depth=depth, id=sp["id"], ties=sp["ties"], gap=sp["gap"],
                 cands=sp["cands"], rim=sp["rim"], near=sp["near"], cg=gp["cg"],
                 wg=gp["wg"], alpha_margin=gp["alpha_margin"],
                 depth_margin=gp["depth_margin"], count=gp["count"], gap_k=sp["gap_k"],
                 rim_k=sp["rim_k"], near_k=sp["near_k"], alpha_k=gp["alpha_k"],
                 depth_k=gp["depth_k"], kz_win=sp["kz_win"])
        if len(sps) > 1:
            o["sample_id"] = torch.stack([x["id"] for x in sps])          # [4, P]
            o["sample_depth"] = torch.stack([x["depth"] for x in sps])    # [4, P]
            o["sample_gap"] = torch.stack([x["gap"] for x in sps])
            o["sample_amb"] = torch.stack([torch.minimum(x["rim_k"], x["near_k"]) for x in sps])
            for k in range(4):
                o[f"sample_cands{k}"] = sps[k]["cands"]
        outs.append(o)
    out = {}
    for k in outs[0]:
        if k == "cands" or k.startswith("sample_cands"):
            kk = max(o[k].shape[1] for o in outs)
            out[k] = torch.cat([torch.nn.functional.pad(o[k], (0, kk - o[k].shape[1]), value=-1)
                                for o in outs], 0)
        elif outs[0][k].dim() == 2 and k != "cands":
            out[k] = torch.cat([o[k] for o in outs], 1)
        else:
            out[k] = torch.cat([o[k] for o in outs], 0)
    out["pix"] = pix
    out["surfel_colour"] = frames["colour"]
    return out


def ambiguous(out, rim_tol=1e-4, tie_tol=None, alpha_tol=1e-4, depth_tol=1e-5, near_tol=1e-5):
    """Pixels where an FP32 evaluation may legitimately take a different
    discrete decision than FP64: surfel rim / near plane, alpha threshold,
    depth test.  Depth ties are reported separately (`ties` > 1)."""
    return ((out["rim"] < rim_tol) | (out["near"] < near_tol)
            | (out["alpha_margin"] < alpha_tol) | (out["depth_margin"] < depth_tol))


# ----------------------------------------------------------------------------
# pruning scores


def score_colour(colour: torch.Tensor) -> torch.Tensor:
    """c_{i,j} of Eq. 9: the largest of the three channels of each
    Gaussian's colour [3][M] in this view."""
    return colour.max(0).values


def pixel_max(val: torch.Tensor) -> torch.Tensor:
    """The max over pixels (rows of [P, M]) of Eq. 9."""
    return val.max(0).values


def frontmost_counts(ids: torch.Tensor, n: int) -> torch.Tensor:
    """n_{i,j}: how many pixels of the id map show surfel i (-1: none)."""
    return torch.bincount(ids[ids >= 0], minlength=n)


def scores(scene, cam_idx=0, opts: Optional[Options] = None, chunk_elems=4_000_000,
           band=32 * 2.0 ** -24, tie_rel=1e-6):
    """Pruning scores of one view, by their plain definitions.

    cover [N] int: n_{i,j} of the surfel pruning step (Sec. 4.1, surfel
      pruning): the number of pixels where surfel i is the frontmost surfel
      covering them, i.e. the pixels of the id map equal to i.
    contrib [M] float: s_{i,j} of Eq. 9 (Sec. 4.2): over the pixels the
      Gaussian covers -- read as the pixels where it contributes to C_G and
      W_G (alpha >= alpha_min and the depth test passes) -- the largest
      c alpha / (W_s + W_G), with c the largest channel of its colour in this
      view; 0 where it contributes to no pixel.
    Bookkeeping for comparisons with an FP32 evaluation: `surfel_band` [N]
    marks surfels that win, or tie for, a pixel where the surfel decision is
    within its band (condition-scaled rim or near-plane margin below `band`,
    or a depth tie closer than `tie_rel`); `gauss_band` [M] marks Gaussians
    with a pixel where their alpha threshold or depth test is within its band,
    or that reach (alpha >= alpha_min, or in band) a pixel whose surfel
    decision is within its band (see `surfel_pass`, `gaussian_pass`)."""
    opts = opts or Options()
    cam = Cam(scene.cameras[cam_idx])
    S, G = scene.surfels, scene.gaussians
    N, M = S.n, G.m
    pix_all = torch.arange(cam.W * cam.H)
    cover = torch.zeros(N, dtype=torch.long)
    contrib = torch.zeros(M, dtype=DT)
    surfel_band = torch.zeros(N, dtype=torch.bool)
    gauss_band = torch.zeros(M, dtype=torch.bool)
    with torch.no_grad():
        frames = surfel_frames(S, cam)
        proj = gaussian_projection(G, cam, opts)
        cmax = score_colour(proj["colour"]) if M else torch.zeros(0, dtype=DT)
        step = max(1, chunk_elems // max(N, M, 1))
        for s0 in range(0, pix_all.shape[0], step):
            p = pix_all[s0:s0 + step]
            sp = surfel_pass(frames, cam, p, opts, tie_rel=tie_rel)
            ids = sp["id"]
            if N:
                cover += frontmost_counts(ids, N)
            amb_s = (sp["rim_k"] < band) | (sp["near_k"] < band) | (sp["ties"] > 1)
            c = sp["cands"][amb_s]
            surfel_band[c[c >= 0]] = True
            wid = ids[amb_s]
            surfel_band[wid[wid >= 0]] = True
            if not M:
                continue
            gp = gaussian_pass(proj, cam, p, sp["depth"], opts, kz_win=sp["kz_win"], band=band)
            val = gp["w"] / (opts.w_s + gp["wg"])[:, None]           # [P, M]
            contrib = torch.maximum(contrib, pixel_max(val))
            gauss_band |= (gp["pair_band"] | (gp["reach"] & amb_s[:, None])).any(0)
        contrib = contrib * cmax
    return dict(cover=cover, contrib=contrib, surfel_band=surfel_band, gauss_band=gauss_band)


def mip_filter3d(G, cams, scale2=0.2) -> np.ndarray:
    """Variance of each Gaussian's Mip-GES world-space filter (Sec. 6.1,
    after Mip-Splatting): scale2 times the squared world size of a pixel of
    the finest view that sees the Gaussian, (z / f_x)^2 minimised over the
    cameras whose image contains its projected centre (z > znear); 0 for a
    Gaussian no camera sees."""
    mean = _t(G.mean)
    best = torch.full((G.m,), math.inf, dtype=DT)
    for c in cams:
        cam = Cam(c)
        mu = (cam.R @ mean).T + cam.t
        z = mu[:, 2]
        zs = torch.where(z > 0, z, torch.ones_like(z))
        u = cam.fx * mu[:, 0] / zs + cam.cx
        w = cam.fy * mu[:, 1] / zs + cam.cy
        seen = (z > cam.znear) & (u >= 0) & (u <= cam.W) & (w >= 0) & (w <= cam.H)
        best = torch.where(seen, torch.minimum(best, z / cam.fx), best)
    return torch.where(torch.isfinite(best), scale2 * best * best, torch.zeros_like(best)).numpy()


# ----------------------------------------------------------------------------
# geometry channels (2D-GES depth / normal smoothing)


def facing(n: torch.Tensor, to_cam: torch.Tensor) -> torch.Tensor:
    """Unit normals n [k,3] flipped to face the camera: n . to_cam >= 0
    (to_cam: the primitive centre -> camera vectors [k,3])."""
    sgn = torch.where((n * to_cam).sum(-1) < 0, -torch.ones_like(n[:, 0]), torch.ones_like(n[:, 0]))
    return n * sgn[:, None]


def gaussian_normals(G, cam: Cam) -> torch.Tensor:
    """n_i of Eq. 11 for 3D Gaussians: the direction of the shortest axis
    (the rotation's column of the smallest scale), world space, facing the
    camera.  [M, 3]."""
    Rq = quat_to_rot(_t(G.quat))                       # [M, 3, 3], columns = axes
    k = torch.argmin(_t(G.scale), dim=0)               # smallest scale
    n = torch.gather(Rq, 2, k[:, None, None].expand(-1, 3, 1))[:, :, 0]
    return facing(n, cam.o[None, :] - _t(G.mean).T)


def geometry(scene, cam_idx=0, pix=None, opts: Optional[Options] = None, chunk_elems=4_000_000):
    """Geometry channels of the pixels `pix` (default: whole image):

    N_s [3,P]      the frontmost surfel's unit normal (world space, facing the
                   camera; 0 where no surfel covers the pixel);
    D_G [P]        Eq. 10: sum over the Gaussians that count at the pixel
                   (the pass-2 depth test and alpha threshold) of d_i alpha_i,
                   d_i the centre depth (camera z);
    N_G [3,P]      Eq. 11: the same sum of n_i alpha_i, n_i the shortest
                   axis (`gaussian_normals`);
    D_smooth [P]   Eq. 12: (D_s W_s + D_G) / (W_s + W_G), with D_s W_s read
                   as 0 where no surfel covers the pixel;
    N_smooth [3,P] Eq. 12: (N_s W_s + N_G) / (W_s + W_G).
    Plus the render's bookkeeping (id, depth, margins) for comparisons."""
    opts = opts or Options()
    cam = Cam(scene.cameras[cam_idx])
    if pix is None:
        pix = torch.arange(cam.W * cam.H)
    pix = torch.as_tensor(pix, dtype=torch.long)
    S, G = scene.surfels, scene.gaussians
    with torch.no_grad():
        out = render(scene, cam_idx, pix, opts, chunk_elems)
        ids = out["id"]
        if S.n:
            ns = facing(surfel_frames(S, cam)["n"] @ cam.R, cam.o[None, :] - _t(S.mean).T)  # world normals
            Ns = torch.where(ids[None, :] >= 0, ns[ids.clamp_min(0)].T, torch.zeros(3, ids.shape[0], dtype=DT))
            Ds = torch.where(ids >= 0, out["depth"], torch.zeros_like(out["depth"]))
        else:
            Ns = torch.zeros(3, ids.shape[0], dtype=DT)
            Ds = torch.zeros(ids.shape[0], dtype=DT)
        DG = torch.zeros(ids.shape[0], dtype=DT)
        NG = torch.zeros(3, ids.shape[0], dtype=DT)
        if G.m:
            proj = gaussian_projection(G, cam, opts)
            ng = gaussian_normals(G, cam)
            step = max(1, chunk_elems // G.m)
            for s0 in range(0, pix.shape[0], step):
                p = pix[s0:s0 + step]
                w = gaussian_pass(proj, cam, p, out["depth"][s0:s0 + step], opts)["w"]   # [P, M]
                DG[s0:s0 + step] = w @ proj["depth"]
                NG[:, s0:s0 + step] = (w @ ng).T
        den = opts.w_s + out["wg"]
        out.update(normal_s=Ns, depth_g=DG, normal_g=NG, depth_smooth=(Ds * opts.w_s + DG) / den,
                   normal_smooth=(Ns * opts.w_s + NG) / den)
    return out


# ----------------------------------------------------------------------------
# candidates (exact-safe filters that only skip work)


def gaussian_candidates(G, cam_obj, rect, opts: Optional[Options] = None):
    """Indices of Gaussians that can reach alpha >= alpha_min at some pixel
    centre of rect = (x0, y0, x1, y1) (pixel indices, inclusive-exclusive).

    alpha >= alpha_min needs q <= 2 ln(sigma/alpha_min); on that ellipse
    |dx| <= sqrt(k Sigma_xx), |dy| <= sqrt(k Sigma_yy).  A small relative pad
    keeps the filter conservative under rounding."""
    opts = opts or Options()
    cam = Cam(cam_obj)
    with torch.no_grad():
        proj = gaussian_projection(G, cam, opts)
        k = 2 * torch.log(torch.clamp_min(proj["opacity"] / opts.alpha_min, 1e-300))
        ok = proj["valid"] & (k >= 0)
        ex = torch.sqrt(torch.clamp_min(k, 0) * proj["cov2"][:, 0, 0]) * 1.001 + 1e-6
        ey = torch.sqrt(torch.clamp_min(k, 0) * proj["cov2"][:, 1, 1]) * 1.001 + 1e-6
        x0, y0, x1, y1 = rect
        px, py = proj["phat"][:, 0], proj["phat"][:, 1]
        ok &= (px + ex >= x0 + 0.5) & (px - ex <= x1 - 0.5)
        ok &= (py + ey >= y0 + 0.5) & (py - ey <= y1 - 0.5)
    return torch.nonzero(ok).flatten().numpy()


def surfel_candidates(S, cam_obj, rect, opts: Optional[Options] = None):
    """Indices of surfels whose disc can cover a pixel centre of rect.

    The disc lies inside the sphere of radius R_s max(s_u, s_v) around its
    centre, hence inside that sphere's camera-space bounding box; when the box
    is in front of the near plane its image is inside the bounding rectangle
    of its 8 projected corners.  Boxes reaching the near plane are kept."""
    opts = opts or Options()
    cam = Cam(cam_obj)
    with torch.no_grad():
        mu = (cam.R @ _t(S.mean)).T + cam.t
        rad = opts.surfel_radius * _t(S.scale).max(0).values * 1.001
        lo = mu - rad[:, None]
        hi = mu + rad[:, None]
        keep_near = lo[:, 2] <= cam.znear
        zs = torch.stack([lo[:, 2], hi[:, 2]], -1).clamp_min(1e-300)
        xs = torch.stack([lo[:, 0], hi[:, 0]], -1)
        ys = torch.stack([lo[:, 1], hi[:, 1]], -1)
        u = cam.fx * xs[:, :, None] / zs[:, None, :] + cam.cx
        v = cam.fy * ys[:, :, None] / zs[:, None, :] + cam.cy
        umin, umax = u.flatten(1).min(1).values, u.flatten(1).max(1).values
        vmin, vmax = v.flatten(1).min(1).values, v.flatten(1).max(1).values
        x0, y0, x1, y1 = rect
        inside = (umax >= x0 + 0.5 - 1e-6) & (umin <= x1 - 0.5 + 1e-6) & \
                 (vmax >= y0 + 0.5 - 1e-6) & (vmin <= y1 - 0.5 + 1e-6)
        ok = keep_near | ((hi[:, 2] > 0) & inside)
    return torch.nonzero(ok).flatten().numpy()


def rect_pixels(cam_obj, rect):
    x0, y0, x1, y1 = rect
    ys, xs = torch.meshgrid(torch.arange(y0, y1), torch.arange(x0, x1), indexing="ij")
    return (ys * int(cam_obj.width) + xs).flatten()


# ----------------------------------------------------------------------------
# gradients


GAUSS_KEYS = ("mean", "quat", "scale", "opacity", "sh")


def gradients(scene, dL_dC: np.ndarray, pix, cam_idx=0, opts: Optional[Options] = None,
              chunk_elems=2_000_000):
    """d(sum dL_dC * C)/d(parameters) by autograd of the FP64 definition.

    dL_dC: [3, P] upstream gradient at the pixels `pix`.  Returns float64
    numpy arrays shaped like the parameter arrays: Gaussian mean, quat,
    scale, opacity, sh and surfel sh.  The surfel geometry is fixed (the joint
    optimisation stage of Sec. 4.2 trains Gaussians and surfel SH only)."""
    opts = opts or Options()
    G, S = scene.gaussians, scene.surfels
    leaves = dict(mean=_t(G.mean, True), quat=_t(G.quat, True), scale=_t(G.scale, True),
                  opacity=_t(G.opacity, True), sh=_t(G.sh, True))
    ssh = _t(S.sh, True)
    pix = torch.as_tensor(pix, dtype=torch.long)
    g = _t(dL_dC).reshape(3, -1)
    width = max(S.n, G.m, 1)
    step = max(1, chunk_elems // width)
    for s0 in range(0, pix.shape[0], step):
        out = render(scene, cam_idx, pix[s0:s0 + step], opts, gauss=leaves, surfel_sh=ssh)
        loss = (out["image"] * g[:, s0:s0 + step]).sum()
        if loss.requires_grad:
            loss.backward()
    res = {k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape)) for k, v in leaves.items()}
    res["surfel_sh"] = ssh.grad.numpy() if ssh.grad is not None else np.zeros(ssh.shape)
    return res


def finite_difference(scene, dL_dC: np.ndarray, pix, which, cam_idx=0,
                      opts: Optional[Options] = None, rel_h=1e-6):
    """Central differences of sum dL_dC * C for the parameters listed in
    `which`: tuples (group, flat index into that array), group one of
    'mean','quat','scale','opacity','sh' (Gaussians) or 'surfel_sh'.

    Each is taken at h and h/4; a parameter whose two estimates disagree
    (the step straddled a discontinuity: alpha threshold, depth test) is
    reported as NaN.  Returns a float64 array."""
    import copy
    opts = opts or Options()
    pix = torch.as_tensor(pix, dtype=torch.long)
    g = _t(dL_dC).reshape(3, -1)
    base = dict(mean=scene.gaussians.mean, quat=scene.gaussians.quat,
                scale=scene.gaussians.scale, opacity=scene.gaussians.opacity,
                sh=scene.gaussians.sh, surfel_sh=scene.surfels.sh)
    base64 = {k: np.asarray(v, dtype=np.float64) for k, v in base.items()}

    def loss_at(group, flat, delta):
        arrs = {k: v.copy() for k, v in base64.items()}
        arrs[group].reshape(-1)[flat] += delta
        sc = copy.copy(scene)
        sc.gaussians = copy.copy(scene.gaussians)
        sc.surfels = copy.copy(scene.surfels)
        for k in GAUSS_KEYS:
            setattr(sc.gaussians, k, arrs[k])
        sc.surfels.sh = arrs["surfel_sh"]
        with torch.no_grad():
            out = render(sc, cam_idx, pix, opts)
        return float((out["image"] * g).sum())

    res = np.empty(len(which))
    for i, (group, flat) in enumerate(which):
        x = base64[group].reshape(-1)[flat]
        h = rel_h * max(1.0, abs(x))
        f1 = (loss_at(group, flat, h) - loss_at(group, flat, -h)) / (2 * h)
        f2 = (loss_at(group, flat, h / 4) - loss_at(group, flat, -h / 4)) / (h / 2)
        scale = max(abs(f1), abs(f2), 1e-12)
        res[i] = f1 if abs(f1 - f2) <= 1e-4 * scale + 1e-9 else np.nan
    return res
