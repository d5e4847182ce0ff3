"""Helpers shared by the GPU tests: move a synthetic scene to the device,
render it through the C ABI, and compare a rendered view with the FP64
oracle at a set of pixels.

Tolerances (see the design notes for their derivation):
  * surfel ids: exact where the winning depth is unique (no other hit within
    1e-5 relative) and no rim / near-plane decision is within its FP32 error
    band; at tie pixels the GPU id must be one of the oracle's tied
    candidates;
  * depth D_s: 2e-6 relative;
  * C_s: 1e-5 absolute against the oracle colour of the GPU's surfel;
  * C_G, W_G and the image: 1e-4 max abs (image per channel), at pixels
    where no alpha-threshold or depth-test decision lies in its band.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
from paper_2504_17545_amd import Renderer

TOL_IMAGE = 1e-4
TOL_ACCUM = 1e-4
TOL_CS = 1e-5
TOL_DEPTH_REL = 2e-6


def to_dev(scene, device="cuda"):
    s, g = scene.surfels, scene.gaussians
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device)
    # the library takes surfel SH per surfel, [n][K][3]; scenes hold [K][3][n]
    S = dict(mean=f(s.mean), quat=f(s.quat), scale=f(s.scale), sh=f(np.transpose(s.sh, (2, 0, 1))))
    G = dict(mean=f(g.mean), quat=f(g.quat), scale=f(g.scale), opacity=f(g.opacity),
             sh=f(np.transpose(g.sh, (2, 0, 1))))
    return S, G


def render(scene, cams=None, **opts):
    S, G = to_dev(scene)
    r = Renderer(**opts)
    frame = r.render(S, G, cams if cams is not None else scene.cameras)
    torch.cuda.synchronize()
    return frame


def view_np(frame, name, v=0):
    return frame.view(name, v).detach().cpu().numpy()


def compare_view(frame, scene, v=0, pix=None, opts=None, max_amb_frac=0.02):
    """Compare view v of `frame` with the oracle at flat pixel indices `pix`
    (all pixels if None).  Returns a dict of statistics; asserts parity."""
    cam = scene.cameras[v]
    W, H = cam.width, cam.height
    if pix is None:
        pix = np.arange(W * H)
    pix = np.asarray(pix, dtype=np.int64)
    out = oracle.render(scene, v, pix, opts=opts)
    gid = view_np(frame, "surfel_id", v).reshape(-1)[pix].astype(np.int64)
    gdep = view_np(frame, "depth", v).reshape(-1)[pix].astype(np.float64)
    gcs = view_np(frame, "color_s", v).reshape(3, -1)[:, pix].astype(np.float64)
    gimg = view_np(frame, "image", v).reshape(3, -1)[:, pix].astype(np.float64)
    gacc = view_np(frame, "accum", v).reshape(4, -1)[:, pix].astype(np.float64)

    oid = out["id"].numpy()
    ties = out["ties"].numpy()
    cands = out["cands"].numpy()
    amb_s = (out["rim"].numpy() < 1e-4) | (out["near"].numpy() < 1e-5)
    amb_g = (out["alpha_margin"].numpy() < 1e-4) | (out["depth_margin"].numpy() < 1e-5)
    tie = ties > 1
    unique = (~tie) & (~amb_s)

    # surfel ids
    mism = unique & (gid != oid)
    assert not mism.any(), f"id mismatch at {int(mism.sum())} unique pixels, e.g. {pix[mism][:5]}"
    tie_ok = np.array([(gid[k] in cands[k]) for k in np.nonzero(tie & ~amb_s)[0]], dtype=bool)
    assert tie_ok.all(), f"GPU id not among tied candidates at {int((~tie_ok).sum())} pixels"
    # depth
    od = out["depth"].numpy()
    hit = (gid >= 0) & ~amb_s
    assert np.array_equal(np.isinf(gdep[~amb_s]), np.isinf(od[~amb_s]))
    rel = np.abs(gdep[hit] - od[hit]) / od[hit]
    assert rel.size == 0 or rel.max() <= (1e-5 if tie.any() else TOL_DEPTH_REL), rel.max()
    # C_s: the oracle colour of the surfel the GPU chose
    scol = out["surfel_colour"].numpy()
    bg = np.asarray(cam.bg, dtype=np.float64)[:, None]
    ecs = np.where(gid[None, :] >= 0, scol[:, np.clip(gid, 0, None)] if scol.shape[1] else bg, bg)
    ok_s = ~amb_s
    err_cs = np.abs(gcs[:, ok_s] - ecs[:, ok_s]).max(initial=0.0)
    assert err_cs <= TOL_CS, err_cs
    # Gaussian accumulation and composite where no decision is ambiguous
    good = ok_s & ~amb_g
    ocg, owg = out["cg"].numpy(), out["wg"].numpy()
    err_cg = np.abs(gacc[:3, good] - ocg[:, good]).max(initial=0.0)
    err_wg = np.abs(gacc[3, good] - owg[good]).max(initial=0.0)
    w_s = 1.0 if opts is None else opts.w_s
    eimg = (w_s * ecs + ocg) / (w_s + owg)
    err_img = np.abs(gimg[:, good] - eimg[:, good]).max(initial=0.0)
    n_amb = int((~good).sum())
    stats = dict(pixels=len(pix), ambiguous=n_amb, ties=int(tie.sum()), err_cs=err_cs, err_cg=err_cg,
                 err_wg=err_wg, err_img=err_img, hit_frac=float((oid >= 0).mean()),
                 mean_count=float(out["count"].numpy().mean()))
    print(f"[parity] view {v}: {stats}", flush=True)
    assert err_cg <= TOL_ACCUM and err_wg <= TOL_ACCUM, stats
    assert err_img <= TOL_IMAGE, stats
    assert n_amb <= max_amb_frac * len(pix) + 2, stats
    return stats


def sample_pixels(cam, k, seed):
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    pts = rng.integers(0, W * H, size=k)
    # plus the four corners and the last row/column (ragged tile edges)
    extra = [0, W - 1, (H - 1) * W, H * W - 1, (H // 2) * W + W - 1, (H - 1) * W + W // 2]
    return np.unique(np.concatenate([pts, extra]))
