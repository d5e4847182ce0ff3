"""Invariants of the method checked on the oracle (Sec. 3 Eq. 2-5; Sec. 7.2).

I1 no Gaussians: C = C_s.            I2 no surfels: C = (bg + C_G)/(1 + W_G).
I3 a Gaussian hidden behind the surfel depth (d >= D_s + eps) changes nothing.
I4 sorting-free: permuting the Gaussian array leaves the image unchanged.
I5 decomposition C = C_s/(1+W_G) + C_G/(1+W_G) (the split shown in Sec. 7.2).
I6 C is a convex combination of the background/surfel colour and the
   colours of the Gaussians counted at the pixel.
I7 permuting the surfels changes only pixels with a depth tie.
Plus: an independent scalar brute-force renderer (world-space ray casting, one
pixel and one primitive at a time) on a tiny scene, and the exact-safe
candidate filters used to speed up crop evaluations.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import (Scene, empty_gaussians, empty_surfels, workload, permute_gaussians,
                   permute_surfels, subset)


@pytest.fixture(scope="module")
def tiny():
    return workload("tiny")


@pytest.fixture(scope="module")
def tiny_out(tiny):
    return oracle.render(tiny)


def test_I1_no_gaussians(tiny):
    sc = Scene(tiny.surfels, empty_gaussians(), tiny.cameras)
    out = oracle.render(sc)
    assert torch.equal(out["image"], out["color_s"])


def test_I2_no_surfels(tiny):
    sc = Scene(empty_surfels(), tiny.gaussians, tiny.cameras)
    out = oracle.render(sc)
    bg = torch.tensor(tiny.cameras[0].bg, dtype=torch.float64)[:, None]
    assert torch.all(out["id"] == -1)
    assert torch.allclose(out["image"], (bg + out["cg"]) / (1 + out["wg"]), atol=1e-15)
    assert out["wg"].max() > 0.5


def test_I3_hidden_gaussian(tiny, tiny_out):
    # put a big opaque Gaussian far behind everything; all pixels in its
    # support have surfel depth < 3 or no surfel -> pick only covered ones
    cam = tiny.cameras[0]
    G = tiny.gaussians
    extra = dict(mean=np.array([[0.0], [0.0], [10.0]]), quat=np.array([[1.0], [0], [0], [0]]),
                 scale=np.array([[0.3], [0.3], [0.3]]), opacity=np.array([0.9]),
                 sh=np.ones((16, 3, 1)))
    from synth import Gaussians
    G2 = Gaussians(np.concatenate([G.mean, extra["mean"]], 1), np.concatenate([G.quat, extra["quat"]], 1),
                   np.concatenate([G.scale, extra["scale"]], 1),
                   np.concatenate([G.opacity, extra["opacity"]]), np.concatenate([G.sh, extra["sh"]], 2))
    out = oracle.render(Scene(tiny.surfels, G2, tiny.cameras))
    covered = tiny_out["id"] >= 0
    assert torch.equal(out["image"][:, covered], tiny_out["image"][:, covered])
    assert not torch.equal(out["image"][:, ~covered], tiny_out["image"][:, ~covered])


def test_I4_permutation_invariance(tiny, tiny_out):
    G2, _ = permute_gaussians(tiny.gaussians, 99)
    out = oracle.render(Scene(tiny.surfels, G2, tiny.cameras))
    assert torch.allclose(out["image"], tiny_out["image"], atol=1e-12, rtol=0)
    assert torch.equal(out["id"], tiny_out["id"])


def test_I5_decomposition(tiny_out):
    o = tiny_out
    lhs = o["color_s"] / (1 + o["wg"]) + o["cg"] / (1 + o["wg"])
    assert torch.allclose(o["image"], lhs, atol=1e-14)


def test_I6_convex_combination(tiny):
    # clamp colours into [0,1] via DC-only SH so that the bound is simple
    sc = workload("tiny")
    sc.gaussians.sh = sc.gaussians.sh.copy()
    sc.gaussians.sh[1:] = 0
    sc.gaussians.sh[0] = np.clip(sc.gaussians.sh[0], -1.7, 1.7)
    sc.surfels.sh = sc.surfels.sh.copy()
    sc.surfels.sh[1:] = 0
    sc.surfels.sh[0] = np.clip(sc.surfels.sh[0], -1.7, 1.7)
    out = oracle.render(sc)
    proj = oracle.gaussian_projection(sc.gaussians, oracle.Cam(sc.cameras[0]), oracle.Options())
    cmax = proj["colour"].max(1).values
    cmin = proj["colour"].min(1).values
    lo = torch.minimum(out["color_s"], cmin[:, None])
    hi = torch.maximum(out["color_s"], cmax[:, None])
    assert torch.all(out["image"] >= lo - 1e-12) and torch.all(out["image"] <= hi + 1e-12)


def test_I7_surfel_permutation(tiny, tiny_out):
    S2, perm = permute_surfels(tiny.surfels, 5)
    out = oracle.render(Scene(S2, tiny.gaussians, tiny.cameras))
    ids = out["id"].clone()
    ids[ids >= 0] = torch.as_tensor(perm)[ids[ids >= 0]]
    unique = tiny_out["ties"] <= 1
    assert torch.equal(ids[unique], tiny_out["id"][unique])
    assert torch.allclose(out["image"][:, unique], tiny_out["image"][:, unique], atol=1e-12)


# ----------------------------------------------------------------------------
# independent scalar brute force


def _qrot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _sh_dc_l1(sh, d):
    # DC and degree 1 only (the tiny scene zeroes higher bands)
    c1 = math.sqrt(3 / (4 * math.pi))
    x, y, z = d
    return 0.5 / math.sqrt(math.pi) * sh[0] - c1 * y * sh[1] + c1 * z * sh[2] - c1 * x * sh[3]


def _scalar_render(sc):
    """World-space ray casting, one pixel and one primitive at a time."""
    cam = sc.cameras[0]
    R, t = np.asarray(cam.R, float), np.asarray(cam.t, float)
    o = -R.T @ t
    S, G = sc.surfels, sc.gaussians
    Rs = oracle.SURFEL_RADIUS
    img = np.zeros((3, cam.height, cam.width))
    for j in range(cam.height):
        for i in range(cam.width):
            dcam = np.array([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, 1.0])
            dw = R.T @ dcam                     # world ray direction, camera-z = 1
            best, bid = math.inf, -1
            for k in range(S.n):
                Rk = _qrot(S.quat[:, k].astype(float))
                p = S.mean[:, k].astype(float)
                nrm = Rk[:, 2]
                den = nrm @ dw
                if abs(den) <= 1e-12 * np.linalg.norm(dcam):
                    continue
                lam = nrm @ (p - o) / den       # world point o + lam dw has camera z = lam
                if lam < cam.znear:
                    continue
                X = o + lam * dw
                u = (X - p) @ Rk[:, 0] / S.scale[0, k]
                v = (X - p) @ Rk[:, 1] / S.scale[1, k]
                if u * u + v * v <= Rs * Rs and lam < best:
                    best, bid = lam, k
            if bid >= 0:
                p = S.mean[:, bid].astype(float)
                dd = (o - p) / np.linalg.norm(o - p)
                cs = np.array([max(0.0, 0.5 + _sh_dc_l1(S.sh[:4, ch, bid], dd)) for ch in range(3)])
            else:
                cs = np.array(cam.bg, float)
            cg = np.zeros(3)
            wg = 0.0
            for k in range(G.m):
                p = G.mean[:, k].astype(float)
                mc = R @ p + t
                if mc[2] <= cam.znear:
                    continue
                Rk = _qrot(G.quat[:, k].astype(float))
                M = Rk @ np.diag(G.scale[:, k].astype(float))
                V = R @ (M @ M.T) @ R.T
                zc = mc[2]
                tx = min(max(mc[0] / zc, -1.3 * cam.width / (2 * cam.fx)), 1.3 * cam.width / (2 * cam.fx)) * zc
                ty = min(max(mc[1] / zc, -1.3 * cam.height / (2 * cam.fy)), 1.3 * cam.height / (2 * cam.fy)) * zc
                J = np.array([[cam.fx / zc, 0, -cam.fx * tx / zc ** 2], [0, cam.fy / zc, -cam.fy * ty / zc ** 2]])
                cov = J @ V @ J.T + 0.3 * np.eye(2)
                ph = np.array([cam.fx * mc[0] / zc + cam.cx, cam.fy * mc[1] / zc + cam.cy])
                dlt = np.array([i + 0.5, j + 0.5]) - ph
                a = G.opacity[k] * math.exp(-0.5 * dlt @ np.linalg.solve(cov, dlt))
                eps = 5.0 / 3.0 * G.scale[:, k].astype(float).sum()
                if a >= 1 / 255 and zc < best + eps:
                    dd = (o - p) / np.linalg.norm(o - p)
                    c = np.array([max(0.0, 0.5 + _sh_dc_l1(G.sh[:4, ch, k], dd)) for ch in range(3)])
                    cg += a * c
                    wg += a
            img[:, j, i] = (cs + cg) / (1 + wg)
    return img.reshape(3, -1)


def test_scalar_bruteforce_tiny():
    sc = workload("tiny", seed=7, n_surfels=12, n_gaussians=10)
    cam = sc.cameras[0]
    from synth import Camera
    sc.cameras = [Camera(24, 20, 14.0, 15.0, 12.2, 9.7, cam.R, cam.t, 0.2, (0.05, 0.1, 0.15))]
    # larger primitives so they cover pixels of the tiny image; bands >= 2 zeroed
    sc.surfels.scale = sc.surfels.scale * 6
    sc.gaussians.scale = sc.gaussians.scale * 8
    sc.surfels.sh = sc.surfels.sh.copy(); sc.surfels.sh[4:] = 0
    sc.gaussians.sh = sc.gaussians.sh.copy(); sc.gaussians.sh[4:] = 0
    ref = _scalar_render(sc)
    out = oracle.render(sc)
    assert (out["id"] >= 0).sum() > 20 and float(out["wg"].max()) > 0.05
    assert np.allclose(out["image"].numpy(), ref, atol=1e-12)


def test_candidate_filters_exact(tiny, tiny_out):
    cam = tiny.cameras[0]
    rect = (40, 50, 72, 80)
    gi = oracle.gaussian_candidates(tiny.gaussians, cam, rect)
    si = oracle.surfel_candidates(tiny.surfels, cam, rect)
    assert 0 < len(gi) < tiny.gaussians.m and 0 < len(si) < tiny.surfels.n
    pix = oracle.rect_pixels(cam, rect)
    sub = subset(tiny, si, gi)
    out = oracle.render(sub, pix=pix)
    ids = out["id"].clone()
    ids[ids >= 0] = torch.as_tensor(si)[ids[ids >= 0]]
    assert torch.equal(ids, tiny_out["id"][pix])
    assert torch.allclose(out["image"], tiny_out["image"][:, pix], atol=1e-14)
