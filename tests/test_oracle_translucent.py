"""Pins of the translucent-surfel oracle (Sec. 4.1, Eq. 6-7: opacity
alpha = min(1, w G) with G = exp(-(x^2 + y^2)/2) on the surfel's local
plane, zero where min(alpha, G) < 1/255; front-to-back alpha blending in
centre-depth order, optionally with the pixel's nearest surfel first).

* One fronto-parallel disc: at a pixel of local radius rho (from the pixel
  geometry alone) the colour is a c + (1 - a) bg with
  a = min(1, w exp(-rho^2/2)) and the 1/255 rule, for w below 1, between 1
  and 255, and at 255; alpha and depth likewise.
* Two fronto-parallel discs: the textbook two-layer blend, nearer centre
  first.
* Order adjustment: two tilted discs whose centre-depth order and whose
  depth order at a pixel disagree; without the adjustment the centre-nearer
  one is blended first, with it the pixel-nearer one -- both closed forms.
* w = 255 with the adjustment reproduces the opaque z-buffer render of
  `render.py` (itself pinned) exactly: colour of the nearest hit, background
  where nothing is hit.
* Gradients (mean, quat, scale, w, sh): autograd against FP64 central
  differences.
* Planted mistakes (no clamp at 1, the 1/255 rule on alpha alone, the blend
  in reverse order, the adjustment ignored) are caught.
"""
import importlib
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Scene, Surfels, empty_gaussians, workload

from test_oracle_closed_forms import Y00, _rot, _rotq, _surfels

T = importlib.import_module("oracle.translucent")


def _cam(W=48, H=40, f=50.0, bg=(0.1, 0.2, 0.3)):
    return Camera(W, H, f, f, W / 2, H / 2, np.eye(3), np.zeros(3), 0.2, bg)


def _render(S, cam, w, front_first=False, pix=None):
    return T.translucent_render(Scene(S, empty_gaussians(), [cam]), np.asarray(w, np.float64), 0, pix, front_first)


def _rho(cam, pix, cx, cy, z, s):
    px = (pix % cam.width) + 0.5
    py = (pix // cam.width) + 0.5
    return np.sqrt(((px - cx) * z / (cam.fx * s)) ** 2 + ((py - cy) * z / (cam.fy * s)) ** 2)


@pytest.mark.parametrize("w", [0.6, 7.5, 255.0])
def test_single_disc_closed_form(w):
    cam = _cam()
    z0, s, dc = 2.0, 0.05, 0.7
    S = _surfels([[0.013, -0.02, z0]], [[1, 0, 0, 0]], [[s, s]], dc)
    pix = np.arange(cam.width * cam.height)
    out = _render(S, cam, [w], pix=pix)
    cx, cy = cam.fx * 0.013 / z0 + cam.cx, cam.fy * -0.02 / z0 + cam.cy
    rho = _rho(cam, pix, cx, cy, z0, s)
    G = np.exp(-0.5 * rho ** 2)
    a = np.minimum(1.0, w * G)
    a = np.where(np.minimum(a, G) < 1 / 255, 0.0, a)
    safe = (np.abs(np.log(np.maximum(G, 1e-300) * 255)) > 1e-9) & (np.abs(np.log(np.maximum(w * G, 1e-300) * 255)) > 1e-9)
    c = 0.5 + Y00 * dc
    bg = np.array(cam.bg)[:, None]
    want = a * c + (1 - a) * bg
    assert (a[safe] > 0).sum() > 20 and (a[safe] == 0).sum() > 20
    assert np.allclose(out["color"].numpy()[:, safe], want[:, safe], atol=1e-12)
    assert np.allclose(out["alpha"].numpy()[safe], a[safe], atol=1e-12)
    assert np.allclose(out["depth"].numpy()[safe], (a * z0)[safe], atol=1e-12)
    if w == 255.0:  # opaque on the whole disc
        assert set(np.unique(a[safe])) <= {0.0, 1.0}


def test_two_layers_nearer_centre_first():
    cam = _cam()
    S = _surfels([[0.0, 0.0, 3.0], [0.01, 0.0, 2.0]], [[1, 0, 0, 0]] * 2, [[0.06, 0.06], [0.04, 0.04]], [[0.9, -0.3]] * 3)
    w = np.array([3.0, 0.8])
    pix = np.arange(cam.width * cam.height)
    out = _render(S, cam, w, pix=pix)
    ca, cb = 0.5 + Y00 * 0.9, 0.5 + Y00 * -0.3
    bg = np.array(cam.bg)[:, None]

    def alpha(cx_w, z, s, wi):
        cx, cy = cam.fx * cx_w / z + cam.cx, cam.cy
        G = np.exp(-0.5 * _rho(cam, pix, cx, cy, z, s) ** 2)
        a = np.minimum(1, wi * G)
        return np.where(np.minimum(a, G) < 1 / 255, 0.0, a)
    a_far, a_near = alpha(0.0, 3.0, 0.06, 3.0), alpha(0.01, 2.0, 0.04, 0.8)
    want = a_near * cb + (1 - a_near) * (a_far * ca + (1 - a_far) * bg)
    both = (a_far > 0.05) & (a_near > 0.05)
    assert both.sum() > 10
    assert np.allclose(out["color"].numpy(), want, atol=1e-12)
    assert np.allclose(out["alpha"].numpy(), 1 - (1 - a_near) * (1 - a_far), atol=1e-12)


def _crossing_pair():
    """Two discs tilted about the y axis in opposite senses, centres at
    depths 2.0 and 2.1 (disc 0 nearer by centre); along the +x side of the
    image disc 1 is nearer at the pixel."""
    cam = _cam(W=40, H=8, f=40.0)
    qa, qb = _rotq([0, 1, 0], 0.9), _rotq([0, 1, 0], -0.9)
    S = _surfels([[0.0, 0.0, 2.0], [0.0, 0.0, 2.1]], [qa, qb], [[0.25, 0.25], [0.25, 0.25]], [[0.8, -0.6]] * 3)
    return cam, S


def _plane_hit(cam, pix, centre, q):
    R = _rot(q)
    n = R[:, 2]
    px = (pix % cam.width) + 0.5
    py = (pix // cam.width) + 0.5
    r = np.stack([(px - cam.cx) / cam.fx, (py - cam.cy) / cam.fy, np.ones_like(px)], 1)
    z = (n @ centre) / (r @ n)
    X = z[:, None] * r - centre
    return z, X @ R[:, 0], X @ R[:, 1]


@pytest.mark.parametrize("front_first", [False, True])
def test_order_adjustment_closed_form(front_first):
    cam, S = _crossing_pair()
    w = np.array([2.0, 40.0])
    pix = np.arange(cam.width * cam.height)
    out = _render(S, cam, w, front_first=front_first, pix=pix)
    zs, als = [], []
    for k, q in enumerate((_rotq([0, 1, 0], 0.9), _rotq([0, 1, 0], -0.9))):
        z, u, v = _plane_hit(cam, pix, S.mean[:, k], q)
        G = np.exp(-0.5 * ((u / 0.25) ** 2 + (v / 0.25) ** 2))
        a = np.minimum(1, w[k] * G)
        zs.append(z)
        als.append(np.where(np.minimum(a, G) < 1 / 255, 0.0, a))
    c = [0.5 + Y00 * 0.8, 0.5 + Y00 * -0.6]
    bg = np.array(cam.bg)[:, None]
    both = (als[0] > 0) & (als[1] > 0)
    pix_first1 = both & (zs[1] < zs[0])        # the pixel sees disc 1 nearer
    assert pix_first1.sum() > 3 and (both & (zs[0] < zs[1])).sum() > 3
    first = np.where(pix_first1 & front_first, 1, 0)
    a_f = np.where(first == 1, als[1], als[0])
    a_s = np.where(first == 1, als[0], als[1])
    c_f = np.where(first == 1, c[1], c[0])
    c_s = np.where(first == 1, c[0], c[1])
    want = a_f * c_f + (1 - a_f) * (a_s * c_s + (1 - a_s) * bg)
    assert np.allclose(out["color"].numpy(), want, atol=1e-12)
    if front_first:
        fid = out["front"].numpy()
        assert np.array_equal(fid[pix_first1], np.ones(pix_first1.sum()))


def test_opaque_limit_equals_zbuffer_render():
    sc = workload("tiny", n_surfels=500, n_gaussians=0)
    c = sc.cameras[0]
    cam = Camera(48, 40, c.fx * 48 / 128, c.fy * 48 / 128, 24.0, 20.0, c.R, c.t, c.znear, (0.3, 0.1, 0.2))
    sc = Scene(sc.surfels, empty_gaussians(), [cam])
    opaque = oracle.render(sc)
    out = T.translucent_render(sc, np.full(sc.surfels.n, 255.0), front_first=True)
    # exact where the opaque winner is unique and not on a rim (the two
    # passes compare the same quantities; these margins exclude rounding ties)
    safe = (opaque["ties"].numpy() <= 1) & (opaque["rim"].numpy() > 1e-9)
    assert safe.sum() > 0.9 * safe.size
    assert 0.2 < (opaque["id"].numpy() >= 0).mean() < 0.95
    assert np.allclose(out["color"].numpy()[:, safe], opaque["color_s"].numpy()[:, safe], atol=1e-12)
    hit = opaque["id"].numpy() >= 0
    assert np.array_equal(out["front"].numpy()[safe & hit], opaque["id"].numpy()[safe & hit])
    assert np.allclose(out["alpha"].numpy()[safe], hit[safe].astype(float), atol=0)


def _small_scene(n=60):
    sc = workload("tiny", n_surfels=n, n_gaussians=0)
    c = sc.cameras[0]
    cam = Camera(24, 20, c.fx * 24 / 128, c.fy * 24 / 128, 12.0, 10.0, c.R, c.t, c.znear, (0.3, 0.1, 0.2))
    S = sc.surfels
    S = Surfels(S.mean, S.quat, S.scale * 4.0, S.sh)  # wider discs: more overlap
    return Scene(S, empty_gaussians(), [cam])


@pytest.mark.parametrize("front_first", [False, True])
def test_gradients_match_finite_differences(front_first):
    sc = _small_scene()
    rng = np.random.default_rng(5)
    w = rng.uniform(0.3, 40.0, sc.surfels.n)
    cam = sc.cameras[0]
    pix = np.arange(cam.width * cam.height)
    d = rng.standard_normal((3, pix.size))
    g = T.translucent_gradients(sc, w, d, pix, front_first=front_first)
    which = []
    for grp in ("mean", "quat", "scale", "w", "sh"):
        flat = np.abs(g[grp]).reshape(-1)
        which += [(grp, int(i)) for i in np.argsort(-flat)[:3]]
    fd = T.translucent_fd(sc, w, d, pix, which, front_first=front_first)
    n = 0
    for (grp, i), v in zip(which, fd):
        if np.isnan(v):
            continue
        n += 1
        a = g[grp].reshape(-1)[i]
        assert abs(a - v) <= 1e-5 * max(abs(v), 1e-3), (grp, i, a, v)
    assert n >= 10


def _fails(test, *args):
    try:
        test(*args)
    except AssertionError:
        return True
    return False


def test_mutation_no_clamp_caught(monkeypatch):
    orig = torch.minimum

    def fake_min(a, b):
        if isinstance(b, torch.Tensor) and b.shape == a.shape and bool((b == 1).all()):
            return a
        return orig(a, b)
    monkeypatch.setattr(T.torch, "minimum", fake_min)
    assert _fails(test_single_disc_closed_form, 255.0)


def test_mutation_rule_on_alpha_alone_caught(monkeypatch):
    orig = T.surfel_alphas

    def wrong(f, cam, pix):
        alpha, z, m = orig(f, cam, pix)
        # the 1/255 rule applied to alpha only: far outside the disc a large
        # w keeps w G >= 1/255
        r = cam.rays(pix)
        nr = r @ f["n"].T
        z2 = (f["n"] * f["mu"]).sum(-1) / nr
        u = (z2 * (r @ f["tu"].T) - (f["mu"] * f["tu"]).sum(-1)) / f["scale"][:, 0]
        v = (z2 * (r @ f["tv"].T) - (f["mu"] * f["tv"]).sum(-1)) / f["scale"][:, 1]
        a = torch.minimum(f["w"][None, :] * torch.exp(-0.5 * (u * u + v * v)), torch.ones_like(u))
        return torch.where((a >= T.ALPHA_MIN) & (z2 >= cam.znear), a, torch.zeros_like(a)), z, m
    monkeypatch.setattr(T, "surfel_alphas", wrong)
    assert _fails(test_single_disc_closed_form, 255.0)


def test_mutation_reverse_order_caught(monkeypatch):
    orig = torch.argsort

    def rev(x, *a, **k):
        return orig(-x, *a, **k)
    monkeypatch.setattr(T.torch, "argsort", rev)
    assert _fails(test_two_layers_nearer_centre_first)


def test_mutation_adjustment_ignored_caught(monkeypatch):
    orig = T.translucent_render

    def wrong(scene, w, cam_idx=0, pix=None, front_first=False, leaves=None, chunk_elems=4_000_000):
        out = orig(scene, w, cam_idx, pix, False, leaves, chunk_elems)
        return out
    monkeypatch.setattr(T, "translucent_render", wrong)
    assert _fails(test_order_adjustment_closed_form, True)
    assert _fails(test_opaque_limit_equals_zbuffer_render)
