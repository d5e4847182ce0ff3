"""Pins of the 2D-GES oracle (Sec. 6.4: 2D Gaussians in pass 2, with the
planar depth and the splat normal in the depth test and the geometry
channels; eps = (5/D) sum s with D = 2, Sec. 5).

* A lone fronto-parallel anisotropic splat: alpha at every pixel from the
  pixel geometry alone (sigma exp(-(u^2+v^2)/2) with u, v the pixel's
  offset scaled by z / (f s)), the 1/255 rule, the composite, D_G = alpha z,
  N_G = alpha times the normal facing the camera.
* A tilted splat: its depth at each pixel is the ray-plane intersection
  written out from the tilt angle, far from the centre depth at the edges.
* The depth test takes the planar depth: a tilted splat whose centre lies
  behind the surfel counts exactly where its plane is in front of D_s + eps.
* eps = 2.5 (s_u + s_v): splats 0.9 eps and 1.1 eps behind a surfel.
* Near plane and edge-on splats do not count.
* Invariants: permuting the splats, a scene without them, hidden splats.
* Planted mistakes (centre depth in the test, D = 3 in eps, no facing flip,
  the scales swapped) are caught.
"""
import importlib
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Gaussians, Scene, Surfels, empty_gaussians

from test_oracle_closed_forms import Y00, _rot, _rotq, _surfels

GS = importlib.import_module("oracle.gs2d")


def _cam(W=48, H=40, f=50.0, bg=(0.1, 0.2, 0.3)):
    return Camera(W, H, f, f * 1.05, W / 2 + 0.25, H / 2 - 0.15, np.eye(3), np.zeros(3), 0.2, bg)


def _splats(mean, quat, scale, opac, dc):
    m = len(mean)
    sh = np.zeros((16, 3, m))
    sh[0] = np.asarray(dc, dtype=np.float64).reshape(3, m) if np.ndim(dc) else dc
    return Gaussians(np.asarray(mean, np.float64).T.copy(), np.asarray(quat, np.float64).T.copy(),
                     np.asarray(scale, np.float64).T.copy(), np.asarray(opac, np.float64), sh)


def _no_surfels():
    return Surfels(np.zeros((3, 0)), np.zeros((4, 0)), np.zeros((2, 0)), np.zeros((16, 3, 0)))


def _ray(cam, pix):
    px = (pix % cam.width) + 0.5
    py = (pix // cam.width) + 0.5
    return np.stack([(px - cam.cx) / cam.fx, (py - cam.cy) / cam.fy, np.ones_like(px, dtype=float)], 1)


def test_lone_fronto_parallel_closed_form():
    cam = _cam()
    z0, su, sv, sig, dc = 2.0, 0.06, 0.025, 0.8, 0.6
    x0, y0 = 0.03, -0.02
    G = _splats([[x0, y0, z0]], [[1, 0, 0, 0]], [[su, sv]], [sig], dc)
    out = GS.render_2dges(Scene(_no_surfels(), G, [cam]))
    pix = np.arange(cam.width * cam.height)
    r = _ray(cam, pix)
    u = (z0 * r[:, 0] - x0) / su
    v = (z0 * r[:, 1] - y0) / sv
    a = sig * np.exp(-0.5 * (u * u + v * v))
    safe = np.abs(np.log(a * 255)) > 1e-9
    a = np.where(a >= 1 / 255, a, 0.0)
    assert (a[safe] > 0).sum() > 30 and (a[safe] == 0).sum() > 30
    c = 0.5 + Y00 * dc
    bg = np.array(cam.bg)[:, None]
    assert np.allclose(out["wg"].numpy()[safe], a[safe], atol=1e-12)
    assert np.allclose(out["image"].numpy()[:, safe], ((bg + a * c) / (1 + a))[:, safe], atol=1e-12)
    assert np.allclose(out["depth_g"].numpy()[safe], (a * z0)[safe], atol=1e-12)
    # the normal (0, 0, 1) turned to face the camera at the origin: (0, 0, -1)
    ng = out["normal_g"].numpy()
    assert np.allclose(ng[:2], 0.0, atol=1e-12) and np.allclose(ng[2][safe], -a[safe], atol=1e-12)
    # no surfels: D_smooth = D_G / (1 + W_G)
    assert np.allclose(out["depth_smooth"].numpy()[safe], (a * z0 / (1 + a))[safe], atol=1e-12)


def _tilted(theta, centre, s=(0.08, 0.08), sig=0.9):
    return _splats([centre], [_rotq([0, 1, 0], theta)], [s], [sig], 0.4)


def test_tilted_splat_planar_depth():
    cam = _cam(W=64, H=32)
    th = 0.9
    c = np.array([0.0, 0.01, 2.0])
    G = _tilted(th, c, s=(0.25, 0.06))
    out = GS.render_2dges(Scene(_no_surfels(), G, [cam]))
    pix = np.arange(cam.width * cam.height)
    r = _ray(cam, pix)
    n = np.array([math.sin(th), 0.0, math.cos(th)])    # third column of the rotation about y
    z = (n @ c) / (r @ n)
    wg = out["wg"].numpy()
    hit = wg > 0
    assert hit.sum() > 40
    assert np.allclose(out["depth_g"].numpy()[hit] / wg[hit], z[hit], rtol=1e-12)
    assert (np.abs(z[hit] - c[2]) > 0.1).any()         # far from the centre depth


def _wall(depth, half=3.0):
    """A fronto-parallel surfel covering the whole view at `depth`."""
    return _surfels([[0.0, 0.0, depth]], [[1, 0, 0, 0]], [[half, half]], 0.1)


def test_depth_test_takes_planar_depth():
    cam = _cam(W=64, H=32)
    th, D = 0.9, 2.0
    s = (0.3, 0.02)
    eps = 2.5 * sum(s)
    c = np.array([0.0, 0.0, D + 1.2 * eps])             # centre behind D_s + eps
    G = _tilted(th, c, s=s)
    out = GS.render_2dges(Scene(_wall(D), G, [cam]))
    pix = np.arange(cam.width * cam.height)
    r = _ray(cam, pix)
    n = np.array([math.sin(th), 0.0, math.cos(th)])
    z = (n @ c) / (r @ n)
    A = np.array(_rot(_rotq([0, 1, 0], th)))
    X = z[:, None] * r - c
    u, v = X @ A[:, 0] / s[0], X @ A[:, 1] / s[1]
    a = 0.9 * np.exp(-0.5 * (u * u + v * v))
    live = a >= 1 / 255
    margin = np.abs(z - (D + eps)) > 1e-9
    want = live & (z < D + eps)
    got = out["count"].numpy() > 0
    assert want[margin].sum() > 10 and (live & ~want)[margin].sum() > 10
    assert np.array_equal(got[margin], want[margin])


@pytest.mark.parametrize("eps_const", [-1.0, 0.05])
def test_eps_two_dimensional(eps_const):
    cam = _cam()
    D = 1.5
    s = (0.04, 0.02)
    eps = 2.5 * sum(s) if eps_const < 0 else eps_const
    G = _splats([[0.0, 0.0, D + 0.9 * eps], [0.0, 0.0, D + 1.1 * eps]], [[1, 0, 0, 0]] * 2, [s, s], [0.7, 0.7],
                [[0.9, 0.2]] * 3)
    opts = oracle.Options(eps_const=eps_const)
    out = GS.render_2dges(Scene(_wall(D), G, [cam]), opts=opts)
    fr = GS.gauss2d_frames(G, oracle.Cam(cam))
    gp = GS.gauss2d_pass(fr, GS.eps_2d(G, opts), oracle.Cam(cam), torch.arange(cam.width * cam.height),
                         out["depth"], opts)
    w = gp["w"].numpy()
    assert (w[:, 0] > 0).sum() > 10 and (w[:, 1] == 0).all()


def test_near_plane_and_edge_on():
    cam = _cam(W=40, H=40)
    # a plane through the camera centre (n . mu = 0) shows no hit in front
    G = _splats([[0.0, 0.0, 1.0]], [_rotq([0, 1, 0], math.pi / 2)], [(0.3, 0.3)], [0.9], 0.3)
    out = GS.render_2dges(Scene(_no_surfels(), G, [cam]))
    assert (out["wg"].numpy() == 0).all()
    # a splat crossing the near plane: hits nearer than znear do not count
    th = 1.2
    c = np.array([0.0, 0.0, 0.25])
    G = _tilted(th, c, s=(0.3, 0.3))
    out = GS.render_2dges(Scene(_no_surfels(), G, [cam]))
    pix = np.arange(cam.width * cam.height)
    r = _ray(cam, pix)
    n = np.array([math.sin(th), 0.0, math.cos(th)])
    z = (n @ c) / (r @ n)
    cnt = out["count"].numpy()
    assert (cnt[(z > 0) & (z < 0.2 * (1 - 1e-6))] == 0).all()
    assert (cnt[(z > 0.2 * (1 + 1e-6))] > 0).any() and ((z > 0) & (z < 0.2)).sum() > 5


def _random_scene(seed=0, m=60):
    rng = np.random.default_rng(seed)
    cam = _cam(W=40, H=32)
    S = _surfels(rng.uniform([-0.4, -0.3, 1.8], [0.4, 0.3, 2.6], (25, 3)), rng.normal(size=(25, 4)),
                 rng.uniform(0.03, 0.12, (25, 2)), rng.normal(0.3, 0.2, (3, 25)))
    G = _splats(rng.uniform([-0.5, -0.4, 1.5], [0.5, 0.4, 2.5], (m, 3)), rng.normal(size=(m, 4)),
                rng.uniform(0.02, 0.1, (m, 2)), rng.uniform(0.1, 0.95, m), rng.normal(0.2, 0.3, (3, m)))
    return Scene(S, G, [cam])


def test_invariants():
    sc = _random_scene()
    out = GS.render_2dges(sc)
    # permuting the splats
    p = np.random.default_rng(1).permutation(sc.gaussians.m)
    G = sc.gaussians
    Gp = Gaussians(G.mean[:, p], G.quat[:, p], G.scale[:, p], G.opacity[p], G.sh[..., p])
    outp = GS.render_2dges(Scene(sc.surfels, Gp, sc.cameras))
    for k in ("image", "wg", "depth_g", "normal_g"):
        assert np.allclose(out[k].numpy(), outp[k].numpy(), atol=1e-12), k
    assert (out["count"].numpy() > 0).mean() > 0.2
    # without splats the image is C_s; splats all behind a near wall add nothing
    none = GS.render_2dges(Scene(sc.surfels, empty_gaussians(), sc.cameras))
    assert np.allclose(none["image"].numpy(), none["color_s"].numpy(), atol=1e-15)
    hid = GS.render_2dges(Scene(_wall(0.5), G, sc.cameras))
    assert (hid["wg"].numpy() == 0).all()
    # the surfel pass is the plain render's
    ref = oracle.render(Scene(sc.surfels, empty_gaussians(), sc.cameras))
    assert np.array_equal(out["id"].numpy(), ref["id"].numpy())


# ----------------------------------------------------------------------------
# planted mistakes


def _fails(test, *args):
    try:
        test(*args)
    except AssertionError:
        return True
    return False


def test_mutation_centre_depth_caught(monkeypatch):
    # the 3D-Gaussian test: the centre depth against D_s + eps
    monkeypatch.setattr(GS, "depth_test", lambda z, fr, ds, eps: (fr["mu"][:, 2][None, :] < ds[:, None] + eps[None, :])
                        .expand_as(z))
    assert _fails(test_depth_test_takes_planar_depth)


def test_mutation_eps_three_dimensional_caught(monkeypatch):
    orig = GS.eps_2d

    def wrong(G, opts):
        e = orig(G, opts)
        return e * 2.0 / 3.0 if opts.eps_const < 0 else e
    monkeypatch.setattr(GS, "eps_2d", wrong)
    assert _fails(test_eps_two_dimensional, -1.0)


def test_mutation_no_facing_flip_caught(monkeypatch):
    monkeypatch.setattr(GS, "facing", lambda n, to_cam: n)
    assert _fails(test_lone_fronto_parallel_closed_form)


def test_mutation_scales_swapped_caught(monkeypatch):
    orig = GS.gauss2d_frames

    def wrong(G, cam):
        fr = orig(G, cam)
        fr["scale"] = fr["scale"].flip(1)
        return fr
    monkeypatch.setattr(GS, "gauss2d_frames", wrong)
    assert _fails(test_lone_fronto_parallel_closed_form)
