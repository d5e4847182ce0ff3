"""Pins of the oracle's Mip-GES filters (Sec. 6.1: the world-space filter
and the screen-space filter of Mip-Splatting applied to the 3D Gaussians).

* Screen-space filter, isotropic Gaussian on the optical axis: with
  a = (f/z)^2 (s^2 + v) the projected variance, the filtered footprint is
  alpha(rho) = sigma' exp(-rho^2 / (2 (a + e))) with sigma' = sigma a/(a+e)
  (the square root of the determinant ratio of two isotropic 2x2
  covariances), read off W_G at pixels at known distances.
* Off axis and anisotropic: the projected covariance is built from an FD
  Jacobian of the world-to-pixel map (as in the projection pins) and the
  opacity factor from numpy determinants of it, the world covariance from
  Hamilton products; the oracle's conic and opacity must match.
* World-space filter: sigma is scaled by sqrt(det Sigma3 / det(Sigma3 + v I))
  = prod s / sqrt(prod (s^2 + v)), checked with numpy eigenvalues of the
  rotated covariance.
* Filter size from cameras: 0.2 (z / f_x)^2 of the nearest camera whose image
  holds the projected centre; cameras that do not see the Gaussian are
  ignored; a Gaussian no camera sees gets 0.
* Gradients with both filters on: autograd against FP64 central
  differences.
* Planted mistakes (the determinant ratio without its square root, no
  compensation, the screen filter added on top of the dilation) are caught.
"""
import importlib
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Gaussians, Scene, empty_surfels

from test_oracle_closed_forms import _gaussians
from test_oracle_projection import _camera, _jac_fd, _sigma3

R = importlib.import_module("oracle.render")


def _axis_cam():
    return Camera(41, 41, 50.0, 50.0, 20.5, 20.5, np.eye(3), np.zeros(3), 0.2, (0.0, 0.0, 0.0))


def test_screen_filter_isotropic_closed_form():
    cam = _axis_cam()
    z, s, sig, e, v = 2.0, 0.03, 0.8, 0.1, 0.0
    G = _gaussians([[0.0, 0.0, z]], [[1, 0, 0, 0]], [[s, s, s]], [sig], 0.3)
    opts = oracle.Options(mip_2d=e)
    centre = 20 * cam.width + 20
    pix = np.array([centre, centre + 1, centre + 2, centre + cam.width + 1])
    rho2 = np.array([0.0, 1.0, 4.0, 2.0])
    out = oracle.render(Scene(empty_surfels(), G, [cam]), 0, pix, opts=opts)
    a = (cam.fx / z) ** 2 * (s * s + v)
    want = sig * a / (a + e) * np.exp(-rho2 / (2 * (a + e)))
    assert np.allclose(out["wg"].numpy(), want, rtol=1e-12, atol=0)


def test_world_filter_compensation_by_eigenvalues():
    rng = np.random.default_rng(3)
    q = rng.standard_normal(4)
    s = np.array([0.04, 0.011, 0.02])
    v = 3e-4
    S3 = _sigma3(q, s)
    ev0 = np.linalg.eigvalsh(S3)
    ev1 = np.linalg.eigvalsh(S3 + v * np.eye(3))
    want = 0.7 * math.sqrt(np.prod(ev0) / np.prod(ev1))
    G = Gaussians(np.array([[0.1], [-0.05], [2.5]]), q[:, None] / np.linalg.norm(q), s[:, None],
                  np.array([0.7]), np.zeros((16, 3, 1)), filter3d=np.array([v]))
    proj = oracle.gaussian_projection(G, oracle.Cam(_axis_cam()), oracle.Options())
    assert abs(float(proj["opacity"][0]) - want) < 1e-13


def test_both_filters_off_axis_against_fd_jacobian():
    rng = np.random.default_rng(11)
    cam = _camera(rng)
    e, v = 0.1, 2e-4
    # centres well inside the clamp, in front of the camera
    from test_oracle_projection import _world_from_cam
    for k in range(6):
        xc = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.3, 0.3), 1.0]) * rng.uniform(1.5, 4.0)
        Xw = _world_from_cam(cam, xc)
        q = rng.standard_normal(4)
        s = np.exp(rng.uniform(np.log(0.003), np.log(0.03), 3))
        sig = rng.uniform(0.1, 0.95)
        G = Gaussians(Xw[:, None], q[:, None], s[:, None], np.array([sig]), np.zeros((16, 3, 1)),
                      filter3d=np.array([v]))
        proj = oracle.gaussian_projection(G, oracle.Cam(cam), oracle.Options(mip_2d=e))
        J = _jac_fd(cam, Xw)
        S3 = _sigma3(q, s)
        base = J @ (S3 + v * np.eye(3)) @ J.T
        S2 = base + e * np.eye(2)
        c3 = math.sqrt(np.linalg.det(S3) / np.linalg.det(S3 + v * np.eye(3)))
        c2 = math.sqrt(np.linalg.det(base) / np.linalg.det(S2))
        assert np.allclose(proj["cov2"][0].numpy(), S2, rtol=1e-7, atol=1e-9), k
        assert abs(float(proj["opacity"][0]) - sig * c3 * c2) < 1e-7 * sig, k


def test_filter_size_from_cameras():
    f = 100.0
    c_near = Camera(64, 48, f, f, 32.0, 24.0, np.eye(3), np.array([0.0, 0.0, 1.0]))   # camera z = world z + 1
    c_far = Camera(64, 48, f, f, 32.0, 24.0, np.eye(3), np.array([0.0, 0.0, 3.0]))    # camera z = world z + 3
    c_off = Camera(64, 48, f, f, 32.0, 24.0, np.eye(3), np.array([5.0, 0.0, 0.5]))
    # columns: (0, 0, 2) seen by c_near (z 3) and c_far (z 5), not by c_off
    # (its image x = 100 * 5 / 2.5 + 32 = 232); (1, 0, 2) outside c_near's
    # image (x = 100 / 3 + 32 = 65.3 > 64) but inside c_far's (52); (0, 0, -10)
    # behind both
    mean = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 0.0], [2.0, 2.0, -10.0]])
    G = Gaussians(mean, np.tile([[1.0], [0], [0], [0]], 3), np.full((3, 3), 0.01), np.full(3, 0.5),
                  np.zeros((16, 3, 3)))
    var = oracle.mip_filter3d(G, [c_near, c_far, c_off])
    assert abs(var[0] - 0.2 * (3.0 / f) ** 2) < 1e-15
    assert abs(var[1] - 0.2 * (5.0 / f) ** 2) < 1e-15
    assert var[2] == 0.0


def test_gradients_with_filters_match_finite_differences():
    sc = __import__("synth").workload("tiny", n_surfels=120, n_gaussians=60)
    c = sc.cameras[0]
    cam = Camera(40, 36, c.fx * 40 / 128, c.fy * 40 / 128, 20.0, 18.0, c.R, c.t)
    sc = Scene(sc.surfels, sc.gaussians, [cam])
    sc.gaussians.filter3d = oracle.mip_filter3d(sc.gaussians, [cam])
    opts = oracle.Options(mip_2d=0.1)
    pix = np.arange(cam.width * cam.height)
    d = np.random.default_rng(2).standard_normal((3, pix.size))
    g = oracle.gradients(sc, d, pix, opts=opts)
    which = []
    for grp in ("mean", "scale", "quat", "opacity"):
        flat = np.abs(g[grp]).reshape(-1)
        which += [(grp, int(i)) for i in np.argsort(-flat)[:2]]
    fd = oracle.finite_difference(sc, d, pix, which, opts=opts)
    n = 0
    for (grp, i), v in zip(which, fd):
        if np.isnan(v):
            continue
        n += 1
        a = g[grp].reshape(-1)[i]
        assert abs(a - v) <= 1e-5 * max(abs(v), 1e-3), (grp, i, a, v)
    assert n >= 5


def _fails(test):
    try:
        test()
    except AssertionError:
        return True
    return False


def test_mutation_compensation_without_sqrt_caught(monkeypatch):
    monkeypatch.setattr(R, "filter_compensation", lambda a, b: a / b)  # the ratio, not its root
    assert _fails(test_screen_filter_isotropic_closed_form)
    assert _fails(test_world_filter_compensation_by_eigenvalues)


def test_mutation_no_compensation_caught(monkeypatch):
    monkeypatch.setattr(R, "filter_compensation", lambda a, b: torch.ones_like(a))
    assert _fails(test_screen_filter_isotropic_closed_form)
    assert _fails(test_world_filter_compensation_by_eigenvalues)


def test_mutation_screen_filter_on_top_of_dilation_caught(monkeypatch):
    orig = R.projected_covariance

    def wrong(J, Rcam, sig3, dilation):
        return orig(J, Rcam, sig3, 0.3 if dilation == 0.0 else dilation)
    monkeypatch.setattr(R, "projected_covariance", wrong)
    assert _fails(test_screen_filter_isotropic_closed_form)
    assert _fails(test_both_filters_off_axis_against_fd_jacobian)
