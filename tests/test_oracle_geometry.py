"""Pins of the oracle's geometry channels (2D-GES smoothing, Eq. 10-12).

* One Gaussian on the optical axis, centred on a pixel centre, no surfel:
  at that pixel alpha = sigma, so D_G = sigma z, N_G = sigma n with n its
  shortest axis written out from the rotation (turned to face the camera),
  D_smooth = sigma z / (1 + sigma), N_smooth = sigma n / (1 + sigma).
* A tilted disc in front: N_s is its rotated z axis facing the camera;
  behind a Gaussian, D_smooth = (z_s + sigma z) / (1 + sigma) (W_s = 1).
* A Gaussian beyond the surfel depth + eps adds nothing (Eq. 10's
  indicator); an uncovered pixel with no Gaussian has all channels 0.
"""
import math

import numpy as np
import pytest

import importlib

import oracle
from synth import Camera, Scene, empty_gaussians, empty_surfels

from test_oracle_closed_forms import _gaussians, _surfels

R = importlib.import_module("oracle.render")


def _cam():
    # a pixel centre on the optical axis: cx, cy at a pixel centre
    return Camera(33, 31, 40.0, 40.0, 16.5, 15.5, np.eye(3), np.zeros(3), 0.2, (0.0, 0.0, 0.0))


def _rot_x(th):
    return [math.cos(th / 2), math.sin(th / 2), 0.0, 0.0]


def _centre(cam):
    return 15 * cam.width + 16


def test_lone_gaussian_depth_and_shortest_axis():
    cam = _cam()
    th, z, sig = 0.7, 2.5, 0.6
    # scales: x 0.05, y 0.03, z 0.01 -> the shortest axis is the rotated z axis
    G = _gaussians([[0.0, 0.0, z]], [_rot_x(th)], [[0.05, 0.03, 0.01]], [sig], 0.3)
    out = oracle.geometry(Scene(empty_surfels(), G, [cam]), 0, [_centre(cam)])
    # rotation about x by th: its z column is (0, -sin th, cos th); the camera
    # at the origin is in the -z direction from the centre, so it flips
    n = np.array([0.0, math.sin(th), -math.cos(th)])
    assert abs(float(out["depth_g"][0]) - sig * z) < 1e-12
    assert np.allclose(out["normal_g"][:, 0].numpy(), sig * n, atol=1e-12)
    assert abs(float(out["depth_smooth"][0]) - sig * z / (1 + sig)) < 1e-12
    assert np.allclose(out["normal_smooth"][:, 0].numpy(), sig * n / (1 + sig), atol=1e-12)
    assert np.allclose(out["normal_s"][:, 0].numpy(), 0.0)


def test_shortest_axis_follows_the_scales():
    cam = _cam()
    th, z, sig = 0.4, 3.0, 0.5
    # now the x axis is the shortest: the rotation leaves it at (1, 0, 0)
    G = _gaussians([[0.0, 0.0, z]], [_rot_x(th)], [[0.004, 0.03, 0.02]], [sig], 0.3)
    n = oracle.gaussian_normals(G, oracle.Cam(cam)).numpy()[0]
    assert np.allclose(np.abs(n), [1.0, 0.0, 0.0], atol=1e-12)


def test_disc_normal_and_smoothed_depth():
    cam = _cam()
    th, zs, z, sig = -0.5, 1.5, 1.52, 0.7
    S = _surfels([[0.0, 0.0, zs]], [_rot_x(th)], [[0.2, 0.2]], 0.4)
    # a Gaussian just behind the disc but within eps = (5/3)(sum of scales)
    G = _gaussians([[0.0, 0.0, z]], [_rot_x(0.0)], [[0.02, 0.02, 0.01]], [sig], 0.3)
    out = oracle.geometry(Scene(S, G, [cam]), 0, [_centre(cam)])
    assert int(out["id"][0]) == 0
    ns = np.array([0.0, math.sin(th), -math.cos(th)])
    ns = ns if ns @ np.array([0.0, 0.0, -zs]) >= 0 else -ns
    assert np.allclose(out["normal_s"][:, 0].numpy(), ns, atol=1e-12)
    ds = float(out["depth"][0])
    assert abs(ds - zs) < 1e-12  # the ray on the axis meets the disc at its centre
    assert abs(float(out["depth_smooth"][0]) - (ds + sig * z) / (1 + sig)) < 1e-12
    ng = np.array([0.0, 0.0, -1.0])
    assert np.allclose(out["normal_smooth"][:, 0].numpy(), (ns + sig * ng) / (1 + sig), atol=1e-12)


def test_hidden_gaussian_and_empty_pixel():
    cam = _cam()
    S = _surfels([[0.0, 0.0, 1.0]], [_rot_x(0.0)], [[0.05, 0.05]], 0.4)
    G = _gaussians([[0.0, 0.0, 2.0]], [_rot_x(0.0)], [[0.02, 0.02, 0.01]], [0.8], 0.3)  # far beyond eps
    out = oracle.geometry(Scene(S, G, [cam]), 0, [_centre(cam), 0])
    assert float(out["depth_g"][0]) == 0.0 and float(out["wg"][0]) == 0.0
    assert abs(float(out["depth_smooth"][0]) - 1.0) < 1e-12
    # the corner pixel: neither the disc nor the Gaussian reaches it
    assert float(out["depth_smooth"][1]) == 0.0
    assert np.all(out["normal_smooth"][:, 1].numpy() == 0.0)


def _fails(test):
    try:
        test()
    except AssertionError:
        return True
    return False


def test_mutation_longest_axis_caught(monkeypatch):
    orig = R.quat_to_rot

    def wrong_normals(G, cam):
        Rq = orig(R._t(G.quat))
        k = R.torch.argmax(R._t(G.scale), dim=0)
        n = R.torch.gather(Rq, 2, k[:, None, None].expand(-1, 3, 1))[:, :, 0]
        return R.facing(n, cam.o[None, :] - R._t(G.mean).T)
    monkeypatch.setattr(R, "gaussian_normals", wrong_normals)
    monkeypatch.setattr(oracle, "gaussian_normals", wrong_normals)
    assert _fails(test_lone_gaussian_depth_and_shortest_axis)


def test_mutation_no_facing_flip_caught(monkeypatch):
    monkeypatch.setattr(R, "facing", lambda n, to_cam: n)
    assert _fails(test_lone_gaussian_depth_and_shortest_axis)
    assert _fails(test_disc_normal_and_smoothed_depth)
