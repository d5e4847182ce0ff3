"""Pins of the oracle's Gaussian projection and view direction, and of the
depth-tie rule, that do not restate the oracle's formulas.

* Projected covariance (Eq. 4's Sigma; readings R10, R11).  The local affine
  approximation of the projection is the Jacobian of the map world point ->
  pixel.  Here that Jacobian is taken by FP64 central differences of the
  composite map X -> pi(R X + t), pi(x, y, z) = (fx x/z + cx, fy y/z + cy),
  in world coordinates, and the world covariance is built from the Gaussian's
  principal axes, each rotated by the quaternion through Hamilton products
  q e_k q*, not from a rotation matrix.  Then
  Sigma2 = J_fd Sigma3 J_fd^T + 0.3 I must hold at off-axis centres to 1e-8.
  Outside 1.3 x the half field of view the clamp of R10 evaluates the
  Jacobian at the centre moved onto that cone, at the same depth: the same
  finite differences taken at the moved point give the expected Sigma2,
  while the projected centre itself is not moved.
* View direction (Sec. 3 after Eq. 1; reading R6): a lone Gaussian whose
  only SH coefficients are one degree-1 term per channel has the colour
  1/2 - C1 d_y a, 1/2 + C1 d_z b, 1/2 - C1 d_x c with d = (o - p)/|o - p| and
  C1 = sqrt(3/(4 pi)).  Read off the rendered pixel under the projected
  centre, where alpha = sigma: c = ((1 + sigma) C - bg)/sigma (Eq. 5).
* Depth ties (reading R5): two overlapping fronto-parallel discs in one plane
  have bit-equal FP64 depths where they overlap; the smaller index wins every
  shared pixel, whichever disc carries it.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Gaussians, Scene, Surfels, empty_gaussians, empty_surfels

C1 = math.sqrt(3.0 / (4.0 * math.pi))


def _hamilton(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _rotate(q, v):
    """v rotated by the unit quaternion q (w, x, y, z): q (0, v) q*."""
    q = np.asarray(q, float) / np.linalg.norm(q)
    qc = q * np.array([1, -1, -1, -1])
    return _hamilton(_hamilton(q, np.concatenate([[0.0], v])), qc)[1:]


def _sigma3(q, s):
    axes = [_rotate(q, e) for e in np.eye(3)]
    return sum(si * si * np.outer(a, a) for si, a in zip(s, axes))


def _camera(rng, W=160, H=120, f=150.0):
    """A camera with a general rotation and position."""
    q = rng.standard_normal(4)
    R = np.stack([_rotate(q, e) for e in np.eye(3)], 1)  # columns: images of the axes
    t = rng.normal(0, 0.5, 3)
    return Camera(W, H, f, f * 1.07, W / 2 + 1.3, H / 2 - 0.7, R, t, 0.2, (0.1, 0.2, 0.3))


def _pix(cam, Xw):
    xc = np.asarray(cam.R) @ Xw + np.asarray(cam.t)
    return np.array([cam.fx * xc[0] / xc[2] + cam.cx, cam.fy * xc[1] / xc[2] + cam.cy])


def _jac_fd(cam, Xw, h=1e-5):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (_pix(cam, Xw + e) - _pix(cam, Xw - e)) / (2 * h)
    return J


def _world_from_cam(cam, xc):
    return np.asarray(cam.R).T @ (np.asarray(xc) - np.asarray(cam.t))


def _gauss(means, quats, scales, opac=0.8, sh=None):
    m = len(means)
    if sh is None:
        sh = np.zeros((16, 3, m))
        sh[0] = 0.3
    return Gaussians(np.asarray(means, float).T.copy(), np.asarray(quats, float).T.copy(),
                     np.asarray(scales, float).T.copy(), np.full(m, opac), sh)


def _projection(G, cam):
    return oracle.gaussian_projection(G, oracle.Cam(cam), oracle.Options())


@pytest.mark.parametrize("seed", [0, 1])
def test_projected_covariance_is_fd_jacobian_off_axis(seed):
    rng = np.random.default_rng(100 + seed)
    cam = _camera(rng)
    limx = 1.3 * cam.width / (2 * cam.fx)
    limy = 1.3 * cam.height / (2 * cam.fy)
    means, quats, scales = [], [], []
    for _ in range(10):  # off axis, inside the clamp
        z = rng.uniform(1.5, 4.0)
        xc = np.array([rng.uniform(0.2, 0.95) * limx * rng.choice([-1, 1]) * z,
                       rng.uniform(0.2, 0.95) * limy * rng.choice([-1, 1]) * z, z])
        means.append(_world_from_cam(cam, xc))
        quats.append(rng.standard_normal(4))
        scales.append(np.exp(rng.uniform(np.log(0.01), np.log(0.2), 3)))
    G = _gauss(means, quats, scales)
    out = _projection(G, cam)
    cov2 = out["cov2"].numpy()
    for k in range(len(means)):
        J = _jac_fd(cam, means[k])
        expect = J @ _sigma3(quats[k], scales[k]) @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(cov2[k], expect, rtol=1e-8, atol=1e-8 * np.abs(expect).max())
        np.testing.assert_allclose(out["phat"].numpy()[k], _pix(cam, means[k]), rtol=1e-12)
    # the third column matters here: without it the covariance would differ
    assert np.abs(_jac_fd(cam, means[0])[:, 2]).max() > 1.0


@pytest.mark.parametrize("side", [(1.6, 0.3), (-0.4, -1.9), (2.2, 1.7)])
def test_projected_covariance_clamped_outside_fov(side):
    """Centres beyond 1.3 x the half-fov tangent: the Jacobian is the one at
    the centre moved onto the clamp cone (same depth), p_hat is not moved."""
    rng = np.random.default_rng(7)
    cam = _camera(rng)
    limx = 1.3 * cam.width / (2 * cam.fx)
    limy = 1.3 * cam.height / (2 * cam.fy)
    z = 2.5
    ax, ay = side
    xc = np.array([ax * limx * z, ay * limy * z, z])
    moved = np.array([np.clip(ax, -1, 1) * limx * z, np.clip(ay, -1, 1) * limy * z, z])
    q = rng.standard_normal(4)
    s = np.array([0.05, 0.12, 0.02])
    p = _world_from_cam(cam, xc)
    out = _projection(_gauss([p], [q], [s]), cam)
    J = _jac_fd(cam, _world_from_cam(cam, moved))
    expect = J @ _sigma3(q, s) @ J.T + 0.3 * np.eye(2)
    cov2 = out["cov2"].numpy()[0]
    np.testing.assert_allclose(cov2, expect, rtol=1e-8, atol=1e-8 * np.abs(expect).max())
    np.testing.assert_allclose(out["phat"].numpy()[0], _pix(cam, p), rtol=1e-12)
    # the clamp changes the answer: the unclamped Jacobian gives another matrix
    J0 = _jac_fd(cam, p)
    other = J0 @ _sigma3(q, s) @ J0.T + 0.3 * np.eye(2)
    assert np.abs(other - expect).max() > 1e-3 * np.abs(expect).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gaussian_view_direction_degree1(seed):
    rng = np.random.default_rng(300 + seed)
    u, v = 20.5, 17.5
    while True:  # a camera whose direction to the centre has no small component
        cam = _camera(rng, W=41, H=37, f=45.0)
        o = -np.asarray(cam.R).T @ np.asarray(cam.t)
        # place the centre so that it projects exactly onto a pixel centre
        z = rng.uniform(1.5, 3.0)
        xc = np.array([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z])
        p = _world_from_cam(cam, xc)
        d = (o - p) / np.linalg.norm(o - p)
        if np.abs(d).min() > 0.15:
            break
    a, b, c = rng.uniform(0.3, 0.6, 3) * rng.choice([-1, 1], 3)
    sh = np.zeros((4, 3, 1))
    sh[1, 0, 0], sh[2, 1, 0], sh[3, 2, 0] = a, b, c
    sigma = 0.7
    G = _gauss([p], [rng.standard_normal(4)], [[0.03, 0.05, 0.04]], opac=sigma, sh=sh)
    out = oracle.render(Scene(empty_surfels(4), G, [cam]))
    centre = 17 * cam.width + 20
    C = out["image"].numpy()[:, centre]
    bg = np.asarray(cam.bg)
    colour = ((1 + sigma) * C - bg) / sigma
    expect = np.array([0.5 - C1 * d[1] * a, 0.5 + C1 * d[2] * b, 0.5 - C1 * d[0] * c])
    assert expect.min() > 0  # no clamp
    np.testing.assert_allclose(colour, expect, atol=1e-12)


@pytest.mark.parametrize("swap", [False, True])
def test_coplanar_tie_goes_to_smaller_index(swap):
    cam = Camera(64, 48, 60.0, 60.0, 32.0, 24.0, np.eye(3), np.zeros(3), 0.2, (0.0, 0.0, 0.0))
    centres = [[-0.12, 0.0, 2.0], [0.10, 0.03, 2.0]]
    scales = [[0.07, 0.07], [0.06, 0.08]]
    dcs = [0.1, 0.9]
    if swap:
        centres, scales, dcs = centres[::-1], scales[::-1], dcs[::-1]
    sh = np.zeros((16, 3, 2))
    sh[0] = np.array(dcs)[None, :]
    S = Surfels(np.asarray(centres).T.copy(), np.tile([[1.0], [0], [0], [0]], (1, 2)),
                np.asarray(scales).T.copy(), sh)
    out = oracle.render(Scene(S, empty_gaussians(), [cam]))
    ids = out["id"].numpy()
    # pixel centres inside both discs (fronto-parallel: circles of radius f R s / z)
    W, H = cam.width, cam.height
    px = (np.arange(W * H) % W) + 0.5
    py = (np.arange(W * H) // W) + 0.5
    inside = []
    for (x, y, z), (su, sv) in zip(centres, scales):
        rx, ry = cam.fx * oracle.SURFEL_RADIUS * su / z, cam.fy * oracle.SURFEL_RADIUS * sv / z
        e = ((px - (cam.fx * x / z + cam.cx)) / rx) ** 2 + ((py - (cam.fy * y / z + cam.cy)) / ry) ** 2
        inside.append(e < 1 - 1e-9)
    both = inside[0] & inside[1]
    assert both.sum() > 30
    assert (ids[both] == 0).all()
    assert (out["depth"].numpy()[both] == 2.0).all()
    only1 = inside[1] & ~inside[0]
    assert only1.sum() > 10 and (ids[only1] == 1).all()
    assert (out["ties"].numpy()[both] == 2).all()
