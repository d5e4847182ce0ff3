"""Closed-form pins of the oracle's two passes.

* A single surfel: its disc boundary maps to the image conic
  Q = H^-T diag(1, 1, -R^2) H^-1 of the plane-to-image homography
  H = K [s_u t_u | s_v t_v | mu] (Sec. 3 surfel definition); a fronto-parallel
  disc is a circle of radius f R s / z pixels.  Depth is checked through the
  homography's inverse (plane point -> camera z), not the ray-plane formula.
* The opaque disc radius R = sqrt(2 ln 255) (Sec. 4.1 after Eq. 7).
* A single isotropic Gaussian on the optical axis (Eq. 4): projected
  covariance ((f s / z)^2 + 0.3) I, support radius
  sqrt(2 ln(255 sigma) ((f s / z)^2 + 0.3)), colour (bg + alpha c)/(1 + alpha)
  with no surfel (Eq. 5).
* The depth test with the adaptive eps_i = (5/3) sum s (Sec. 5, Eq. 2-3).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Gaussians, Scene, Surfels, empty_gaussians, empty_surfels

Y00 = 0.28209479177387814


def _cam(W=64, H=48, f=60.0, bg=(0.1, 0.2, 0.3)):
    return Camera(W, H, f, f * 1.1, W / 2 + 0.3, H / 2 - 0.2, np.eye(3), np.zeros(3), 0.2, bg)


def _surfels(mean, quat, scale, dc):
    n = len(mean)
    sh = np.zeros((16, 3, n))
    sh[0] = np.asarray(dc, dtype=np.float64).reshape(3, n) if np.ndim(dc) else dc
    return Surfels(np.asarray(mean, np.float64).T.copy(), np.asarray(quat, np.float64).T.copy(),
                   np.asarray(scale, np.float64).T.copy(), sh)


def _gaussians(mean, quat, scale, opac, dc):
    m = len(mean)
    sh = np.zeros((16, 3, m))
    sh[0] = dc
    return Gaussians(np.asarray(mean, np.float64).T.copy(), np.asarray(quat, np.float64).T.copy(),
                     np.asarray(scale, np.float64).T.copy(), np.asarray(opac, np.float64), sh)


def test_disc_radius():
    assert abs(oracle.SURFEL_RADIUS - math.sqrt(2 * math.log(255))) < 1e-15
    assert abs(oracle.SURFEL_RADIUS - 3.3290) < 1e-4


def test_fronto_parallel_circle():
    cam = _cam()
    z0, s = 3.0, 0.08
    S = _surfels([[0.02, -0.01, z0]], [[1, 0, 0, 0]], [[s, s]], 0.4)
    out = oracle.render(Scene(S, empty_gaussians(), [cam]))
    W, H = cam.width, cam.height
    px = (np.arange(W * H) % W) + 0.5
    py = (np.arange(W * H) // W) + 0.5
    cx = cam.fx * 0.02 / z0 + cam.cx
    cy = cam.fy * -0.01 / z0 + cam.cy
    # ellipse with semi-axes f R s / z (fx != fy here)
    rho = ((px - cx) / (cam.fx * oracle.SURFEL_RADIUS * s / z0)) ** 2 + \
          ((py - cy) / (cam.fy * oracle.SURFEL_RADIUS * s / z0)) ** 2
    inside = rho <= 1
    safe = np.abs(rho - 1) > 1e-9
    assert inside.sum() > 50
    ids = out["id"].numpy()
    assert np.array_equal((ids == 0)[safe], inside[safe])
    assert np.allclose(out["depth"].numpy()[inside], z0, rtol=0, atol=1e-12)
    c = 0.5 + Y00 * 0.4
    assert np.allclose(out["image"].numpy()[:, inside], c, atol=1e-12)
    assert np.allclose(out["image"].numpy()[:, ~inside], np.array(cam.bg)[:, None], atol=1e-15)


def _rotq(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return [math.cos(ang / 2), *(math.sin(ang / 2) * axis)]


def _rot(q):
    w, x, y, z = np.asarray(q) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tilted_disc_is_homography_conic(seed):
    rng = np.random.default_rng(seed)
    cam = _cam(80, 60, 70.0)
    # camera not at the origin: a general world->camera transform
    Rc = _rot(_rotq(rng.standard_normal(3), 0.3))
    tc = rng.normal(0, 0.2, 3)
    cam = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, Rc, tc, 0.2, cam.bg)
    mu_c = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2), rng.uniform(2.0, 3.0)])
    p = Rc.T @ (mu_c - tc)
    q = _rotq(rng.standard_normal(3), rng.uniform(0.2, 1.2))
    su, sv = rng.uniform(0.03, 0.08, 2)
    S = _surfels([p], [q], [[su, sv]], 0.2)
    out = oracle.render(Scene(S, empty_gaussians(), [cam]))
    A = Rc @ _rot(q)
    K = np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1]])
    Hm = K @ np.stack([su * A[:, 0], sv * A[:, 1], mu_c], 1)
    Hi = np.linalg.inv(Hm)
    R2 = oracle.SURFEL_RADIUS ** 2
    Q = Hi.T @ np.diag([1, 1, -R2]) @ Hi
    W, Hh = cam.width, cam.height
    X = np.stack([(np.arange(W * Hh) % W) + 0.5, (np.arange(W * Hh) // W) + 0.5,
                  np.ones(W * Hh)], 1)
    val = np.einsum("pi,ij,pj->p", X, Q, X)
    # the side of the conic containing the projected centre
    c0 = Hm @ np.array([0, 0, 1.0])
    sgn = np.sign(c0 @ Q @ c0)
    inside = sgn * val >= 0
    uvw = X @ Hi.T                           # plane coordinates (u s, v s, 1) up to scale
    uv = uvw[:, :2] / uvw[:, 2:]
    rho = (uv ** 2).sum(1)
    safe = np.abs(rho - R2) > 1e-7 * R2
    assert inside.sum() > 30
    ids = out["id"].numpy()
    assert np.array_equal((ids == 0)[safe], inside[safe])
    # depth: camera z of the plane point mu + u su tu + v sv tv
    Xc = mu_c[None, :] + uv[:, :1] * su * A[:, 0] + uv[:, 1:] * sv * A[:, 1]
    hit = ids == 0
    assert np.allclose(out["depth"].numpy()[hit], Xc[hit, 2], rtol=1e-12)


@pytest.mark.parametrize("sigma,s,z", [(0.9, 0.01, 3.0), (0.3, 0.004, 2.0), (0.99, 0.03, 4.0)])
def test_isotropic_gaussian_on_axis(sigma, s, z):
    cam = Camera(65, 65, 80.0, 80.0, 32.5, 32.5, np.eye(3), np.zeros(3), 0.2, (0.1, 0.2, 0.3))
    dc = np.array([0.7, -0.2, 0.1])
    G = _gaussians([[0, 0, z]], [[1, 0, 0, 0]], [[s, s, s]], [sigma], dc[:, None])
    out = oracle.render(Scene(empty_surfels(), G, [cam]))
    var = (cam.fx * s / z) ** 2 + 0.3
    px = (np.arange(65 * 65) % 65) + 0.5 - 32.5
    py = (np.arange(65 * 65) // 65) + 0.5 - 32.5
    rho2 = px ** 2 + py ** 2
    alpha = sigma * np.exp(-rho2 / (2 * var))
    support = rho2 <= 2 * math.log(255 * sigma) * var
    assert np.array_equal(support, alpha >= 1 / 255)
    a = np.where(support, alpha, 0.0)
    assert np.allclose(out["wg"].numpy(), a, atol=1e-14)
    c = np.maximum(0.0, 0.5 + Y00 * dc)
    bg = np.array(cam.bg)
    expect = (bg[:, None] + a[None, :] * c[:, None]) / (1 + a[None, :])
    assert np.allclose(out["image"].numpy(), expect, atol=1e-14)


def test_sigma_below_threshold_never_contributes():
    cam = _cam()
    G = _gaussians([[0, 0, 2.0]], [[1, 0, 0, 0]], [[0.05, 0.05, 0.05]], [0.9 / 255], np.zeros((3, 1)))
    out = oracle.render(Scene(empty_surfels(), G, [cam]))
    assert float(out["wg"].abs().max()) == 0.0


@pytest.mark.parametrize("frac,counted", [(0.9, True), (1.1, False), (-0.5, True)])
def test_depth_test_adaptive_eps(frac, counted):
    """A fronto-parallel surfel at depth 2; a Gaussian centred at depth
    2 + frac*eps on the axis counts iff d < D_s + eps with eps = 5/3 sum s."""
    cam = _cam()
    s = np.array([0.01, 0.02, 0.015])
    eps = 5.0 / 3.0 * s.sum()
    S = _surfels([[0, 0, 2.0]], [[1, 0, 0, 0]], [[0.2, 0.2]], 0.0)
    G = _gaussians([[0, 0, 2.0 + frac * eps]], [[1, 0, 0, 0]], [s], [0.8], np.zeros((3, 1)))
    out = oracle.render(Scene(S, G, [cam]))
    centre = (cam.height // 2) * cam.width + cam.width // 2
    assert out["id"][centre] == 0
    assert (float(out["wg"][centre]) > 0) == counted


def test_depth_test_strict_at_boundary():
    """d == D_s + eps exactly (dyadic numbers, exact in FP64): not counted;
    a hair in front: counted (Eq. 2-3 use a strict inequality)."""
    cam = _cam()
    S = _surfels([[0, 0, 2.0]], [[1, 0, 0, 0]], [[0.2, 0.2]], 0.0)
    centre = (cam.height // 2) * cam.width + cam.width // 2
    opts = oracle.Options(eps_const=0.125)
    for z, counted in [(2.125, False), (2.125 - 2.0 ** -40, True)]:
        G = _gaussians([[0, 0, z]], [[1, 0, 0, 0]], [[0.01, 0.01, 0.01]], [0.8], np.zeros((3, 1)))
        out = oracle.render(Scene(S, G, [cam]), opts=opts)
        assert float(out["depth"][centre]) == 2.0
        assert (float(out["wg"][centre]) > 0) == counted, z


def test_eps_constant_and_zero_knobs():
    cam = _cam()
    s = np.array([0.01, 0.01, 0.01])
    S = _surfels([[0, 0, 2.0]], [[1, 0, 0, 0]], [[0.2, 0.2]], 0.0)
    G = _gaussians([[0, 0, 2.05]], [[1, 0, 0, 0]], [s], [0.8], np.zeros((3, 1)))
    sc = Scene(S, G, [cam])
    centre = (cam.height // 2) * cam.width + cam.width // 2
    assert float(oracle.render(sc, opts=oracle.Options(eps_const=0.1))["wg"][centre]) > 0
    assert float(oracle.render(sc, opts=oracle.Options(eps_const=0.0))["wg"][centre]) == 0
    G0 = _gaussians([[0, 0, 1.99]], [[1, 0, 0, 0]], [s], [0.8], np.zeros((3, 1)))
    assert float(oracle.render(Scene(S, G0, [cam]), opts=oracle.Options(eps_const=0.0))["wg"][centre]) > 0


def test_near_plane_and_behind_camera():
    cam = _cam()
    # surfel straddling the near plane: only hits with z >= znear count
    S = _surfels([[0, 0, 0.2]], [[math.cos(0.6), math.sin(0.6), 0, 0]], [[0.3, 0.3]], 0.1)
    out = oracle.render(Scene(S, empty_gaussians(), [cam]))
    hit = out["id"].numpy() == 0
    assert hit.any() and (~hit).any()
    assert float(out["depth"][torch.tensor(hit)].min()) >= 0.2
    # a Gaussian centred in front of the near plane or behind the camera is culled
    G = _gaussians([[0, 0, 0.19], [0, 0, -1.0]], [[1, 0, 0, 0]] * 2, [[0.05] * 3] * 2, [0.9, 0.9],
                   np.ones((3, 2)))
    out = oracle.render(Scene(empty_surfels(), G, [cam]))
    assert float(out["wg"].abs().max()) == 0.0
