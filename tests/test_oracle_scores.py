"""Pins of the oracle's pruning scores (Sec. 4.1 surfel pruning: covering
score n_{i,j}; Sec. 4.2, Eq. 9: contribution score s_{i,j}).

* A lone fronto-parallel disc covers exactly the pixel centres inside its
  image ellipse (semi-axes f R s / z), counted here as lattice points; of two
  overlapping discs the nearer keeps the shared pixels.
* A lone Gaussian centred on a pixel centre, with no surfel behind it: its
  largest c alpha / (W_s + W_G) is at that pixel, c sigma / (1 + sigma), c the
  largest channel of its colour; two Gaussians centred on the same pixel
  with the same footprint: c_1 sigma_1 / (1 + sigma_1 + sigma_2).
* A Gaussian beyond a surfel's depth + eps, or below the alpha threshold,
  contributes nowhere: score 0.
"""
import math

import numpy as np
import pytest

import oracle
from synth import Scene, empty_gaussians, empty_surfels

from test_oracle_closed_forms import Y00, _cam, _gaussians, _surfels


def _ellipse_lattice(cam, cx, cy, ax, ay):
    """Pixel-centre lattice points inside the axis-aligned ellipse, and the
    smallest distance of any lattice point from its boundary (in rho)."""
    inside, margin = set(), math.inf
    for j in range(cam.height):
        for i in range(cam.width):
            rho = ((i + 0.5 - cx) / ax) ** 2 + ((j + 0.5 - cy) / ay) ** 2
            margin = min(margin, abs(rho - 1.0))
            if rho <= 1.0:
                inside.add(j * cam.width + i)
    return inside, margin


def _disc_footprint(cam, x, y, z, s):
    R = oracle.SURFEL_RADIUS
    return _ellipse_lattice(cam, cam.fx * x / z + cam.cx, cam.fy * y / z + cam.cy,
                            cam.fx * R * s / z, cam.fy * R * s / z)


def test_cover_lone_disc_is_its_lattice_count():
    cam = _cam()
    S = _surfels([[0.021, -0.013, 3.0]], [[1, 0, 0, 0]], [[0.07, 0.07]], 0.4)
    inside, margin = _disc_footprint(cam, 0.021, -0.013, 3.0, 0.07)
    assert margin > 1e-6 and len(inside) > 50
    sc = oracle.scores(Scene(S, empty_gaussians(), [cam]))
    assert int(sc["cover"][0]) == len(inside)


def test_cover_nearer_disc_keeps_the_shared_pixels():
    cam = _cam()
    a = (0.03, -0.01, 2.5, 0.05)   # nearer
    b = (0.09, 0.02, 3.5, 0.09)    # farther, overlapping on screen
    S = _surfels([a[:3], b[:3]], [[1, 0, 0, 0]] * 2, [[a[3]] * 2, [b[3]] * 2], 0.4)
    ia, ma = _disc_footprint(cam, *a)
    ib, mb = _disc_footprint(cam, *b)
    assert min(ma, mb) > 1e-6 and len(ia & ib) > 10 and len(ib - ia) > 10
    sc = oracle.scores(Scene(S, empty_gaussians(), [cam]))
    assert int(sc["cover"][0]) == len(ia)
    assert int(sc["cover"][1]) == len(ib - ia)
    # the same two discs listed the other way round
    S2 = _surfels([b[:3], a[:3]], [[1, 0, 0, 0]] * 2, [[b[3]] * 2, [a[3]] * 2], 0.4)
    sc2 = oracle.scores(Scene(S2, empty_gaussians(), [cam]))
    assert [int(v) for v in sc2["cover"]] == [len(ib - ia), len(ia)]


def _centred_x(cam, z, col=30):
    """World x (camera at the origin, identity rotation) that projects onto
    the centre of pixel column `col`."""
    return (col + 0.5 - cam.cx) * z / cam.fx


def _centred_y(cam, z, row=20):
    return (row + 0.5 - cam.cy) * z / cam.fy


@pytest.mark.parametrize("sigma,s", [(0.8, 0.01), (0.3, 0.02), (0.95, 0.005)])
def test_contrib_lone_gaussian(sigma, s):
    cam = _cam()
    z = 2.0
    dc = np.array([[0.3], [0.9], [-0.2]])
    G = _gaussians([[_centred_x(cam, z), _centred_y(cam, z), z]], [[1, 0, 0, 0]], [[s, s, s]], [sigma], dc)
    sc = oracle.scores(Scene(empty_surfels(), G, [cam]))
    c = max(0.5 + Y00 * 0.3, 0.5 + Y00 * 0.9, 0.5 + Y00 * -0.2)
    assert abs(float(sc["contrib"][0]) - c * sigma / (1 + sigma)) < 1e-12


def test_contrib_two_gaussians_on_one_pixel():
    cam = _cam()
    z = 2.0
    x, y = _centred_x(cam, z), _centred_y(cam, z)
    dc = np.array([[0.1, 0.5], [0.2, -0.4], [0.7, 0.0]])
    G = _gaussians([[x, y, z], [x, y, z]], [[1, 0, 0, 0]] * 2, [[0.01] * 3] * 2, [0.6, 0.25], dc)
    sc = oracle.scores(Scene(empty_surfels(), G, [cam]))
    c0 = 0.5 + Y00 * 0.7
    c1 = 0.5 + Y00 * 0.5
    assert abs(float(sc["contrib"][0]) - c0 * 0.6 / 1.85) < 1e-12
    assert abs(float(sc["contrib"][1]) - c1 * 0.25 / 1.85) < 1e-12


def test_contrib_hidden_or_faint_gaussian_is_zero():
    cam = _cam()
    zs = 2.0
    S = _surfels([[_centred_x(cam, zs), _centred_y(cam, zs), zs]], [[1, 0, 0, 0]], [[0.2, 0.2]], 0.4)
    s = 0.01
    eps = 5.0 / 3.0 * 3 * s
    zf, zb = zs - 0.1, zs + 2 * eps  # in front; beyond depth + eps
    G = _gaussians([[_centred_x(cam, zf), _centred_y(cam, zf), zf],
                    [_centred_x(cam, zb), _centred_y(cam, zb), zb],
                    [_centred_x(cam, zf), _centred_y(cam, zf), zf]],
                   [[1, 0, 0, 0]] * 3, [[s] * 3] * 3, [0.5, 0.9, 0.9 / 255.0], 0.2)
    sc = oracle.scores(Scene(S, G, [cam]))
    c = 0.5 + Y00 * 0.2
    # the front one: the surfel's W_s = 1 and its own alpha at the centre pixel
    # (the faint one adds less than 1/255 nowhere: below the threshold)
    assert abs(float(sc["contrib"][0]) - c * 0.5 / 1.5) < 1e-12
    assert float(sc["contrib"][1]) == 0.0
    assert float(sc["contrib"][2]) == 0.0
