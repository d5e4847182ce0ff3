"""Pins of the oracle's 4-sample surfel pass (Sec. 5: the surfel pass is
rendered at twice the resolution and downsampled; the OpenGL renderer's
4x MSAA is stated to be equivalent for opaque surfels).

* Against that definition itself: C_s at 4 samples equals the 2x2 mean of a
  1-sample render through a camera of twice the resolution (focal lengths
  and principal point doubled); D_s equals the mean of the finite depths of
  the 2x2 block.
* A fronto-parallel disc: a pixel shows bg + (c - bg) k / 4, k the number
  of its sample points (the pixel centres of the doubled image) inside the
  disc's circle, counted here as lattice points.
* The colour gradient of such a pixel is k/4 of a fully covered one's.
* A planted mistake (sample offsets of half a pixel instead of a quarter)
  is caught.
"""
import importlib
import math

import numpy as np
import pytest

import oracle
from synth import Camera, Scene, empty_gaussians, workload

from test_oracle_closed_forms import Y00, _gaussians, _surfels

R = importlib.import_module("oracle.render")
MS = oracle.Options(surfel_samples=4)


def _double(cam):
    return Camera(2 * cam.width, 2 * cam.height, 2 * cam.fx, 2 * cam.fy, 2 * cam.cx, 2 * cam.cy, cam.R, cam.t,
                  cam.znear, cam.bg)


def test_four_samples_equal_the_doubled_render_downsampled():
    sc = workload("tiny", n_surfels=400, n_gaussians=0)
    c = sc.cameras[0]
    cam = Camera(40, 36, c.fx * 40 / 128, c.fy * 40 / 128, 20.0, 18.0, c.R, c.t, 0.2, (0.1, 0.2, 0.3))
    sc = Scene(sc.surfels, empty_gaussians(), [cam])
    out = oracle.render(sc, opts=MS)
    big = oracle.render(Scene(sc.surfels, empty_gaussians(), [_double(cam)]))
    W, H = cam.width, cam.height
    cs2 = big["color_s"].numpy().reshape(3, H, 2, W, 2)
    assert np.allclose(out["color_s"].numpy().reshape(3, H, W), cs2.mean(axis=(2, 4)), atol=1e-12)
    d2 = big["depth"].numpy().reshape(H, 2, W, 2)
    fin = np.isfinite(d2)
    nh = fin.sum(axis=(1, 3))
    mean = np.where(nh > 0, np.where(fin, d2, 0).sum(axis=(1, 3)) / np.maximum(nh, 1), np.inf)
    got = out["depth"].numpy().reshape(H, W)
    assert np.array_equal(np.isinf(got), np.isinf(mean))
    assert np.allclose(got[np.isfinite(got)], mean[np.isfinite(mean)], atol=1e-12)
    # the samples' ids are the doubled image's, in (0,0), (1,0), (0,1), (1,1) order
    ids2 = big["id"].numpy().reshape(H, 2, W, 2)
    sid = out["sample_id"].numpy().reshape(4, H, W)
    for k, (a, b) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        assert np.array_equal(sid[k], ids2[:, b, :, a])
    assert 0.2 < (sid >= 0).mean() < 0.95  # edges present


def _disc_case():
    cam = Camera(30, 28, 40.0, 40.0, 15.0, 14.0, np.eye(3), np.zeros(3), 0.2, (0.2, 0.1, 0.0))
    z, s = 2.0, 0.11
    S = _surfels([[0.013, -0.021, z]], [[1, 0, 0, 0]], [[s, s]], 0.6)
    cx, cy = cam.fx * 0.013 / z + cam.cx, cam.fy * -0.021 / z + cam.cy
    r = cam.fx * oracle.SURFEL_RADIUS * s / z
    return cam, S, cx, cy, r


def test_disc_edge_pixels_show_the_covered_sample_fraction():
    cam, S, cx, cy, r = _disc_case()
    out = oracle.render(Scene(S, empty_gaussians(), [cam]), opts=MS)
    c = 0.5 + Y00 * 0.6
    bg = np.array(cam.bg)
    W, H = cam.width, cam.height
    partial = 0
    for j in range(H):
        for i in range(W):
            k, margin = 0, math.inf
            for a in (0, 1):
                for b in (0, 1):
                    x, y = i + 0.25 + 0.5 * a, j + 0.25 + 0.5 * b
                    rho = ((x - cx) ** 2 + (y - cy) ** 2) / r ** 2
                    margin = min(margin, abs(rho - 1))
                    k += rho <= 1
            if margin < 1e-9:
                continue
            partial += 0 < k < 4
            want = bg + (c - bg) * k / 4
            assert np.allclose(out["color_s"][:, j * W + i].numpy(), want, atol=1e-12), (i, j, k)
    assert partial > 10


def test_edge_pixel_gradient_is_the_covered_fraction():
    cam, S, cx, cy, r = _disc_case()
    sc = Scene(S, empty_gaussians(), [cam])
    # a pixel whose 4 samples are all inside, and one on the rim with 1..3 inside
    inside = int(cy) * cam.width + int(cx)
    out = oracle.render(sc, opts=MS)
    frac = None
    for p in range(cam.width * cam.height):
        k = int((out["sample_id"][:, p] == 0).sum())
        if 0 < k < 4:
            frac = (p, k)
            break
    assert frac is not None
    for p, k in ((inside, 4), frac):
        d = np.zeros((3, 1))
        d[0, 0] = 1.0
        g = oracle.gradients(sc, d, np.array([p]), opts=MS)
        assert abs(g["surfel_sh"][0, 0, 0] - Y00 * k / 4) < 1e-12, (p, k)


def _fails(test):
    try:
        test()
    except AssertionError:
        return True
    return False


def test_mutation_sample_offsets_caught(monkeypatch):
    monkeypatch.setattr(R, "SAMPLE_OFFSETS", ((-0.5, -0.5), (0.5, -0.5), (-0.5, 0.5), (0.5, 0.5)))
    assert _fails(test_four_samples_equal_the_doubled_render_downsampled)
    assert _fails(test_disc_edge_pixels_show_the_covered_sample_fraction)
