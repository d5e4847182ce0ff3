"""Pins of the oracle's gradients (autograd of the FP64 definition).

* Against FP64 central finite differences on every parameter group the
  joint optimisation stage trains (Sec. 4.2: Gaussians p, s, r, sigma, SH and
  the surfel SH), steps that straddle a discontinuity excluded.
* Closed forms: a lone Gaussian over the background,
  C = (bg + alpha c)/(1 + alpha) gives dC/dsigma = (c - bg)/(1 + sigma)^2 at
  its centre pixel (alpha = sigma there); a pixel showing only a surfel has
  dC/dSH_0 = Y_00.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import Camera, Gaussians, Scene, Surfels, empty_gaussians, empty_surfels, workload, subset

Y00 = 0.28209479177387814


def _crop_scene():
    sc = workload("tiny")
    cam = sc.cameras[0]
    rect = (52, 52, 68, 68)
    gi = oracle.gaussian_candidates(sc.gaussians, cam, rect)
    si = oracle.surfel_candidates(sc.surfels, cam, rect)
    return subset(sc, si, gi), rect


def test_autograd_matches_fd():
    sc, rect = _crop_scene()
    cam = sc.cameras[0]
    pix = oracle.rect_pixels(cam, rect)
    rng = np.random.default_rng(0)
    g = rng.standard_normal((3, len(pix)))
    grads = oracle.gradients(sc, g, pix)
    # pick, per group, the entries with the largest analytic gradient plus a few random ones
    which = []
    for grp, arr in [("mean", grads["mean"]), ("quat", grads["quat"]), ("scale", grads["scale"]),
                     ("opacity", grads["opacity"]), ("sh", grads["sh"]), ("surfel_sh", grads["surfel_sh"])]:
        flat = np.abs(arr).reshape(-1)
        top = np.argsort(-flat)[:6]
        which += [(grp, int(i)) for i in top if flat[i] > 0]
    assert len(which) >= 30
    fd = oracle.finite_difference(sc, g, pix, which)
    ok = ~np.isnan(fd)
    assert ok.sum() >= 0.8 * len(which)
    an = np.array([grads[grp].reshape(-1)[i] for grp, i in which])
    err = np.abs(an[ok] - fd[ok]) / np.maximum(np.abs(fd[ok]), 1e-6)
    assert err.max() < 1e-5, list(zip(np.array(which, dtype=object)[ok][err > 1e-5], an[ok][err > 1e-5], fd[ok][err > 1e-5]))


def test_dsigma_closed_form():
    cam = Camera(33, 33, 40.0, 40.0, 16.5, 16.5, np.eye(3), np.zeros(3), 0.2, (0.2, 0.1, 0.4))
    sh = np.zeros((16, 3, 1))
    sh[0] = np.array([[0.5], [0.9], [-0.3]])
    sigma = 0.6
    G = Gaussians(np.array([[0.0], [0.0], [2.0]]), np.array([[1.0], [0], [0], [0]]),
                  np.full((3, 1), 0.02), np.array([sigma]), sh)
    sc = Scene(empty_surfels(), G, [cam])
    centre = 16 * 33 + 16
    for ch in range(3):
        g = np.zeros((3, 1))
        g[ch, 0] = 1.0
        grads = oracle.gradients(sc, g, [centre])
        c = 0.5 + Y00 * sh[0, ch, 0]
        expect = (c - cam.bg[ch]) / (1 + sigma) ** 2
        assert abs(grads["opacity"][0] - expect) < 1e-12
        # mean gradient vanishes at the centre pixel by symmetry (x, y), z via scale of footprint only
        assert abs(grads["mean"][0, 0]) < 1e-12 and abs(grads["mean"][1, 0]) < 1e-12


def test_surfel_sh_dc_gradient():
    cam = Camera(16, 16, 20.0, 20.0, 8.0, 8.0, np.eye(3), np.zeros(3), 0.2, (0.0, 0.0, 0.0))
    sh = np.zeros((16, 3, 1))
    sh[0] = 0.3
    S = Surfels(np.array([[0.0], [0.0], [2.0]]), np.array([[1.0], [0], [0], [0]]),
                np.full((2, 1), 0.2), sh)
    sc = Scene(S, empty_gaussians(), [cam])
    pix = [8 * 16 + 8, 8 * 16 + 9, 7 * 16 + 8]
    g = np.ones((3, 3))
    grads = oracle.gradients(sc, g, pix)
    assert np.allclose(grads["surfel_sh"][0, :, 0], 3 * Y00, atol=1e-14)
    # degree-1 band: direction from surfel to camera is (0,0,-1): Y_10 = C1 z
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(grads["surfel_sh"][2, :, 0], 3 * c1 * -1.0, atol=1e-14)
