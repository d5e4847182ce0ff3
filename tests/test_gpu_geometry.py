"""GPU parity of ges_geometry (2D-GES geometry channels, Eq. 10-12) against
the FP64 oracle, through the C ABI.

Bars, at pixels where no decision is within FP32 reach (gpu_util bands) and
no depth tie below 1e-6: N_s within 1e-5 (a rotation column); D_G and
D_smooth within 1e-4 x max(1, depth scale) (the sums carry the 2^-24
fixed-point rounding and the FP32 alpha of the image's C_G); N_G, N_smooth
within 1e-4 (as W_G).  The channels are bit-identical under a permutation of
the Gaussian array and across splat tile shapes."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_17545_amd import Renderer
from synth import Camera, Scene, permute_gaussians, workload

from gpu_util import bands, sample_pixels, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("normal_s", "depth_g", "normal_g", "depth_smooth", "normal_smooth")


def _gpu(scene, **opts):
    S, G = to_dev(scene)
    r = Renderer(**opts)
    f = r.render(S, G, scene.cameras)
    g = r.geometry(f)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}, f


def _compare(g, scene, v, off, pix, label):
    cam = scene.cameras[v]
    P = cam.width * cam.height
    out = oracle.geometry(scene, v, pix)
    b = bands(out)
    ok = b["safe"]
    dscale = max(1.0, float(np.nanmax(np.where(np.isfinite(out["depth"].numpy()), out["depth"].numpy(), 0))))
    chans = {}
    for k in KEYS:
        c = 3 if k.startswith("normal") else 1
        chans[k] = g[k][c * off: c * (off + P)].reshape(c, P)[:, pix].astype(np.float64)
    err = {}
    err["normal_s"] = np.abs(chans["normal_s"][:, ok] - out["normal_s"].numpy()[:, ok]).max(initial=0.0)
    err["depth_g"] = np.abs(chans["depth_g"][0, ok] - out["depth_g"].numpy()[ok]).max(initial=0.0)
    err["depth_smooth"] = np.abs(chans["depth_smooth"][0, ok] - out["depth_smooth"].numpy()[ok]).max(initial=0.0)
    err["normal_g"] = np.abs(chans["normal_g"][:, ok] - out["normal_g"].numpy()[:, ok]).max(initial=0.0)
    err["normal_smooth"] = np.abs(chans["normal_smooth"][:, ok] - out["normal_smooth"].numpy()[:, ok]).max(initial=0.0)
    print(f"[geometry] {label}: {int(ok.sum())} of {len(pix)} pixels compared, depth scale {dscale:.2f}, "
          f"max errors {err}", flush=True)
    assert err["normal_s"] <= 1e-5, err
    assert err["depth_g"] <= 1e-4 * dscale and err["depth_smooth"] <= 1e-4 * dscale, err
    assert err["normal_g"] <= 1e-4 and err["normal_smooth"] <= 1e-4, err
    # something was actually compared
    assert np.abs(out["depth_g"].numpy()[ok]).max(initial=0.0) > 0
    assert np.abs(out["normal_s"].numpy()[:, ok]).max(initial=0.0) > 0


def test_tiny_geometry_vs_oracle():
    print("[case] tiny 128x128 geometry channels", flush=True)
    sc = workload("tiny")
    g, _ = _gpu(sc)
    _compare(g, sc, 0, 0, np.arange(128 * 128), "tiny")


def test_geometry_tile_shapes_and_permutation_bitwise():
    print("[case] tiny geometry: splat tiles 8x8 / 16x8, Gaussian permutation", flush=True)
    sc = workload("tiny")
    a, _ = _gpu(sc)
    for sp in ((8, 8), (16, 8)):
        b, _ = _gpu(sc, splat_tile=sp)
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (sp, k)
    G2, _ = permute_gaussians(sc.gaussians, 13)
    c, _ = _gpu(Scene(sc.surfels, G2, sc.cameras))
    for k in KEYS:
        assert np.array_equal(a[k], c[k]), k


def test_multiview_geometry_vs_oracle():
    print("[case] tiny, 3 views of different sizes: geometry channels", flush=True)
    sc = workload("tiny")
    c = sc.cameras[0]
    cams = [c, Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
            Camera(65, 33, 60.0, 60.0, 32.5, 16.5, c.R, c.t + np.array([0.0, -0.1, 0.3]))]
    full = Scene(sc.surfels, sc.gaussians, cams)
    g, f = _gpu(full)
    for v in range(3):
        _compare(g, full, v, f.offsets[v], np.arange(cams[v].width * cams[v].height), f"view {v}")


def test_surfaces_1m_1080p_geometry_sampled():
    print("[case] 1M surfels 1080p: geometry channels at sampled pixels", flush=True)
    sc = workload("surfaces_1m_1080p")
    g, _ = _gpu(sc)
    _compare(g, sc, 0, 0, sample_pixels(sc.cameras[0], 48, 9), "1080p sampled")
