"""Batched multi-view frames (Sec. 4, multi-view optimisation) against the
FP64 oracle, forward and backward, in the launch configuration the
benchmark times: one autotuned plan, captured into a graph and replayed.

* tiny, 3 views of different sizes: the batched gradient equals the sum over
  views of the oracle's gradients (each view's band pixels zeroed);
* the 16-camera ring of mixed resolutions (640x360, 1280x720, 1600x1060,
  1920x1080) around the 1M-surfel / 500k-Gaussian scene, forward and
  backward: sampled pixels of one view of each resolution against the
  oracle; the gradient of a 64x64 crop loss on one view against the
  oracle's on the primitives that reach the crop; and the batched gradient
  of a full random upstream gradient against the sum of the 16 single-view
  ges_backward results."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_17545_amd import PlannedFrame, Renderer
from synth import Camera, Scene, workload

from gpu_util import (bands, check_grads, compare_view, crop_gradient_reference, grads_np, sample_pixels,
                      to_dev)

pytestmark = pytest.mark.gpu


def test_tiny_three_views_gradient_vs_oracle_sum():
    print("[case] tiny, 3 views batched backward vs the sum of oracle gradients", flush=True)
    sc = workload("tiny")
    c = sc.cameras[0]
    cams = [c, Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
            Camera(64, 64, 60.0, 60.0, 32.0, 32.0, c.R, c.t + np.array([0.0, -0.1, 0.3]))]
    rng = np.random.default_rng(21)
    ds, ref = [], None
    for cam in cams:
        sc1 = Scene(sc.surfels, sc.gaussians, [cam])
        out = oracle.render(sc1)
        d = rng.standard_normal((3, cam.width * cam.height))
        d[:, ~bands(out)["safe"]] = 0.0
        ds.append(d)
        g = oracle.gradients(sc1, d, np.arange(cam.width * cam.height))
        ref = g if ref is None else {k: ref[k] + g[k] for k in g}
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=True)
    pf.d_image.copy_(torch.as_tensor(np.concatenate([d.reshape(-1) for d in ds]).astype(np.float32)))
    pf.launch()
    torch.cuda.synchronize()
    pf.poll()
    check_grads(grads_np(pf.grads), ref, "3 views batched vs oracle sum")


@pytest.fixture(scope="module")
def ring16():
    sc = workload("ring16_1m")
    S, G = to_dev(sc)
    print("[case] ring16_1m: plan (autotuned), 16 views, forward + backward", flush=True)
    pf = PlannedFrame(S, G, sc.cameras, backward=True, autotune=True)
    yield sc, S, G, pf
    pf.close()


def test_ring16_forward_vs_oracle(ring16):
    sc, S, G, pf = ring16
    pf.d_image.zero_()
    pf.launch()
    torch.cuda.synchronize()
    st = pf.poll()
    assert st.flags == 0
    for v in (0, 1, 2, 3):  # 640x360, 1280x720, 1600x1060, 1920x1080
        cam = sc.cameras[v]
        print(f"[case] ring16 view {v} ({cam.width}x{cam.height}): sampled pixels vs oracle", flush=True)
        compare_view(pf, sc, v=v, pix=sample_pixels(cam, 40, 100 + v))


def test_ring16_crop_gradient_vs_oracle(ring16):
    sc, S, G, pf = ring16
    v = 7  # a 1920x1080 view
    cam = sc.cameras[v]
    x0, y0 = cam.width // 2 - 32, cam.height // 2 - 32
    d_view, ref = crop_gradient_reference(sc, v, (x0, y0, x0 + 64, y0 + 64), seed=17)
    d = torch.zeros_like(pf.d_image)
    off = pf.offsets[v]
    d[3 * off: 3 * off + d_view.size] = torch.as_tensor(d_view.reshape(-1).astype(np.float32))
    pf.d_image.copy_(d)
    pf.launch()
    torch.cuda.synchronize()
    pf.poll()
    check_grads(grads_np(pf.grads), ref, f"ring16 view {v} 64x64 crop")


def test_ring16_batched_gradient_equals_sum_of_single_views(ring16):
    sc, S, G, pf = ring16
    gen = torch.Generator(device="cuda").manual_seed(23)
    d = torch.randn(pf.d_image.shape, generator=gen, device="cuda") * 1e-3
    pf.d_image.copy_(d)
    pf.launch()
    torch.cuda.synchronize()
    pf.poll()
    batched = grads_np(pf.grads)
    o = pf.options()
    r = Renderer(raster_tile=o.raster_tile, splat_tile=(o.splat_tile_w, o.splat_tile_h))
    total = None
    for v, cam in enumerate(sc.cameras):
        f = r.render(S, G, [cam])
        off, P = pf.offsets[v], cam.width * cam.height
        g = grads_np(r.backward(f, d[3 * off: 3 * (off + P)]))
        # the single-view frame equals the plan's view bit for bit
        assert torch.equal(f.view("image", 0), pf.view("image", v)), v
        total = g if total is None else {k: total[k] + g[k] for k in g}
    torch.cuda.synchronize()
    check_grads(batched, total, "ring16 batched vs sum of 16 single-view backward")
