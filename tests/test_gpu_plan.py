"""Plans: a multi-view frame (forward + backward) captured into one hipGraph.

Every replay is checked bitwise against the eager call sequence with the same
options, with eager work and synchronisations between replays; the replayed
results are also held to the oracle.  Camera changes between replays, the
autotuner's choice and its cache are covered."""
import json
import math
import os

import numpy as np
import pytest
import torch

from paper_2504_17545_amd import PlannedFrame, Renderer, _lib
from synth import Camera, Scene, workload

from gpu_util import compare_view, to_dev

pytestmark = pytest.mark.gpu


def _cams(sc):
    c = sc.cameras[0]
    return [c,
            Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
            Camera(65, 33, 60.0, 60.0, 32.5, 16.5, c.R, c.t + np.array([0.0, -0.1, 0.3]))]


def _eager(sc, cams, d_image, opt):
    S, G = to_dev(sc)
    r = Renderer(raster_tile=opt.raster_tile, splat_tile=(opt.splat_tile_w, opt.splat_tile_h),
                 surfel_pair_capacity=opt.surfel_pair_capacity, gauss_pair_capacity=opt.gauss_pair_capacity)
    f = r.render(S, G, cams)
    g = r.backward(f, d_image)
    torch.cuda.synchronize()
    return f, g


def test_plan_replays_match_eager():
    print("[case] plan, 3 views, fwd+bwd, 4 replays", flush=True)
    sc = workload("tiny")
    cams = _cams(sc)
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=True)
    opt = pf.options()
    rng = np.random.default_rng(4)
    d = torch.as_tensor(rng.standard_normal(pf.image.numel()).astype(np.float32), device="cuda")
    pf.d_image.copy_(d)
    f, g = _eager(sc, cams, d, opt)
    for rep in range(4):
        pf.launch()
        torch.cuda.synchronize()
        for name in ("surfel_id", "depth", "color_s", "image", "accum"):
            assert torch.equal(getattr(pf, name), getattr(f, name)), (rep, name)
        for k, v in g.items():
            assert torch.equal(pf.grads[k], v), (rep, k)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        pf.grads["mean"].zero_()
    st = pf.poll()
    assert st.flags == 0
    for v in range(3):
        compare_view(pf, Scene(sc.surfels, sc.gaussians, cams), v=v)


def test_plan_camera_change():
    print("[case] plan, moved cameras", flush=True)
    sc = workload("tiny")
    cams = _cams(sc)
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=False)
    opt = pf.options()
    moved = []
    for k, c in enumerate(cams):
        ang = 0.05 * (k + 1)
        Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
        moved.append(Camera(c.width, c.height, c.fx * 1.02, c.fy * 1.02, c.cx, c.cy, Rz @ np.asarray(c.R),
                            np.asarray(c.t) + 0.01, c.znear, c.bg))
    for rep in range(2):
        pf.launch(moved if rep == 0 else cams)
        torch.cuda.synchronize()
        ref, _ = _eager(sc, moved if rep == 0 else cams,
                        torch.zeros(pf.image.numel(), device="cuda"), opt)
        assert torch.equal(pf.image, ref.image), rep
        assert torch.equal(pf.surfel_id, ref.surfel_id), rep
    bad = list(cams)
    bad[1] = Camera(97, 80, 90.0, 90.0, 48.0, 40.0, cams[1].R, cams[1].t)
    with pytest.raises(_lib.GESError):
        pf.launch(bad)


def test_plan_camera_changes_without_waiting():
    """Six launches with new cameras each (more than the staging buffers),
    no synchronisation in between: each replay's image, copied on the stream
    right after it, equals the eager render of its own cameras."""
    print("[case] plan, cameras changed on every launch, no sync", flush=True)
    sc = workload("tiny")
    cams = _cams(sc)
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=False)
    opt = pf.options()
    sets, images = [], []
    for k in range(6):
        ang = 0.03 * (k + 1)
        Rz = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0], [0, 0, 1]])
        cs = [Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, Rz @ np.asarray(c.R), np.asarray(c.t) - 0.01 * k,
                     c.znear, c.bg) for c in cams]
        sets.append(cs)
        pf.launch(cs)
        images.append(pf.image.clone())  # stream-ordered after the replay
    pf.launch()  # no cameras: the last set stays
    images.append(pf.image.clone())
    sets.append(sets[-1])
    torch.cuda.synchronize()
    assert pf.poll().flags == 0
    for k, (cs, img) in enumerate(zip(sets, images)):
        ref, _ = _eager(sc, cs, torch.zeros(pf.image.numel(), device="cuda"), opt)
        assert torch.equal(img, ref.image), k


def test_plan_autotune_and_cache(tmp_path, monkeypatch):
    print("[case] plan autotune + cache", flush=True)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("GES_AUTOTUNE_CACHE", str(cache))
    sc = workload("tiny")
    cams = _cams(sc)
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=True, autotune=True)
    o = pf.options()
    assert o.raster_tile in (8, 16) and (o.splat_tile_w, o.splat_tile_h) in ((8, 8), (16, 8), (16, 16))
    assert o.tile_queue in (0, 8 if o.raster_tile == 16 else 24)
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert (rec["raster_tile"], rec["splat_tile_w"], rec["splat_tile_h"], rec["tile_queue"]) == (
        o.raster_tile, o.splat_tile_w, o.splat_tile_h, o.tile_queue)
    assert rec["ms"] > 0
    # a second plan with the same key reads the cache and appends nothing
    pf2 = PlannedFrame(S, G, cams, backward=True, autotune=True)
    o2 = pf2.options()
    assert (o2.raster_tile, o2.splat_tile_w, o2.splat_tile_h, o2.tile_queue) == (
        o.raster_tile, o.splat_tile_w, o.splat_tile_h, o.tile_queue)
    assert len(cache.read_text().strip().splitlines()) == 1
    pf2.launch()
    torch.cuda.synchronize()
    for v in range(3):
        compare_view(pf2, Scene(sc.surfels, sc.gaussians, cams), v=v)


def test_plan_ring16_cameras_surfaces_300k():
    """The 16-camera ring of uneven resolutions, on the 300k/150k scene:
    one graph replay equals 16 separate single-view renders."""
    print("[case] plan, 16 mixed-resolution ring views", flush=True)
    sc = workload("surfaces_300k")
    cams = workload("ring16_1m", n_surfels=1, n_gaussians=1).cameras
    S, G = to_dev(sc)
    pf = PlannedFrame(S, G, cams, backward=False)
    pf.launch()
    torch.cuda.synchronize()
    r = Renderer(raster_tile=pf.options().raster_tile,
                 splat_tile=(pf.options().splat_tile_w, pf.options().splat_tile_h))
    for v in (0, 5, 10, 15):
        f = r.render(S, G, [cams[v]])
        assert torch.equal(pf.view("image", v), f.view("image", 0)), v
        assert torch.equal(pf.view("surfel_id", v), f.view("surfel_id", 0)), v
