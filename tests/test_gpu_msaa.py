"""GPU parity of the 4-sample surfel pass (options.surfel_samples = 4;
Sec. 5: the surfel pass supersampled 2x2, as Mip-GES renders it) against
the FP64 oracle, forward and backward, through the C ABI.

Per sample: the surfel id is bit-exact unless the sample's surfel decision
is within FP32 reach or its depth tie is below 1e-6 (then the GPU's surfel
must be a tied candidate).  Per pixel: C_s equals the mean of the oracle
colours of the GPU's sample surfels within 1e-5; D_s (the mean depth of the
hit samples) within the derived bound; C_G, W_G and the image within 1e-4
where no decision is in band; gradients as in the 1-sample tests."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_17545_amd import Renderer, _lib
from synth import Camera, Scene, permute_gaussians, workload

from gpu_util import BAND, TIE_REL, bands, check_grads, grads_np, sample_pixels, to_dev

pytestmark = pytest.mark.gpu

MS = oracle.Options(surfel_samples=4)


def _render(scene, **opts):
    S, G = to_dev(scene)
    r = Renderer(surfel_samples=4, **opts)
    f = r.render(S, G, scene.cameras)
    torch.cuda.synchronize()
    return f, r


def _compare(f, scene, v, pix, label, opts=MS):
    cam = scene.cameras[v]
    W, H = cam.width, cam.height
    out = oracle.render(scene, v, pix, opts=opts)
    sid = f.view("surfel_id", v).cpu().numpy()                       # [2H, 2W]
    i, j = pix % W, pix // W
    gsid = np.stack([sid[2 * j + b, 2 * i + a] for a, b in ((0, 0), (1, 0), (0, 1), (1, 1))]).astype(np.int64)
    osid = out["sample_id"].numpy()
    sgap = out["sample_gap"].numpy()
    samb = out["sample_amb"].numpy() < BAND
    stie = sgap < TIE_REL
    bad = (~samb) & (~stie) & (gsid != osid)
    assert not bad.any(), f"{label}: sample id mismatch at {int(bad.sum())} samples"
    for k in range(4):
        cands = out[f"sample_cands{k}"].numpy()
        for q in np.nonzero(stie[k] & ~samb[k])[0]:
            assert gsid[k, q] in cands[q], (label, k, q)
    # C_s: mean of the oracle colours of the GPU's sample surfels
    scol = out["surfel_colour"].numpy()
    bg = np.asarray(cam.bg, dtype=np.float64)[:, None]
    ecs = sum(np.where(gsid[k][None, :] >= 0, scol[:, np.clip(gsid[k], 0, None)] if scol.shape[1] else bg, bg)
              for k in range(4)) / 4
    gcs = f.view("color_s", v).cpu().numpy().reshape(3, -1)[:, pix].astype(np.float64)
    any_amb = samb.any(0)
    err_cs = np.abs(gcs[:, ~any_amb] - ecs[:, ~any_amb]).max(initial=0.0)
    assert err_cs <= 1e-5, (label, err_cs)
    # D_s: mean depth of the hit samples
    gd = f.view("depth", v).cpu().numpy().reshape(-1)[pix].astype(np.float64)
    od = out["depth"].numpy()
    hit = np.isfinite(od) & ~any_amb & ~stie.any(0)
    assert np.array_equal(np.isinf(gd[~any_amb & ~stie.any(0)]), np.isinf(od[~any_amb & ~stie.any(0)]))
    rel = np.abs(gd[hit] - od[hit]) / od[hit]
    bound = BAND * out["kz_win"].numpy()[hit]
    assert (rel <= bound).all(), (label, float((rel / bound).max()))
    # pass 2 and the composite where nothing is in band
    b = bands(out)
    good = b["safe"]
    gacc = f.view("accum", v).cpu().numpy().reshape(4, -1)[:, pix].astype(np.float64)
    gimg = f.view("image", v).cpu().numpy().reshape(3, -1)[:, pix].astype(np.float64)
    err_acc = max(np.abs(gacc[:3, good] - out["cg"].numpy()[:, good]).max(initial=0.0),
                  np.abs(gacc[3, good] - out["wg"].numpy()[good]).max(initial=0.0))
    eimg = (ecs + out["cg"].numpy()) / (1.0 + out["wg"].numpy())
    err_img = np.abs(gimg[:, good] - eimg[:, good]).max(initial=0.0)
    partial = int(((osid >= 0).sum(0) % 4 != 0).sum())
    print(f"[msaa] {label}: {len(pix)} pixels, {partial} partly covered, sample ties {int(stie.sum())}, "
          f"sample bands {int(samb.sum())}, err C_s {err_cs:.2e}, accum {err_acc:.2e}, image {err_img:.2e}",
          flush=True)
    assert err_acc <= 1e-4 and err_img <= 1e-4, (label, err_acc, err_img)
    return partial


def test_tiny_msaa_forward_vs_oracle():
    print("[case] tiny 128x128, 4 samples per pixel: forward", flush=True)
    sc = workload("tiny")
    f, _ = _render(sc)
    assert f.surfel_id.numel() == 4 * 128 * 128
    assert _compare(f, sc, 0, np.arange(128 * 128), "tiny") > 100


def test_msaa_multiview_and_ragged():
    print("[case] 4 samples, 3 views incl. a ragged 65x33", flush=True)
    sc = workload("tiny")
    c = sc.cameras[0]
    cams = [c, Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
            Camera(65, 33, 60.0, 60.0, 32.5, 16.5, c.R, c.t + np.array([0.0, -0.1, 0.3]))]
    full = Scene(sc.surfels, sc.gaussians, cams)
    f, _ = _render(full)
    for v in range(3):
        _compare(f, full, v, np.arange(cams[v].width * cams[v].height), f"view {v}")


def test_msaa_tile_shapes_and_permutation_bitwise():
    print("[case] 4 samples: raster 8 / 16, splat 8x8, Gaussian permutation", flush=True)
    sc = workload("tiny")
    a, _ = _render(sc, raster_tile=8)
    for kw in (dict(raster_tile=16), dict(raster_tile=16, splat_tile=(8, 8)), dict(raster_tile=16, tile_queue=4)):
        b, _ = _render(sc, **kw)
        for name in ("surfel_id", "depth", "color_s", "image", "accum"):
            assert torch.equal(getattr(a, name), getattr(b, name)), (kw, name)
    G2, _ = permute_gaussians(sc.gaussians, 3)
    c, _ = _render(Scene(sc.surfels, G2, sc.cameras), raster_tile=8)
    assert torch.equal(a.image, c.image) and torch.equal(a.accum, c.accum)


def test_msaa_surfaces_300k_sampled():
    print("[case] 300k scene 1600x1060, 4 samples: sampled pixels", flush=True)
    sc = workload("surfaces_300k")
    f, _ = _render(sc, raster_tile=16)
    _compare(f, sc, 0, sample_pixels(sc.cameras[0], 96, 31), "300k sampled")


def test_mip_ges_1080p_workload_sampled():
    """The Mip-GES set-up at the benchmark's workload (1M surfels, 500k
    Gaussians, 1920x1080, raster and splat tiles 16x16): 4 surfel samples,
    the world-space filter sized from the view (oracle.mip_filter3d) and the
    screen-space filter 0.1, the whole frame rendered, sampled pixels
    against the oracle with the same options."""
    print("[case] surfaces_1m_1080p, 4 samples + both Mip filters: sampled pixels", flush=True)
    sc = workload("surfaces_1m_1080p")
    sc.gaussians.filter3d = oracle.mip_filter3d(sc.gaussians, list(sc.cameras))
    f, _ = _render(sc, raster_tile=16, splat_tile=(16, 16), mip_2d=0.1)
    st = f.status
    assert st.flags == 0
    _compare(f, sc, 0, sample_pixels(sc.cameras[0], 96, 37), "1080p Mip-GES",
             opts=oracle.Options(surfel_samples=4, mip_2d=0.1))


def test_msaa_backward_vs_oracle():
    print("[case] tiny, 4 samples: backward vs oracle autograd", flush=True)
    sc = workload("tiny")
    cam = sc.cameras[0]
    out = oracle.render(sc, opts=MS)
    d = np.random.default_rng(14).standard_normal((3, cam.width * cam.height))
    d[:, ~bands(out)["safe"]] = 0.0
    f, r = _render(sc)
    g = grads_np(r.backward(f, torch.as_tensor(d.astype(np.float32).reshape(-1), device="cuda")))
    ref = oracle.gradients(sc, d, np.arange(cam.width * cam.height), opts=MS)
    check_grads(g, ref, "tiny 4 samples")


def test_msaa_scores_and_geometry_refused():
    print("[case] 4 samples: scores and geometry are refused", flush=True)
    sc = workload("tiny")
    f, r = _render(sc)
    with pytest.raises(_lib.GESError) as e:
        r.scores(f)
    assert e.value.status == _lib.GES_ERR_UNSUPPORTED
    with pytest.raises(_lib.GESError) as e:
        r.geometry(f)
    assert e.value.status == _lib.GES_ERR_UNSUPPORTED
