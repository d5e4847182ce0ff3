"""GPU parity of ges_scores (pruning scores: the covering score n_{i,j} of
Sec. 4.1 and the contribution score s_{i,j} of Sec. 4.2, Eq. 9) against the
FP64 oracle's plain definitions, through the C ABI.

Bars: covering counts bit-exact for every surfel the oracle does not flag
(a surfel winning or tying for a pixel whose surfel decision lies inside its
FP32 band); contribution scores within 1e-4 absolute (the image tolerance:
the score is a quotient of the same alpha and W_G) for every Gaussian the
oracle does not flag; keep flags equal to the thresholded GPU scores.
Scores over several views are the maxima over views; `accumulate` folds a
frame into earlier scores; results are reproducible and the Gaussian scores
follow a permutation of the Gaussian array exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_17545_amd import Renderer, _lib
from synth import Camera, Scene, permute_gaussians, workload

from gpu_util import bands, to_dev

pytestmark = pytest.mark.gpu

TOL_CONTRIB = 1e-4


def _gpu_scores(scene, cams=None, cover_min=16, contrib_min=0.02, **opts):
    S, G = to_dev(scene)
    r = Renderer(**opts)
    f = r.render(S, G, cams if cams is not None else scene.cameras)
    sc = r.scores(f, cover_min, contrib_min)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in sc.items()}, (r, f, S, G)


def _oracle_scores(scene, views):
    cover = contrib = None
    sb = gb = None
    for v in views:
        o = oracle.scores(scene, v)
        c, s = o["cover"].numpy(), o["contrib"].numpy()
        cover = c if cover is None else np.maximum(cover, c)
        contrib = s if contrib is None else np.maximum(contrib, s)
        sb = o["surfel_band"].numpy() if sb is None else sb | o["surfel_band"].numpy()
        gb = o["gauss_band"].numpy() if gb is None else gb | o["gauss_band"].numpy()
    return cover, contrib, sb, gb


def _compare(g, cover, contrib, sb, gb, label, cover_min=16, contrib_min=0.02):
    gc, gs = g["cover"].astype(np.int64), g["contrib"].astype(np.float64)
    bad = (~sb) & (gc != cover)
    assert not bad.any(), f"{label}: covering counts differ for {int(bad.sum())} surfels, e.g. " \
                          f"{np.nonzero(bad)[0][:5]} gpu={gc[bad][:5]} oracle={cover[bad][:5]}"
    err = np.abs(gs - contrib)[~gb]
    worst = float(err.max(initial=0.0))
    assert worst <= TOL_CONTRIB, f"{label}: contribution score error {worst}"
    # flags are the thresholded GPU scores
    assert np.array_equal(g["keep_surfel"].astype(bool), g["cover"] >= cover_min)
    assert np.array_equal(g["keep_gauss"].astype(bool), g["contrib"] >= np.float32(contrib_min))
    # and agree with the oracle's wherever the oracle's score is clear of the threshold
    clear_g = (~gb) & (np.abs(contrib - contrib_min) > TOL_CONTRIB)
    assert np.array_equal(g["keep_gauss"].astype(bool)[clear_g], (contrib >= contrib_min)[clear_g])
    print(f"[scores] {label}: {int((cover > 0).sum())} surfels cover a pixel ({int(sb.sum())} in the band), "
          f"{int((contrib > 0).sum())} Gaussians contribute ({int(gb.sum())} in the band), "
          f"max |contrib err| {worst:.2e}", flush=True)


def test_tiny_scores_vs_oracle():
    print("[case] tiny 128x128 scores", flush=True)
    sc = workload("tiny")
    g, _ = _gpu_scores(sc)
    _compare(g, *_oracle_scores(sc, [0]), "tiny")


@pytest.mark.parametrize("rt,splat", [(16, (8, 8)), (8, (16, 8))])
def test_tiny_scores_other_tiles_identical(rt, splat):
    print(f"[case] tiny scores, raster {rt}, splat {splat}", flush=True)
    sc = workload("tiny")
    a, _ = _gpu_scores(sc)
    b, _ = _gpu_scores(sc, raster_tile=rt, splat_tile=splat)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_small_surface_scene_scores_vs_oracle():
    """A reduced surface scene (8k surfels on 64 surfaces, 4k Gaussians) seen
    by a 200x132 camera of the same ring: several tiles, ragged edges,
    coplanar patches."""
    print("[case] surfaces 8k/4k, 200x132 scores", flush=True)
    sc = workload("surfaces_300k", n_surfels=8000, n_gaussians=4000)
    c = sc.cameras[0]
    s = 200 / c.width
    sc.cameras = [Camera(200, 132, c.fx * s, c.fy * s, 100.0, 66.0, c.R, c.t)]
    g, _ = _gpu_scores(sc, cover_min=4)
    _compare(g, *_oracle_scores(sc, [0]), "surfaces 8k", cover_min=4)


def test_multiview_scores_are_max_over_views_and_accumulate():
    print("[case] tiny, 3 views: max over views; accumulate", flush=True)
    sc = workload("tiny")
    c = sc.cameras[0]
    cams = [c, Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
            Camera(64, 64, 60.0, 60.0, 32.0, 32.0, c.R, c.t + np.array([0.0, -0.1, 0.3]))]
    full = Scene(sc.surfels, sc.gaussians, cams)
    g, (r, f, S, G) = _gpu_scores(full)
    _compare(g, *_oracle_scores(full, [0, 1, 2]), "3 views")
    # the same three views one frame at a time, folded with accumulate
    acc = None
    for cam in cams:
        fv = r.render(S, G, [cam])
        acc = r.scores(fv, 16, 0.02, into=acc)
    torch.cuda.synchronize()
    for k in g:
        assert np.array_equal(acc[k].cpu().numpy(), g[k]), k


def test_scores_reproducible_and_follow_gaussian_permutation():
    print("[case] tiny scores: repeat, Gaussian permutation", flush=True)
    sc = workload("tiny")
    a, (r, f, S, G) = _gpu_scores(sc)
    b = {k: v.cpu().numpy() for k, v in r.scores(f).items()}
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    G2, perm = permute_gaussians(sc.gaussians, 31)
    c, _ = _gpu_scores(Scene(sc.surfels, G2, sc.cameras))
    assert np.array_equal(c["contrib"], a["contrib"][perm])
    assert np.array_equal(c["cover"], a["cover"])


def test_scores_empty_sets_and_state_errors():
    print("[case] scores: no Gaussians / no surfels; call order", flush=True)
    from synth import empty_gaussians, empty_surfels
    sc = workload("tiny")
    g, _ = _gpu_scores(Scene(sc.surfels, empty_gaussians(), sc.cameras))
    assert g["contrib"].size == 0
    cov, _, sb, _ = _oracle_scores(Scene(sc.surfels, empty_gaussians(), sc.cameras), [0])
    assert np.array_equal(g["cover"][~sb], cov[~sb])
    g, _ = _gpu_scores(Scene(empty_surfels(), sc.gaussians, sc.cameras))
    assert g["cover"].size == 0
    _, con, _, gb = _oracle_scores(Scene(empty_surfels(), sc.gaussians, sc.cameras), [0])
    assert np.abs(g["contrib"] - con)[~gb].max() <= TOL_CONTRIB
    # a context that has not splatted cannot score
    ctx = _lib.Context(0)
    z = torch.zeros(4, device="cuda")
    with pytest.raises(_lib.GESError) as e:
        _lib.ges_scores(ctx, z, z, z, 16, 0.02, False, z, z, None, None, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == _lib.GES_ERR_STATE


def test_surfaces_1m_1080p_scores_properties_and_samples():
    """The benchmark workload at full size: the covering counts sum to the
    covered pixels and equal a recount of the id map; the contribution of
    sampled Gaussians equals the oracle's maximum over their own pixel boxes
    (C_G, W_G and D_s from the oracle at those pixels)."""
    print("[case] 1M surfels 1080p: scores", flush=True)
    sc = workload("surfaces_1m_1080p")
    g, (r, f, S, G) = _gpu_scores(sc)
    sid = f.surfel_id.cpu().numpy().astype(np.int64)
    cnt = np.bincount(sid[sid >= 0], minlength=sc.surfels.n)
    assert np.array_equal(g["cover"], cnt)
    assert int(g["cover"].sum()) == int((sid >= 0).sum())
    # sampled Gaussians with a positive score and a small footprint
    cam = sc.cameras[0]
    proj = oracle.gaussian_projection(sc.gaussians, oracle.Cam(cam), oracle.Options())
    pos = np.nonzero(g["contrib"] > 0)[0]
    rng = np.random.default_rng(7)
    picks = rng.choice(pos, size=min(6, pos.size), replace=False)
    cmax = proj["colour"].detach().numpy().max(0)
    for i in picks:
        px, py = proj["phat"][i].detach().numpy()
        k = 2 * np.log(float(proj["opacity"][i]) * 255.0)
        cov = proj["cov2"][i].detach().numpy()
        ex, ey = np.sqrt(k * cov[0, 0]) + 1, np.sqrt(k * cov[1, 1]) + 1
        rect = (max(0, int(px - ex)), max(0, int(py - ey)), min(cam.width, int(px + ex) + 1),
                min(cam.height, int(py + ey) + 1))
        pix = oracle.rect_pixels(cam, rect).numpy()
        out = oracle.render(sc, 0, pix)
        x = np.stack([pix % cam.width + 0.5, pix // cam.width + 0.5], 1)
        d = x - proj["phat"][i].detach().numpy()
        con = proj["conic"][i].detach().numpy()
        q = con[0] * d[:, 0] ** 2 + 2 * con[1] * d[:, 0] * d[:, 1] + con[2] * d[:, 1] ** 2
        al = float(proj["opacity"][i]) * np.exp(-0.5 * q)
        dep = out["depth"].numpy()
        keep = (al >= 1 / 255) & (float(proj["depth"][i]) < dep + float(proj["eps"][i]))
        e = cmax[i] * np.max(np.where(keep, al / (1.0 + out["wg"].numpy()), 0.0), initial=0.0)
        amb = ~bands(out)["safe"]
        if (amb & (al >= 1 / 255 * (1 - 1e-4))).any():
            continue  # a decision at one of its pixels is within FP32 reach
        assert abs(float(g["contrib"][i]) - e) <= TOL_CONTRIB, (i, float(g["contrib"][i]), e)
    print(f"[scores] 1080p: {int((g['cover'] > 0).sum())} surfels cover pixels, "
          f"{int((g['contrib'] > 0).sum())} Gaussians contribute, "
          f"{int(g['keep_surfel'].sum())} / {int(g['keep_gauss'].sum())} kept", flush=True)
