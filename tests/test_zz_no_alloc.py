"""ges_scores_static (the allocation-free variant of ges_scores, whose
counters live in the library's own device array) against ges_scores,
through the C ABI: bit-identical results on two calls in a row, the second
on a smaller frame (fewer surfels, Gaussians and pixels), with and without
accumulate; a frame above its surfel limit is refused on the host."""
import numpy as np
import pytest
import torch

from paper_2504_17545_amd import Renderer, _lib
from synth import Camera, workload

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _out(n, m):
    return dict(cover=torch.full((n,), -7, dtype=torch.int32, device="cuda"),
                contrib=torch.full((m,), -1.0, dtype=torch.float32, device="cuda"),
                keep_surfel=torch.full((n,), 9, dtype=torch.uint8, device="cuda"),
                keep_gauss=torch.full((m,), 9, dtype=torch.uint8, device="cuda"))


def _call(fn, f, out, accumulate=False, cover_min=16, contrib_min=0.02):
    stream = torch.cuda.current_stream().cuda_stream
    fn(f.ctx, f.surfel_id, f.depth, f.accum, cover_min, contrib_min, accumulate, out["cover"], out["contrib"],
       out["keep_surfel"], out["keep_gauss"], stream)


def _frame(sc):
    S, G = to_dev(sc)
    r = Renderer()
    return r.render(S, G, sc.cameras), int(S["mean"].shape[1]), int(G["mean"].shape[1])


def _same(a, b, label):
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), (label, k)


def test_static_scores_match_workspace_scores_twice_second_smaller():
    print("[case] ges_scores_static vs ges_scores: tiny 128x128 (2000/1000), then 72x56 (600/400)", flush=True)
    big = workload("tiny")
    small = workload("tiny", n_surfels=600, n_gaussians=400)
    c = small.cameras[0]
    small.cameras = [Camera(72, 56, c.fx * 72 / 128, c.fy * 72 / 128, 36.0, 28.0, c.R, c.t)]
    for label, sc in (("first (larger)", big), ("second (smaller)", small)):
        f, n, m = _frame(sc)
        ref, got = _out(n, m), _out(n, m)
        _call(_lib.ges_scores, f, ref)
        _call(_lib.ges_scores_static, f, got)
        _same(ref, got, label)
        assert int(ref["cover"].sum()) == int((f.surfel_id >= 0).sum()), label
        # folded into the previous values: same again
        _call(_lib.ges_scores, f, ref, accumulate=True)
        _call(_lib.ges_scores_static, f, got, accumulate=True)
        _same(ref, got, label + ", accumulate")


def test_static_scores_multiview():
    print("[case] ges_scores_static vs ges_scores: 3 views", flush=True)
    sc = workload("tiny")
    c = sc.cameras[0]
    sc.cameras = [c, Camera(96, 80, 90.0, 90.0, 48.0, 40.0, c.R, c.t + np.array([0.2, 0.0, 0.0])),
                  Camera(64, 64, 60.0, 60.0, 32.0, 32.0, c.R, c.t + np.array([0.0, -0.1, 0.3]))]
    f, n, m = _frame(sc)
    ref, got = _out(n, m), _out(n, m)
    _call(_lib.ges_scores, f, ref)
    _call(_lib.ges_scores_static, f, got)
    _same(ref, got, "3 views")


def test_static_scores_refuse_more_surfels_than_the_scratch():
    print("[case] ges_scores_static: 4,194,305 surfels refused on the host", flush=True)
    n = (1 << 22) + 1
    sc = workload("tiny", n_gaussians=10)
    dev = "cuda"
    # surfels with a zero quaternion are culled at set-up: no list entries
    S = dict(mean=torch.zeros((3, n), device=dev), quat=torch.zeros((4, n), device=dev),
             scale=torch.ones((2, n), device=dev), sh=torch.zeros((n, 1, 3), device=dev))
    _, G = to_dev(sc)
    r = Renderer(surfel_pair_capacity=1 << 16)
    f = r.render(S, G, sc.cameras)
    got = _out(n, 10)
    with pytest.raises(_lib.GESError) as e:
        _call(_lib.ges_scores_static, f, got)
    assert e.value.status == _lib.GES_ERR_ARG
    torch.cuda.synchronize()
    assert int((got["cover"] != -7).sum()) == 0  # nothing was enqueued
    ref = _out(n, 10)
    _call(_lib.ges_scores, f, ref)
    torch.cuda.synchronize()
    assert int(ref["cover"].abs().sum()) == 0
