"""Every SH degree the library builds kernels for (0..3: K = 1, 4, 9, 16
coefficients per channel; the default workloads use 3) against the FP64
oracle: the full tiny frame forward, and the backward's gradients under a
random upstream gradient, with both primitive kinds' SH truncated to the
degree (Eq. 1 with fewer bands)."""
import numpy as np
import pytest

import oracle
from synth import workload

from gpu_util import compare_view, render
from test_gpu_backward import _check, _gpu_grads, _safe_mask

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_tiny_sh_degree_forward_and_backward(degree):
    print(f"[case] tiny 128x128, SH degree {degree}: forward + backward vs oracle", flush=True)
    sc = workload("tiny")
    K = (degree + 1) ** 2
    sc.surfels.sh = np.ascontiguousarray(sc.surfels.sh[:K])
    sc.gaussians.sh = np.ascontiguousarray(sc.gaussians.sh[:K])
    f = render(sc)
    st = compare_view(f, sc)
    assert st["hit_frac"] > 0.3
    cam = sc.cameras[0]
    out = oracle.render(sc)
    d = np.random.default_rng(40 + degree).standard_normal((3, cam.width * cam.height))
    d[:, ~_safe_mask(out)] = 0.0
    gpu, _ = _gpu_grads(sc, d)
    assert gpu["sh"].shape[0] == K and gpu["surfel_sh"].shape[0] == K
    ref = oracle.gradients(sc, d, np.arange(cam.width * cam.height))
    _check(gpu, ref, f"SH degree {degree}")


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_tiny_sh_degree_crop_backward(degree):
    """An upstream gradient on a 20x20 crop only: most waves of the surfel
    chain rule then hold a few surfels with a gradient among many without,
    and every surfel and Gaussian the crop does not reach must get exactly
    zero (the tolerance's floor is zero where the oracle's gradient is)."""
    print(f"[case] tiny 128x128, SH degree {degree}: crop backward vs oracle", flush=True)
    sc = workload("tiny")
    K = (degree + 1) ** 2
    sc.surfels.sh = np.ascontiguousarray(sc.surfels.sh[:K])
    sc.gaussians.sh = np.ascontiguousarray(sc.gaussians.sh[:K])
    cam = sc.cameras[0]
    W, H = cam.width, cam.height
    out = oracle.render(sc)
    crop = np.zeros((H, W), bool)
    crop[50:70, 40:60] = True
    crop = crop.reshape(-1) & _safe_mask(out)
    d = np.zeros((3, W * H))
    d[:, crop] = np.random.default_rng(70 + degree).standard_normal((3, int(crop.sum())))
    gpu, _ = _gpu_grads(sc, d)
    idx = np.nonzero(crop)[0]
    ref = oracle.gradients(sc, d[:, idx], idx)
    reached = int((np.abs(ref["surfel_sh"]).sum((0, 1)) > 0).sum())
    assert 5 < reached < sc.surfels.n // 4, reached
    _check(gpu, ref, f"SH degree {degree}, crop")
