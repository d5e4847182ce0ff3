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
