"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/ges.h declares, and rejects bad arguments on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2504_17545_amd import _lib
from paper_2504_17545_amd._lib import GESError
from synth import Camera, workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ges.h")).read()
    return sorted(set(re.findall(r"\b(ges_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    names = _declared()
    assert "ges_project" in names and "ges_backward" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.exported_symbols())


def test_probe_library_exports_its_header():
    """The measurement probes (include/ges_probe.h) live in their own library."""
    src = open(os.path.join(ROOT, "include", "ges_probe.h")).read()
    names = sorted(set(re.findall(r"\b(ges_probe_[a-z_]+)\s*\(", src)))
    assert names == ["ges_probe_atomics", "ges_probe_copy"]
    lib = C.CDLL(os.path.join(ROOT, "paper_2504_17545_amd", "lib", "libges_probe.so"))
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # sizes implied by the header's field lists (natural alignment)
    assert C.sizeof(_lib.ges_camera) == 4 * (2 + 4 + 9 + 3 + 1 + 3)
    assert C.sizeof(_lib.ges_surfels) == 8 + 4 + 4 + 4 * 8
    assert C.sizeof(_lib.ges_gaussians) == 8 + 4 + 4 + 6 * 8
    assert C.sizeof(_lib.ges_options) == 6 * 4 + 4 * 4 + 2 * 8 + 2 * 4
    assert C.sizeof(_lib.ges_run_status) == 4 + 4 + 8 * 8
    assert C.sizeof(_lib.ges_gradients) == 6 * 8


def test_default_options():
    o = _lib.options()
    assert abs(o.surfel_radius - np.sqrt(2 * np.log(255))) < 1e-6
    assert o.eps_factor == 5.0 and o.eps_const < 0
    assert abs(o.alpha_min - 1 / 255) < 1e-9
    assert abs(o.dilation - 0.3) < 1e-7 and o.w_s == 1.0
    assert (o.raster_tile, o.splat_tile_w, o.splat_tile_h) == (8, 16, 16)


def _cam(**kw):
    c = workload("tiny").cameras[0]
    d = dict(width=c.width, height=c.height, fx=c.fx, fy=c.fy, cx=c.cx, cy=c.cy, R=c.R, t=c.t)
    d.update(kw)
    return Camera(**d)


@pytest.mark.parametrize("bad", [dict(width=0), dict(height=20000), dict(fx=0.0), dict(fy=-1.0),
                                 dict(cx=float("nan")), dict(znear=0.0),
                                 dict(R=np.full((3, 3), np.inf))])
def test_bad_camera_rejected(bad):
    with pytest.raises(GESError) as e:
        _lib.ges_workspace_query([_cam(**bad)], 10, 10, _lib.options())
    assert e.value.status == _lib.GES_ERR_ARG


def test_bad_counts_and_options():
    cam = [_cam()]
    with pytest.raises(GESError):
        _lib.ges_workspace_query(cam, -1, 0, _lib.options())
    with pytest.raises(GESError) as e:
        _lib.ges_workspace_query(cam, 1, 1, _lib.options(raster_tile=4))
    assert e.value.status == _lib.GES_ERR_UNSUPPORTED
    with pytest.raises(GESError) as e:
        _lib.ges_workspace_query(cam, 1, 1, _lib.options(splat_tile=(8, 16)))
    assert e.value.status == _lib.GES_ERR_UNSUPPORTED
    with pytest.raises(GESError):
        _lib.ges_workspace_query(cam, 1, 1, _lib.options(alpha_min=0.0))
    with pytest.raises(GESError):
        _lib.ges_workspace_query(cam, 1, 1, _lib.options(w_s=0.0))
    with pytest.raises(GESError):
        _lib.ges_workspace_query([], 1, 1, _lib.options())


def test_workspace_grows_with_problem():
    cam = [_cam()]
    o = _lib.options()
    a = _lib.ges_workspace_query(cam, 100, 100, o)
    b = _lib.ges_workspace_query(cam, 1000, 100, o)
    c = _lib.ges_workspace_query(cam * 3, 100, 100, o)
    d = _lib.ges_workspace_query(cam, 0, 0, o)
    assert d < a < b and a < c
    o2 = _lib.options(gauss_pair_capacity=10_000_000)
    assert _lib.ges_workspace_query(cam, 100, 100, o2) > 10_000_000 * 4 * 11


def test_total_pixels_mixed_views():
    sc = workload("ring16_1m", n_surfels=100, n_gaussians=100)
    assert _lib.ges_total_pixels(sc.cameras) == 4 * (640 * 360 + 1280 * 720 + 1600 * 1060 + 1920 * 1080)


def test_calls_without_context_fail_cleanly():
    lib = _lib.lib()
    assert lib.ges_raster_surfels(None, None, None, None, None) == _lib.GES_ERR_ARG
    assert lib.ges_backward(None, None, None, None, None, None, None, None) == _lib.GES_ERR_ARG
    assert b"NULL" in lib.ges_last_error()
    assert lib.ges_context_destroy(None) == _lib.GES_OK


def test_sh_layout_checked_when_descriptors_are_built():
    """SH is per primitive, [n][K][3] and [m][K][3]; the binding refuses the
    coefficient-major [K][3][n] and a K that is not a square before any call."""
    import torch
    n, m, K = 5, 7, 16
    z = torch.zeros
    sd = _lib.make_surfels(z(3, n), z(4, n), z(2, n), z(n, K, 3))
    assert sd.n == n and sd.sh_degree == 3
    gd = _lib.make_gaussians(z(3, m), z(4, m), z(3, m), z(m), z(m, K, 3))
    assert gd.m == m and gd.sh_degree == 3
    assert _lib.make_gaussians(z(3, m), z(4, m), z(3, m), z(m), z(m, 1, 3)).sh_degree == 0
    with pytest.raises(ValueError):
        _lib.make_surfels(z(3, n), z(4, n), z(2, n), z(K, 3, n))
    with pytest.raises(ValueError):
        _lib.make_gaussians(z(3, m), z(4, m), z(3, m), z(m), z(K, 3, m))
    with pytest.raises(ValueError):
        _lib.make_gaussians(z(3, m), z(4, m), z(3, m), z(m), z(m, 5, 3))


def test_translucent_and_2d_gaussian_arguments_on_the_host():
    """The translucent entry points and the 2D-Gaussian descriptor: argument
    checks that need no device."""
    import torch
    cam = [_cam()]
    o = _lib.options()
    a = _lib.ges_translucent_workspace_query(cam, 100, o)
    assert _lib.ges_translucent_workspace_query(cam, 1000, o) > a > _lib.ges_translucent_workspace_query(cam, 0, o)
    with pytest.raises(GESError):
        _lib.ges_translucent_workspace_query(cam, -1, o)
    with pytest.raises(GESError) as e:
        _lib.ges_translucent_workspace_query(cam, 10, _lib.options(raster_tile=4))
    assert e.value.status == _lib.GES_ERR_UNSUPPORTED
    lib = _lib.lib()
    assert lib.ges_translucent_render(None, None, 0, None, None, 0, None, None, 0, None, None) == _lib.GES_ERR_ARG
    assert lib.ges_translucent_backward(None, None, None, None) == _lib.GES_ERR_ARG
    z = torch.zeros
    m = 6
    g2 = _lib.make_gaussians(z(3, m), z(4, m), z(2, m), z(m), z(m, 4, 3))
    g3 = _lib.make_gaussians(z(3, m), z(4, m), z(3, m), z(m), z(m, 4, 3))
    assert g2.dims == 2 and g3.dims == 3 and g2.sh_degree == 1
