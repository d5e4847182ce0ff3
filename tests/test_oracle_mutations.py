"""The oracle's pins must catch plausible mistakes in it.

Each case plants one mistake in the oracle (monkeypatched, CPU only) -- a
transposed rotation, a sign flip in the SH basis, a dropped dilation term, a
wrong eps dimension, a non-strict depth test, a wrong SH view direction (both
kinds, or the Gaussians' alone), the projected centre without its principal
point, a sign flip in the Jacobian's third column, a dropped Jacobian clamp,
the camera rotation transposed inside the projected covariance, depth ties
going to the larger index -- and asserts that at least one pin of the pinned
test modules fails against the mutated oracle.
"""
import math

import numpy as np
import pytest
import torch

import importlib

import oracle

R = importlib.import_module("oracle.render")
SH = importlib.import_module("oracle.sh")

import test_oracle_closed_forms as CF
import test_oracle_invariants as INV
import test_oracle_sh as TSH


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _surfel_pins():
    return [_fails(CF.test_fronto_parallel_circle)] + \
           [_fails(CF.test_tilted_disc_is_homography_conic, s) for s in range(4)]


def _gauss_pins():
    out = [_fails(CF.test_isotropic_gaussian_on_axis, *p) for p in
           [(0.9, 0.01, 3.0), (0.3, 0.004, 2.0), (0.99, 0.03, 4.0)]]
    out += [_fails(CF.test_depth_test_adaptive_eps, *p) for p in [(0.9, True), (1.1, False), (-0.5, True)]]
    out.append(_fails(CF.test_eps_constant_and_zero_knobs))
    out.append(_fails(INV.test_scalar_bruteforce_tiny))
    return out


def test_transposed_rotation_caught(monkeypatch):
    orig = R.quat_to_rot
    monkeypatch.setattr(R, "quat_to_rot", lambda q: orig(q).transpose(1, 2))
    assert any(_surfel_pins())


def test_sh_sign_flip_caught(monkeypatch):
    orig = SH.sh_basis

    def flipped(d, deg):
        y = orig(d, deg).clone()
        if y.shape[-1] > 3:
            y[..., 3] = -y[..., 3]  # drop the Condon-Shortley sign of Y_11
        return y
    monkeypatch.setattr(SH, "sh_basis", flipped)
    monkeypatch.setattr(TSH, "sh_basis", flipped)  # the name the pin calls
    assert _fails(TSH.test_textbook_closed_forms)


def test_sh_normalisation_caught(monkeypatch):
    monkeypatch.setattr(SH, "norm_const", lambda l, m: math.sqrt((2 * l + 1) / (4 * math.pi)))
    assert _fails(TSH.test_orthonormal_degree3) or _fails(TSH.test_textbook_closed_forms)


def test_dropped_dilation_caught(monkeypatch):
    orig = R.gaussian_projection
    monkeypatch.setattr(R, "gaussian_projection",
                        lambda G, cam, opts, params=None: orig(G, cam, R.Options(**{**opts.__dict__, "dilation": 0.0}),
                                                               params))
    assert any(_gauss_pins())


def test_eps_dimension_caught(monkeypatch):
    orig = R.gaussian_projection

    def wrong(G, cam, opts, params=None):
        out = orig(G, cam, opts, params)
        if opts.eps_const < 0:
            out["eps"] = out["eps"] * 3.0 / 2.0  # (5/2) sum s instead of (5/3) sum s
        return out
    monkeypatch.setattr(R, "gaussian_projection", wrong)
    assert any(_gauss_pins())


def test_non_strict_depth_test_caught(monkeypatch):
    orig = R.gaussian_pass

    def wrong(proj, cam, pix, depth_s, opts, band_rel=1e-4, **kw):
        p2 = dict(proj)
        p2["eps"] = proj["eps"] + 1e-12  # d <= D_s + eps instead of d < D_s + eps
        return orig(p2, cam, pix, depth_s, opts, band_rel, **kw)
    monkeypatch.setattr(R, "gaussian_pass", wrong)
    assert _fails(CF.test_depth_test_strict_at_boundary)


def test_reversed_view_direction_caught(monkeypatch):
    orig = R.sh_colour
    monkeypatch.setattr(R, "sh_colour", lambda sh, d, deg: orig(sh, -d, deg))
    assert _fails(INV.test_scalar_bruteforce_tiny)


def test_missing_principal_point_caught(monkeypatch):
    orig = R.gaussian_projection

    def wrong(G, cam, opts, params=None):
        out = orig(G, cam, opts, params)
        out["phat"] = out["phat"] - torch.tensor([cam.cx, cam.cy], dtype=out["phat"].dtype)
        return out
    monkeypatch.setattr(R, "gaussian_projection", wrong)
    assert any(_gauss_pins())


def test_gradient_pins_catch_wrong_colour_offset(monkeypatch):
    import test_oracle_grad as GR
    orig = SH.sh_colour
    monkeypatch.setattr(R, "sh_colour", lambda sh, d, deg: orig(sh, d, deg) * 1.01)
    assert _fails(GR.test_dsigma_closed_form) or _fails(GR.test_surfel_sh_dc_gradient)


# ----------------------------------------------------------------------------
# projection, view direction and tie rule (pinned by test_oracle_projection)

import test_oracle_projection as PROJ


def _projection_pins():
    return [_fails(PROJ.test_projected_covariance_is_fd_jacobian_off_axis, s) for s in (0, 1)] + \
           [_fails(PROJ.test_projected_covariance_clamped_outside_fov, p)
            for p in [(1.6, 0.3), (-0.4, -1.9), (2.2, 1.7)]]


def test_jacobian_third_column_sign_caught(monkeypatch):
    orig = R.ewa_jacobian

    def wrong(mu, cam):
        J = orig(mu, cam).clone()
        J[:, :, 2] = -J[:, :, 2]
        return J
    monkeypatch.setattr(R, "ewa_jacobian", wrong)
    assert any(_projection_pins())


def test_dropped_jacobian_clamp_caught(monkeypatch):
    def unclamped(mu, cam):
        z = mu[:, 2]
        zero = torch.zeros_like(z)
        return torch.stack([
            torch.stack([cam.fx / z, zero, -cam.fx * mu[:, 0] / (z * z)], dim=-1),
            torch.stack([zero, cam.fy / z, -cam.fy * mu[:, 1] / (z * z)], dim=-1)], dim=1)
    monkeypatch.setattr(R, "ewa_jacobian", unclamped)
    assert any(_projection_pins())


def test_transposed_camera_rotation_in_covariance_caught(monkeypatch):
    orig = R.projected_covariance
    monkeypatch.setattr(R, "projected_covariance", lambda J, Rc, s3, dil: orig(J, Rc.T, s3, dil))
    assert any(_projection_pins())


def test_flipped_gaussian_view_direction_caught(monkeypatch):
    orig = R.gaussian_projection

    def wrong(G, cam, opts, params=None):
        out = orig(G, cam, opts, params)
        sh = params["sh"] if params is not None else R._t(G.sh)
        mean = params["mean"] if params is not None else R._t(G.mean)
        out["colour"] = R.sh_colour(sh, -R.view_directions(mean, cam), R._degree(sh))
        return out
    monkeypatch.setattr(R, "gaussian_projection", wrong)
    assert any(_fails(PROJ.test_gaussian_view_direction_degree1, s) for s in (0, 1, 2))


def test_tie_to_larger_index_caught(monkeypatch):
    """The planted mistake: the z-buffer keeps the last of equal depths."""
    orig = R.surfel_pass

    def wrong(frames, cam, pix, opts, **kw):
        rev = {k: torch.flip(v, [0]) for k, v in frames.items()}
        out = orig(rev, cam, pix, opts, **kw)
        n = frames["mu"].shape[0]
        out["id"] = torch.where(out["id"] >= 0, n - 1 - out["id"], out["id"])
        return out
    monkeypatch.setattr(R, "surfel_pass", wrong)
    assert _fails(PROJ.test_coplanar_tie_goes_to_smaller_index, False) or \
        _fails(PROJ.test_coplanar_tie_goes_to_smaller_index, True)
