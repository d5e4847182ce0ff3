"""Pins of the oracle's spherical-harmonic basis (Sec. 3, Eq. 1).

The oracle builds the basis from Rodrigues' formula and the associated
Legendre functions; these tests hold it to facts fixed independently of that
construction: orthonormality on the sphere (exact product quadrature), a
textbook table of closed forms with the Condon-Shortley phase, the addition
theorem, and the degree-0 colour.
"""
import math

import numpy as np
import pytest
import torch

from oracle.sh import sh_basis, sh_colour

DT = torch.float64


def _quadrature(n_theta=8, n_phi=16):
    # Gauss-Legendre in cos(theta) (exact to degree 15) x uniform phi (exact
    # for trigonometric degree < 16): exact for products of degree <= 6.
    z, w = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * math.pi * np.arange(n_phi) / n_phi
    Z, PHI = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(w[:, None], n_phi, 1) * (2 * math.pi / n_phi)
    s = np.sqrt(1 - Z ** 2)
    dirs = np.stack([s * np.cos(PHI), s * np.sin(PHI), Z], -1).reshape(-1, 3)
    return torch.tensor(dirs, dtype=DT), torch.tensor(W.reshape(-1), dtype=DT)


def test_orthonormal_degree3():
    d, w = _quadrature()
    Y = sh_basis(d, 3)
    gram = (Y * w[:, None]).T @ Y
    assert torch.allclose(gram, torch.eye(16, dtype=DT), atol=1e-12)


def _rand_dirs(n=64, seed=0):
    g = np.random.default_rng(seed).standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return torch.tensor(g, dtype=DT)


def test_textbook_closed_forms():
    """Real SH with the Condon-Shortley phase, index k = l^2 + l + m."""
    d = _rand_dirs()
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    table = {
        0: torch.full_like(x, 0.5 / math.sqrt(pi)),
        1: -math.sqrt(3 / (4 * pi)) * y,                       # l=1, m=-1
        2: math.sqrt(3 / (4 * pi)) * z,                        # l=1, m=0
        3: -math.sqrt(3 / (4 * pi)) * x,                       # l=1, m=1
        4: 0.5 * math.sqrt(15 / pi) * x * y,                   # l=2, m=-2
        5: -0.5 * math.sqrt(15 / pi) * y * z,                  # l=2, m=-1
        6: 0.25 * math.sqrt(5 / pi) * (3 * z * z - 1),         # l=2, m=0
        7: -0.5 * math.sqrt(15 / pi) * x * z,                  # l=2, m=1
        8: 0.25 * math.sqrt(15 / pi) * (x * x - y * y),        # l=2, m=2
        9: -0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y),   # l=3, m=-3
        10: 0.5 * math.sqrt(105 / pi) * x * y * z,                       # l=3, m=-2
        11: -0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1),      # l=3, m=-1
        12: 0.25 * math.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),             # l=3, m=0
        13: -0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1),      # l=3, m=1
        14: 0.25 * math.sqrt(105 / pi) * (x * x - y * y) * z,            # l=3, m=2
        15: -0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y),  # l=3, m=3
    }
    Y = sh_basis(d, 3)
    for k, ref in table.items():
        assert torch.allclose(Y[:, k], ref, atol=1e-13), k


def test_addition_theorem():
    """sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a . b)."""
    a, b = _rand_dirs(32, 1), _rand_dirs(32, 2)
    Ya, Yb = sh_basis(a, 3), sh_basis(b, 3)
    c = (a * b).sum(-1).numpy()
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(-1).numpy()
        Pl = np.polynomial.legendre.legval(c, [0] * l + [1])
        assert np.allclose(lhs, (2 * l + 1) / (4 * math.pi) * Pl, atol=1e-13)


def test_degree0_colour_and_clamp():
    sh = torch.zeros((4, 3, 2), dtype=DT)
    sh[0, :, 0] = 0.3
    sh[0, :, 1] = -3.0
    d = _rand_dirs(2, 3)
    c0 = sh_colour(sh[:1], d, 0)
    assert torch.allclose(c0[:, 0], torch.full((3,), 0.5 + 0.28209479177387814 * 0.3, dtype=DT))
    assert torch.all(c0[:, 1] == 0)          # clamped at zero from below
    # degree 1 with zero higher coefficients equals degree 0
    assert torch.allclose(sh_colour(sh, d, 1), c0)
