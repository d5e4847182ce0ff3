"""Real spherical harmonics for the FP64 oracle, built from their definition.

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

The paper colours each surfel and Gaussian with a spherical-harmonic function
Y(dir, SH) of the viewing direction (Sec. 3, Eq. 1) and says it builds on the
3DGS code base (Sec. 5); the coefficient convention taken here is that code
base's: real harmonics with the Condon-Shortley phase, coefficient index
k = l^2 + l + m.

Construction (no tabulated constants): the Legendre polynomial P_l comes from
Rodrigues' formula P_l(z) = 1/(2^l l!) d^l/dz^l (z^2 - 1)^l; the associated
function is P_l^m(z) = (-1)^m (1 - z^2)^(m/2) d^m P_l/dz^m; and on the unit
sphere (1 - z^2)^(m/2) cos(m phi) = Re (x + i y)^m, (1 - z^2)^(m/2) sin(m phi)
= Im (x + i y)^m.  With N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!):

  Y_l0      = N_l0 P_l(z)
  Y_lm, m>0 = sqrt(2) N_lm (-1)^m P_l^(m)(z) Re (x+iy)^m
  Y_lm, m<0 = sqrt(2) N_l|m| (-1)^|m| P_l^(|m|)(z) Im (x+iy)^|m|

where P_l^(m) is the m-th derivative of P_l.  Everything is a polynomial in
(x, y, z), so torch autograd differentiates it everywhere.
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import List

import torch


def _legendre_coeffs(l: int) -> List[Fraction]:
    """Exact coefficients c_k of P_l(z) = sum_k c_k z^k (Rodrigues' formula)."""
    # (z^2 - 1)^l = sum_j C(l, j) (-1)^(l-j) z^(2j)
    poly = [Fraction(0)] * (2 * l + 1)
    for j in range(l + 1):
        poly[2 * j] = Fraction(math.comb(l, j) * (-1) ** (l - j))
    for _ in range(l):  # differentiate l times
        poly = [poly[k] * k for k in range(1, len(poly))] or [Fraction(0)]
    scale = Fraction(1, 2 ** l * math.factorial(l))
    return [c * scale for c in poly]


def _derivative(coeffs: List[Fraction], m: int) -> List[Fraction]:
    for _ in range(m):
        coeffs = [coeffs[k] * k for k in range(1, len(coeffs))] or [Fraction(0)]
    return coeffs


def _polyval(coeffs: List[Fraction], z: torch.Tensor) -> torch.Tensor:
    out = torch.zeros_like(z)
    for c in reversed(coeffs):  # Horner
        out = out * z + float(c)
    return out


def norm_const(l: int, m: int) -> float:
    m = abs(m)
    return math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.factorial(l - m) / math.factorial(l + m))


def sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH basis at unit directions.

    dirs: [..., 3] float64 (x, y, z), assumed unit length.
    returns [..., (degree+1)^2] with index k = l^2 + l + m.
    """
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    # Re/Im of (x + i y)^m for m = 0..degree
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for _ in range(degree):
        r0, i0 = re[-1], im[-1]
        re.append(r0 * x - i0 * y)
        im.append(r0 * y + i0 * x)
    out = []
    for l in range(degree + 1):
        pl = _legendre_coeffs(l)
        for m in range(-l, l + 1):
            am = abs(m)
            dp = _polyval(_derivative(pl, am), z)
            if m == 0:
                out.append(norm_const(l, 0) * dp)
            else:
                c = math.sqrt(2.0) * norm_const(l, am) * (-1) ** am
                out.append(c * dp * (re[am] if m > 0 else im[am]))
    return torch.stack(out, dim=-1)


def sh_colour(sh: torch.Tensor, dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """Per-primitive colour from SH coefficients (Sec. 3, Eq. 1).

    sh:   [K][3][n] coefficients (K >= (degree+1)^2; extra ones unused)
    dirs: [n, 3] unit viewing directions
    returns [3][n]: max(0, 1/2 + sum_k SH_k Y_k(dir)) -- the 3DGS offset and
    lower clamp (no upper clamp).
    """
    k = (degree + 1) ** 2
    basis = sh_basis(dirs, degree)  # [n, k]
    raw = torch.einsum("kcn,nk->cn", sh[:k], basis)
    return torch.clamp_min(raw + 0.5, 0.0)
