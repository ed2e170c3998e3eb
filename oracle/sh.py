"""Real spherical harmonics for the view-dependent surfel colour (oracle;
test infrastructure only).

The paper gives each Gaussian an "appearance" (Section 3.1); as in the
Gaussian-splatting renderers it builds on, that appearance is read here as
real spherical-harmonic coefficients of degree D <= 3 per colour channel,
evaluated in the direction from the camera centre to the surfel centre:

    rgb = max(0, sum_{l<=D} sum_{m=-l..l} Y_lm(d) f_lm + 1/2)

Basis: the orthonormal real harmonics built from the complex ones that
include the Condon-Shortley phase,
    Y_{l,m>0} = sqrt(2) Re Y_l^m,  Y_{l,0} = Y_l^0,  Y_{l,m<0} = sqrt(2) Im Y_l^|m|,
stored l-major with m from -l to l (index l^2 + l + m).

Two independent constructions are given: ``sh_basis_scipy`` converts
scipy's complex harmonics (used to pin the other), and ``real_sh_basis``
evaluates the same functions differentiably with the associated-Legendre
three-term recurrence in z and the real/imaginary parts of (x + i y)^m.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def sh_coeff_count(degree: int) -> int:
    return (degree + 1) ** 2


def sh_basis_scipy(d: np.ndarray, degree: int) -> np.ndarray:
    """Real SH basis (M,K) at unit directions d (M,3) from scipy's complex
    harmonics (polar angle from +z, azimuth from +x)."""
    from scipy.special import sph_harm_y
    d = np.asarray(d, np.float64)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    out = np.zeros((d.shape[0], sh_coeff_count(degree)))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            k = l * l + l + m
            if m == 0:
                out[:, k] = sph_harm_y(l, 0, theta, phi).real
            elif m > 0:
                out[:, k] = math.sqrt(2.0) * sph_harm_y(l, m, theta, phi).real
            else:
                out[:, k] = math.sqrt(2.0) * sph_harm_y(l, -m, theta, phi).imag
    return out


def _legendre_reduced(z: torch.Tensor, degree: int):
    """P~_l^m(z) = P_l^m(z) / (1 - z^2)^(m/2) (Condon-Shortley phase
    included) for 0 <= m <= l <= degree, by the standard recurrences
      P~_m^m = (-1)^m (2m-1)!!,  P~_{m+1}^m = (2m+1) z P~_m^m,
      (l-m) P~_l^m = (2l-1) z P~_{l-1}^m - (l+m-1) P~_{l-2}^m."""
    P = {}
    for m in range(degree + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        P[(m, m)] = torch.full_like(z, ((-1.0) ** m) * dfact)
        if m + 1 <= degree:
            P[(m + 1, m)] = (2 * m + 1) * z * P[(m, m)]
        for l in range(m + 2, degree + 1):
            P[(l, m)] = ((2 * l - 1) * z * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH basis (..., K) at unit directions d (..., 3), differentiable."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    P = _legendre_reduced(z, degree)
    # (x + i y)^m = C_m + i S_m
    C = [torch.ones_like(x)]
    S = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        C.append(x * C[m - 1] - y * S[m - 1])
        S.append(x * S[m - 1] + y * C[m - 1])
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                cols.append(norm * P[(l, 0)])
            elif m > 0:
                cols.append(math.sqrt(2.0) * norm * P[(l, m)] * C[m])
            else:
                cols.append(math.sqrt(2.0) * norm * P[(l, am)] * S[am])
    return torch.stack(cols, dim=-1)


def sh_colour(sh: torch.Tensor, dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """rgb (M,3) = max(0, sum_k Y_k(d) f_k + 1/2) for coefficients sh (M,K,3)
    and unit directions dirs (M,3); K may exceed (degree+1)^2 (extra bands
    are ignored)."""
    K = sh_coeff_count(degree)
    Y = real_sh_basis(dirs, degree)                      # (M,K)
    raw = (Y.unsqueeze(-1) * sh[:, :K, :]).sum(dim=1) + 0.5
    return torch.clamp(raw, min=0.0), raw
