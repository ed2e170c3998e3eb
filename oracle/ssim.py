"""Masked structural similarity: the D-SSIM part of the photometric loss of
Eq. 2 and the masked evaluation metrics (oracle; test infrastructure only).

Eq. 2 applies the 3DGS photometric loss to the masked images M*R and M*I.
That loss is (1 - lambda) L1 + lambda (1 - SSIM) with lambda = 0.2; Section 5.1
keeps the 3DGS coefficients.  The readings taken here (listed with reasons
in the design notes):

  window   11 x 11 Gaussian, sigma = 1.5, normalised to sum 1 (separable:
           the outer product of the normalised 1-D Gaussian with itself)
  filter   correlation with zero padding of 5 pixels, output the image size,
           each colour channel separately
  maps     mu_x = G*x, mu_y = G*y, s_x = G*x^2 - mu_x^2, s_y = G*y^2 - mu_y^2,
           s_xy = G*(x y) - mu_x mu_y
           SSIM(p) = (2 mu_x mu_y + C1)(2 s_xy + C2)
                     / ((mu_x^2 + mu_y^2 + C1)(s_x + s_y + C2)),
           C1 = 0.01^2, C2 = 0.03^2
  SSIM_v   mean of SSIM(p) over the 3 channels and all pixels of view v
  D-SSIM   L_s = (1/V) sum_v w_s (1 - SSIM_v), on x = M R, y = M I
  PSNR_v   -10 log10(mean over channels and pixels of (M R - M I)^2)

Float64 torch; conv2d is the filtering primitive; gradients by autograd.
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_1d64(size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    """Normalised 1-D Gaussian taps g[k] ~ exp(-(k - size//2)^2 / (2 sigma^2))."""
    k = torch.arange(size, dtype=torch.float64) - (size // 2)
    g = torch.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def window_2d64(size: int = WINDOW, sigma: float = SIGMA) -> torch.Tensor:
    g = gaussian_1d64(size, sigma)
    return torch.outer(g, g)


def _filter(img: torch.Tensor) -> torch.Tensor:
    """(3,H,W) -> (3,H,W): per-channel correlation with the window, zero padding."""
    w = window_2d64().to(img.dtype)[None, None].expand(3, 1, WINDOW, WINDOW).contiguous()
    return F.conv2d(img[None], w, padding=WINDOW // 2, groups=3)[0]


def ssim_map64(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Per-pixel, per-channel SSIM of two (3,H,W) float64 images."""
    mx, my = _filter(x), _filter(y)
    sx = _filter(x * x) - mx * mx
    sy = _filter(y * y) - my * my
    sxy = _filter(x * y) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))


def _t(a):
    return a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, np.float64))


def masked_ssim64(color, target, mask) -> torch.Tensor:
    """SSIM_v of M*R and M*I; color, target (3,H,W), mask (H,W)."""
    m = _t(mask).to(torch.float64)[None]
    return ssim_map64(m * _t(color), m * _t(target)).mean()


def masked_psnr64(color, target, mask) -> float:
    m = np.asarray(mask, np.float64)[None]
    d = m * np.asarray(color, np.float64) - m * np.asarray(target, np.float64)
    mse = float((d * d).mean())
    return math.inf if mse == 0.0 else -10.0 * math.log10(mse)


def dssim_loss64(colors, targets, masks, w_s: float):
    """Per-view SSIM, the D-SSIM total (1/V) sum_v w_s (1 - SSIM_v) and its
    gradient with respect to every colour image (numpy float64)."""
    V = len(colors)
    cs = [torch.tensor(np.asarray(c, np.float64), requires_grad=True) for c in colors]
    per_view, total = [], 0.0
    for v in range(V):
        s = masked_ssim64(cs[v], targets[v], masks[v])
        per_view.append(float(s.detach()))
        total = total + w_s * (1.0 - s)
    total = total / V
    total.backward()
    return {"ssim": per_view, "total": float(total.detach()), "grads": [c.grad.numpy() for c in cs]}
