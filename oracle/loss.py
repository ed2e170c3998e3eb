"""Losses of the object-centric method (oracle; test infrastructure only).

Background loss, Eq. 1:  L_b = (1 / (h w)) sum_p A(p) (1 - M(p)), the mean of
the accumulated alpha over the pixels outside the object mask.

Masked photometric loss, Eq. 2: the photometric loss of the rendered and the
target image, both multiplied by the mask.  The hot path uses its L1 part,
normalised per channel and pixel: (1 / (3 h w)) sum_{p,ch} |M R - M I|.

Total (Eq. 3, with the 2DGS regularisers left to the caller):
  L = (1/V) sum_v (w_c L1_v + gamma L_b,v), gamma = 0.5 (Section 5.1).
All functions accept numpy arrays or float64 torch tensors.
"""
from __future__ import annotations

import numpy as np
import torch


def _lib(x):
    return torch if isinstance(x, torch.Tensor) else np


def background_loss64(alpha, mask):
    """Eq. 1 for one view; alpha and mask of the same shape (H,W)."""
    xp = _lib(alpha)
    m = mask.to(alpha.dtype) if xp is torch else np.asarray(mask, np.float64)
    return (alpha * (1 - m)).sum() / alpha.numel() if xp is torch else \
        float((np.asarray(alpha, np.float64) * (1 - m)).sum() / np.asarray(alpha).size)


def masked_l1_64(color, target, mask):
    """L1 part of Eq. 2 for one view; color, target (3,H,W), mask (H,W)."""
    xp = _lib(color)
    if xp is torch:
        m = mask.to(color.dtype)[None]
        return (m * color - m * target).abs().sum() / color.numel()
    c = np.asarray(color, np.float64)
    m = np.asarray(mask, np.float64)[None]
    return float(np.abs(m * c - m * np.asarray(target, np.float64)).sum() / c.size)


def total_loss64(colors, alphas, targets, masks, gamma=0.5, w_c=1.0):
    """Mean over views of w_c L1 + gamma L_b (lists of per-view arrays)."""
    V = len(alphas)
    tot = 0.0
    for v in range(V):
        tot = tot + w_c * masked_l1_64(colors[v], targets[v], masks[v]) + \
            gamma * background_loss64(alphas[v], masks[v])
    return tot / V
