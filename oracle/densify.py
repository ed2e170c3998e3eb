"""Density-control statistic of the training loop (oracle; test
infrastructure only).

The method keeps 2DGS's adaptive density control (Section 5.1), which
accumulates, per Gaussian, the norm of the loss gradient with respect to the
Gaussian's position on the screen, over the views in which it is inside the
frustum, with a count of those views.  Reading (listed in the design notes):
the position on the screen is a translation delta of the whole splat in
pixel units (the splat is then evaluated at x - delta, surface and low-pass
alike); per view the statistic is |dL/d delta|_2, summed over views, and the
count is the number of views in which the surfel is not culled.
"""
from __future__ import annotations

import numpy as np
import torch

from .render import render_pixels


def screen_grad_stats64(P, cams, geoms, pix_per_view, rp, loss_fn_per_view):
    """(sum over views of |dL/d delta|, count of views not culled, per-view
    gradients (V,N,2)) for the loss given per view by
    ``loss_fn_per_view[v](out_chunk, rows)``."""
    N = P.means.shape[0]
    total = np.zeros(N)
    count = np.zeros(N, np.int64)
    per_view = []
    flagged = []
    for v, cam in enumerate(cams):
        shift = torch.zeros((N, 2), dtype=torch.float64, requires_grad=True)
        res = render_pixels(P, cam, geoms[v], pix_per_view[v], rp, loss_fn=loss_fn_per_view[v],
                            screen_shift=shift)
        g = shift.grad.numpy().copy() if shift.grad is not None else np.zeros((N, 2))
        per_view.append(g)
        vis = ~geoms[v]["culled"]
        total[vis] += np.sqrt((g[vis] ** 2).sum(axis=1))
        count[vis] += 1
        flagged.append(res["tie_ids"])
    return total, count, np.stack(per_view), np.unique(np.concatenate(flagged)) if flagged else np.zeros(0)
