"""Occlusion-aware pruning statistics (oracle; test infrastructure only).

Section 4.3: a Gaussian counts as visible when some pixel of some view
blends it, i.e. it passed the alpha cutoff before that pixel's transmittance
terminated; Gaussians that no pixel of any view blends are pruned, even when
they lie inside the viewing frustum (the 3DGS visibility filter, which only
records "inside the frustum", keeps them).

For every blended (pixel, surfel) pair over all views:
  hits[g] += 1, max_alpha[g] = max(max_alpha[g], a), max_weight[g] =
  max(max_weight[g], a T).
prune[g] = max_alpha[g] < tau; with tau = alpha_min every blended pair has
a >= tau, so the mask equals "never blended" (hits == 0).
in_frustum[g] = OR over views of "not culled".
"""
from __future__ import annotations

import numpy as np


def prune_stats64(n: int, pair_lists, culled_per_view=None, tau: float = float(np.float32(1 / 255))):
    """pair_lists: iterable of (pairs, a, omega) as returned by
    ``render_pixels(...)['pairs']`` (pairs[:,1] is the surfel id)."""
    hits = np.zeros(n, np.int64)
    max_alpha = np.zeros(n, np.float64)
    max_weight = np.zeros(n, np.float64)
    for pairs, a, w in pair_lists:
        gid = np.asarray(pairs[:, 1], np.int64)
        np.add.at(hits, gid, 1)
        np.maximum.at(max_alpha, gid, np.asarray(a, np.float64))
        np.maximum.at(max_weight, gid, np.asarray(w, np.float64))
    out = dict(hits=hits, max_alpha=max_alpha, max_weight=max_weight, prune=max_alpha < tau)
    if culled_per_view is not None:
        inf = np.zeros(n, bool)
        for c in culled_per_view:
            inf |= ~np.asarray(c, bool)
        out["in_frustum"] = inf
    return out
