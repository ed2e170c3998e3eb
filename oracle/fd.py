"""Central finite differences of the FP64 oracle (test infrastructure only).

Used to pin the oracle's autograd gradients (and, through them, the GPU
backward).  Gradients of the renderer are piecewise: the alpha cutoff, the
transmittance stop, the surface/low-pass branch and the two clamps are jumps
or kinks.  A parameter is accepted for comparison only when the set of those
decisions is the same at theta + h and theta - h.
"""
from __future__ import annotations

import numpy as np
import torch

from .render import Params64, render_pixels, DT

NAMES = ("means", "scales", "quats", "opac", "sh")


def _decisions(res):
    out = []
    for d in res["decisions"]:
        bl = d["blended"]
        out.append((bl.tobytes(), (d["surf"] & bl).tobytes(), d["first_stop"].tobytes(),
                    (d["clamp"] & bl).tobytes()))
    return out


def loss_and_decisions(P: Params64, cams, geoms, pixsets, loss_fn, rp):
    """Sum over views of loss_fn(view, outputs) (no gradient) plus the
    decision sets of every view."""
    total = 0.0
    dec = []
    with torch.no_grad():
        for v, cam in enumerate(cams):
            res = render_pixels(P, cam, geoms[v], pixsets[v], rp, keep_decisions=True)
            total += float(loss_fn(v, res))
            dec.append(_decisions(res))
            # colour clamp state of every surfel in this view
            from .render import surfel_view_quantities
            ids = np.arange(P.means.shape[0])
            Q = surfel_view_quantities(P, ids, cam, geoms[v]["flip"])
            dec.append((Q["rgb_raw"] > 0).numpy().tobytes())
    return total, dec


def central_fd(P: Params64, cams, geoms, pixsets, loss_fn, rp, which, rel_h=1e-6):
    """which: list of (name, flat_index).  Returns list of
    (name, index, derivative, accepted)."""
    out = []
    for name, flat in which:
        t = getattr(P, name)
        base = float(t.detach().reshape(-1)[flat])
        h = rel_h * max(1.0, abs(base))
        vals, decs = [], []
        for sgn in (1.0, -1.0):
            with torch.no_grad():
                t.view(-1)[flat] = base + sgn * h
            L, d = loss_and_decisions(P, cams, geoms, pixsets, loss_fn, rp)
            vals.append(L)
            decs.append(d)
        with torch.no_grad():
            t.view(-1)[flat] = base
        out.append((name, flat, (vals[0] - vals[1]) / (2 * h), decs[0] == decs[1]))
    return out
