"""Occlusion statistics over many views with the plain-C per-pixel loop
(oracle; test infrastructure only).

The same statistics as ``prune.prune_stats64`` over ``render.render_pixels``
(Section 4.3: hits, maximum alpha and maximum blending weight of every
blended pair, the in-frustum flag, the mask), from the float64 geometry of
``geometry.view_geometry64``, for scenes where the vectorised torch
compositing is too slow (a million surfels over a hundred 800x800 views).
The C source (prune_native.c) is built with gcc on first use.
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes
import os
import subprocess

import numpy as np

from . import render as _render
from .geometry import RasterParams, view_geometry64

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "prune_native.c")
LIB = os.path.join(_HERE, "_prune_native.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile prune_native.c (gcc, -O2, no fast-math: IEEE float64)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        l = ctypes.CDLL(build())
        P = ctypes.c_void_p
        d = ctypes.c_double
        l.prune_view_stats.restype = ctypes.c_int
        l.prune_view_stats.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P, d, d, d, d, ctypes.c_int32,
                                       ctypes.c_int32, d, d, d, d, d, P, P, P, P, P]
        _lib = l
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def prune_stats_view64(means, scales, quats, opac, cam, rp: RasterParams = RasterParams(), geom=None,
                       pix_mask=None, windows=None):
    """Statistics of one view: dict(hits int64 [N], max_alpha, max_weight
    float64 [N], tie uint32 [N] (each surfel's entries exposed to a float32
    tie of their pixel: its hits can change by at most that many),
    visible bool [N]).  ``windows`` = (cutoff, termination) relative tie
    windows, by default those of oracle.render."""
    n = np.asarray(means).shape[0]
    g = geom if geom is not None else view_geometry64(means, scales, quats, opac, cam, rp)
    vis = np.nonzero(~g["culled"])[0]
    order = vis[np.lexsort((vis, g["depth_bits"][vis]))]
    c = lambda a, dt: np.ascontiguousarray(a, dtype=dt)
    ids = c(order, np.int64)
    rect = c(g["rect"][order], np.int32)
    p, au, av = c(g["p"][order], np.float64), c(g["au"][order], np.float64), c(g["av"][order], np.float64)
    ctr = c(g["center"][order], np.float64)
    op = c(np.asarray(opac, np.float64)[order], np.float64)
    out = dict(hits=np.zeros(n, np.int64), max_alpha=np.zeros(n), max_weight=np.zeros(n),
               tie=np.zeros(n, np.uint32), visible=~g["culled"])
    pm = None if pix_mask is None else c(pix_mask, np.uint8)
    f32 = lambda v: float(np.float32(v))
    w_cut, w_term = (_render.TIE_CUTOFF_REL, _render.TIE_TERM_REL) if windows is None else windows
    st = _load().prune_view_stats(ids.size, _ptr(ids), _ptr(rect), _ptr(p), _ptr(au), _ptr(av), _ptr(ctr), _ptr(op),
                                  f32(cam.fx), f32(cam.fy), f32(cam.cx), f32(cam.cy), int(cam.width),
                                  int(cam.height), rp.alpha_min, rp.alpha_max, rp.t_min, w_cut, w_term, _ptr(pm), _ptr(out["hits"]), _ptr(out["max_alpha"]),
                                  _ptr(out["max_weight"]), _ptr(out["tie"]))
    if st != 0:
        raise MemoryError("prune_view_stats: out of memory")
    return out


def prune_stats_views64(means, scales, quats, opac, cams, rp: RasterParams = RasterParams(), workers: int = 1,
                        tau: float = None, windows=None):
    """Statistics accumulated over the views ``cams`` (sums of the hits and
    tie counts, maxima, OR of the in-frustum flags), and the mask max_alpha < tau
    (tau = alpha_min by default); views are spread over ``workers``
    threads (the C loop releases the interpreter lock)."""
    n = np.asarray(means).shape[0]
    tot = dict(hits=np.zeros(n, np.int64), max_alpha=np.zeros(n), max_weight=np.zeros(n),
               tie=np.zeros(n, np.uint32), in_frustum=np.zeros(n, bool))

    def one(cam):
        return prune_stats_view64(means, scales, quats, opac, cam, rp, windows=windows)

    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for r in ex.map(one, cams):
            tot["hits"] += r["hits"]
            np.maximum(tot["max_alpha"], r["max_alpha"], out=tot["max_alpha"])
            np.maximum(tot["max_weight"], r["max_weight"], out=tot["max_weight"])
            tot["tie"] += r["tie"]
            tot["in_frustum"] |= r["visible"]
    t = rp.alpha_min if tau is None else tau
    tot["prune"] = tot["max_alpha"] < t
    return tot
