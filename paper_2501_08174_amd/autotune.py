"""Autotuner for the compositing kernels: tile shape x backward LDS batch.

Times one full training step (projection, binning, forward with the usage
counts, loss, backward) for every compiled tile shape and, for each, every
compiled backward batch (records staged per LDS batch: 32, 64, 128, 256 up
to the tile's pixel count) on the caller's own workload, and keeps the
fastest pair.  Results are cached in a JSON file keyed by GPU architecture,
resolution bucket, surfel-count bucket and SH degree.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import _lib
from .raster import Params, Rasterizer, ViewBatch

CANDIDATES: Tuple[Tuple[int, int], ...] = ((16, 16), (16, 8), (8, 8), (32, 8))
BATCHES: Tuple[int, ...] = (32, 64, 128, 256)
CACHE = os.environ.get("SR_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "surfelrast",
                                                         "autotune.json"))


def _bucket(x: float) -> int:
    return int(round(math.log2(max(x, 1.0))))


def cache_key(cams: Sequence, n: int, sh_degree: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    mean_px = sum(c.width * c.height for c in cams) / max(len(cams), 1)
    return f"{arch}|px2^{_bucket(mean_px)}|v{len(cams)}|n2^{_bucket(n)}|sh{sh_degree}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict[str, dict]):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
    except OSError:
        pass


def time_step(rast: Rasterizer, p: Params, g: Params, mask, target, stats=None, steps: int = 3) -> float:
    """Mean milliseconds of one training step on the current stream; stats
    (the hits tensor alone, or hits with both maxima) are accumulated by the
    forward as in Rasterizer.forward."""

    def step():
        rast.preprocess(p)
        rast.bin()
        rast.train_step_raster(mask, target, 0.5, 1.0, stats=stats, accumulate=True)
        rast.backward_project(p, g)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def autotune(cams: Sequence, p: Params, sh_degree: int, sh_stride: int, mask, target,
             candidates: Sequence[Tuple[int, int]] = CANDIDATES, batches: Sequence[int] = BATCHES, steps: int = 3,
             use_cache: bool = True, report: Optional[dict] = None) -> Tuple[Tuple[int, int], int]:
    """Fastest compiled (tile shape, backward batch) for this workload: times
    every pair, returns ((tile_w, tile_h), batch)."""
    n = p.means.shape[0]
    key = cache_key(cams, n, sh_degree)
    cache = _load() if use_cache else {}
    if key in cache and "batch" in cache[key]:
        if report is not None:
            report.update(cache[key])
        return tuple(cache[key]["tile"]), int(cache[key]["batch"])
    l = _lib.lib()
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    used = torch.zeros(n, dtype=torch.int32, device=p.means.device)
    times = {}
    for tw, th in candidates:
        if not l.sr_tile_supported(tw, th):
            continue
        views = ViewBatch(cams, tile=(tw, th))
        rast = Rasterizer(n, views, sh_degree, sh_stride=sh_stride)
        rast.plan_capacity(p, slack=1.02)
        for b in batches:
            if not l.sr_bwd_batch_supported(tw, th, b):
                continue
            rast.set_bwd_batch(b)
            times[f"{tw}x{th}/b{b}"] = time_step(rast, p, g, mask, target, used, steps)
        del rast
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    ts, bs = best.split("/b")
    tile = tuple(int(x) for x in ts.split("x"))
    entry = {"tile": list(tile), "batch": int(bs), "ms": times}
    if use_cache:
        cache[key] = entry
        _store(cache)
    if report is not None:
        report.update(entry)
    return tile, int(bs)
