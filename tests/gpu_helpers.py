"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle (no renderer arithmetic here)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle.render import Params64, render_pixels
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch
from tests.grouping import expand_to_tile_lists, grouped_from_rectangles, instance_count

FWD_TOL = 1e-4


def gpu_run(scene, stats=False, keys64=False, capacity=None, device="cuda", tile=(16, 16)):
    views = ViewBatch(scene.cams, tile=tile, device=device)
    rast = Rasterizer(scene.n, views, scene.sh_degree, sh_stride=scene.sh.shape[1], device=device)
    p = Params.from_scene(scene, device=device)
    if capacity is None:
        rast.plan_capacity(p)
    else:
        rast.set_capacity(capacity)
    rast.preprocess(p)
    k64 = torch.zeros(max(rast.capacity, 1), dtype=torch.int64, device=device) if keys64 else None
    rast.bin(keys64=k64)
    st = None
    if stats:
        st = (torch.zeros(scene.n, dtype=torch.int32, device=device),
              torch.zeros(scene.n, dtype=torch.float32, device=device),
              torch.zeros(scene.n, dtype=torch.float32, device=device))
    rast.forward(stats=st)
    torch.cuda.synchronize()
    out = {"rast": rast, "views": views, "params": p, "status": rast.status()}
    out["keys64"] = k64
    out["stats"] = st
    return out


def per_view(rast: Rasterizer, v: int):
    views = rast.views
    W, H = views.sizes[v]
    o = views.pix_offsets[v]
    n = W * H
    g = lambda t, ch: t[ch * o: ch * (o + n)].detach().cpu().numpy()
    return {
        "color": g(rast.color, 3).reshape(3, H, W),
        "alpha": g(rast.alpha, 1).reshape(H, W),
        "depth": g(rast.depth, 1).reshape(H, W),
        "normal": g(rast.normal, 3).reshape(3, H, W),
        "dist": g(rast.dist, 1).reshape(H, W),
        "T_final": g(rast.T_final, 1).reshape(H, W),
        "n_contrib": g(rast.n_contrib, 1).view(np.uint32).reshape(H, W),
    }


def geometry(scene, rp=oracle.RasterParams()):
    return [oracle.view_geometry64(scene.means, scene.scales, scene.quats, scene.opac, c, rp) for c in scene.cams]


ID_MASK = np.uint32(0xFFFFFF)   # surfel-id bits of a sorted instance value


def compare_binning(scene, run, geoms, rp=oracle.RasterParams(), full_sort=True, expand=True):
    """Bit-exact comparison of the per-(view, surfel) binning outputs and,
    when ``full_sort``, of the whole sorted grouped instance list, its 64-bit
    keys and the per-tile ranges with the layout built from the oracle's
    tile rectangles; with ``expand`` the GPU's group runs are also expanded
    to every tile's list and compared with the oracle's per-tile lists."""
    rast = run["rast"]
    N, V = scene.n, scene.v
    tt = rast.tiles_touched[: V * N].cpu().numpy().view(np.uint32).reshape(V, N)
    dk = rast.depth_key[: V * N].cpu().numpy().view(np.uint32).reshape(V, N)
    rect = rast.rect[: 4 * V * N].cpu().numpy().view(np.uint16).reshape(V, N, 4).astype(np.int64)
    exempt = 0
    for v, g in enumerate(geoms):
        ok = ~g["culled"]
        mism = (tt[v] != g["tiles_touched"]) | (ok & (dk[v] != g["depth_bits"])) | \
            (ok[:, None] & (rect[v] != g["rect"])).any(axis=1)
        # surfels whose cutoff radius sits on a 2^-16 grid point may differ
        bad = mism & ~g["grid_tie"]
        assert not bad.any(), f"view {v}: {bad.sum()} records differ, e.g. {np.nonzero(bad)[0][:5]}"
        exempt += int((mism & g["grid_tie"]).sum())
        assert np.all(dk[v][~ok] == 0xFFFFFFFF)
    vis, need, stored, status = run["status"]
    assert status == 0
    assert vis == sum(int((~g["culled"]).sum()) for g in geoms)
    assert need == stored == instance_count(geoms)
    if full_sort:
        keys, vals, ranges = grouped_from_rectangles(geoms, scene.cams, rp.tile_w, rp.tile_h)
        gv = rast.vals[:need].cpu().numpy().view(np.uint32)
        gr = rast.ranges[: 2 * rast.views.T].cpu().numpy().view(np.uint32).reshape(-1, 2)
        np.testing.assert_array_equal(gv, vals)
        np.testing.assert_array_equal(gr, ranges)
        if run["keys64"] is not None:
            gk = run["keys64"][:need].cpu().numpy().view(np.uint64)
            np.testing.assert_array_equal(gk, keys)
        if expand:
            _, v1, r1 = oracle.bin64(geoms, scene.cams, rp)
            ids, rg = expand_to_tile_lists(gv, gr, scene.cams, rp.tile_w, rp.tile_h)
            np.testing.assert_array_equal(ids, v1)
            np.testing.assert_array_equal(rg, r1)
    return exempt


def oracle_pixels(scene, v, pix, geoms, rp=oracle.RasterParams(), P64=None, loss_fn=None):
    if P64 is None:
        P64 = Params64.from_arrays(scene.means, scene.scales, scene.quats, scene.opac, scene.sh,
                                   scene.sh_degree)
    return render_pixels(P64, scene.cams[v], geoms[v], pix, rp, loss_fn=loss_fn)


def crop_pixels(x0, y0, w, h):
    jj, ii = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1)


def compare_forward(gpu_view, res, pix, rast=None, v=None, tol=FWD_TOL):
    """Max abs errors on unflagged pixels; returns (errors dict, flagged fraction)."""
    i, j = pix[:, 0], pix[:, 1]
    f_ct = res["flag_cut"] | res["flag_term"]
    f_geo = f_ct | res["flag_branch"]
    errs = {}
    checks = (("color", lambda d: d["color"][:, j, i].T, f_ct), ("alpha", lambda d: d["alpha"][j, i], f_ct),
              ("depth", lambda d: d["depth"][j, i], f_geo), ("normal", lambda d: d["normal"][:, j, i].T, f_ct),
              ("dist", lambda d: d["dist"][j, i], f_geo))
    for name, get, flag in checks:
        a = get(gpu_view)
        b = res[name]
        ok = ~flag
        e = np.abs(a[ok] - b[ok])
        errs[name] = float(e.max()) if e.size else 0.0
    for name, e in errs.items():
        assert e <= tol, f"{name}: max abs error {e:.3e} > {tol}"
    if rast is not None:
        # the last blended surfel of every unflagged pixel
        views = rast.views
        W, H = views.sizes[v]
        T0 = int(rast.views.host[v].tile_offset)
        tx = int(rast.views.host[v].tiles_x)
        tw, th = views.tile
        tile = T0 + (j // th) * tx + (i // tw)
        rg = rast.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
        vals = (rast.vals.cpu().numpy().view(np.uint32) & ID_MASK).astype(np.int64)
        nc = gpu_view["n_contrib"][j, i].astype(np.int64)
        last = np.where(nc > 0, vals[np.minimum(rg[tile, 0] + np.maximum(nc - 1, 0), vals.size - 1)], -1)
        ok = ~f_ct
        mism = (last.astype(np.int64) != res["last_gid"]) & ok
        assert not mism.any(), f"{mism.sum()} pixels with a different last blended surfel"
    return errs, float(f_geo.mean())
