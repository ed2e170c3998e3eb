"""Helpers of the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle (no renderer arithmetic here)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle.render import (TIE_KINDS, WIDE_CUTOFF_REL, WIDE_TERM_REL, Params64, render_alternatives,
                           render_pixels)
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


def _gpu_last_gid(gpu_view, pix, rast, v):
    """Surfel id of the last blended entry of each pixel (-1 if none), read
    from the GPU's n_contrib and its sorted lists."""
    i, j = pix[:, 0], pix[:, 1]
    views = rast.views
    T0 = int(views.host[v].tile_offset)
    tx = int(views.host[v].tiles_x)
    tw, th = views.tile
    tile = T0 + (j // th) * tx + (i // tw)
    rg = rast.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    vals = (rast.vals.cpu().numpy().view(np.uint32) & ID_MASK).astype(np.int64)
    nc = gpu_view["n_contrib"][j, i].astype(np.int64)
    return np.where(nc > 0, vals[np.minimum(rg[tile, 0] + np.maximum(nc - 1, 0), vals.size - 1)], -1)


def _gpu_values(gpu_view, pix):
    i, j = pix[:, 0], pix[:, 1]
    return {"color": gpu_view["color"][:, j, i].T, "alpha": gpu_view["alpha"][j, i],
            "depth": gpu_view["depth"][j, i], "normal": gpu_view["normal"][:, j, i].T,
            "dist": gpu_view["dist"][j, i]}


def _row_err(g, ref, rows_g, rows_r, names=("color", "alpha", "depth", "normal", "dist")):
    e = np.zeros(len(rows_g))
    for k in names:
        d = np.abs(np.asarray(g[k])[rows_g] - np.asarray(ref[k])[rows_r])
        e = np.maximum(e, d.reshape(len(rows_g), -1).max(axis=1))
    return e


def _match(g, last, r_gpu, cands, ref_rows, tol):
    """Indices of the candidate results (res, row) that the GPU's pixel
    r_gpu matches within tol (and, with ``last``, by its last blended
    surfel), and their errors."""
    errs, good = [], []
    for k, (ref, rr) in enumerate(zip(cands, ref_rows)):
        e = float(_row_err(g, ref, [r_gpu], [rr])[0])
        errs.append(e)
        if e <= tol and (last is None or int(ref["last_gid"][rr]) == last[r_gpu]):
            good.append(k)
    return good, errs


def _resolve(g, last, r_gpu, res, row, alts, ares, tol, what):
    """The flips (possibly none) of the correct result the GPU's pixel
    matches best; asserts that it matches one."""
    cands, rows, flips = [res], [row], [()]
    for k, (rr, f) in enumerate(alts):
        if rr == row:
            cands.append(ares)
            rows.append(k)
            flips.append(f)
    good, errs = _match(g, last, r_gpu, cands, rows, tol)
    assert good, (f"{what} pixel matches none of its {len(cands)} correct results: errors {errs}, last surfel "
                  f"gpu {None if last is None else last[r_gpu]} vs {[int(c['last_gid'][r]) for c, r in zip(cands, rows)]}")
    return list(flips[min(good, key=lambda k: errs[k])])


def compare_forward(gpu_view, res, pix, rast=None, v=None, tol=FWD_TOL, oracle_ctx=None):
    """Forward parity with the tie protocol.

    A pixel whose list holds no tie entry must match the oracle within
    ``tol`` on every output and (with ``rast``) blend the same last surfel.
    A pixel with a tie entry (a value within float32 reach of the cutoff,
    the termination test or the surface/low-pass choice: the primary
    windows) must match one of the oracle's correct results
    (``render_alternatives``: each subset of its tie entries taken the other
    way).  A pixel without a tie entry that does not match is re-examined
    under the wide windows (WIDE_CUTOFF_REL, WIDE_TERM_REL) and must then
    match one of its correct results.  Needs ``oracle_ctx`` = (P64, cam,
    geom, rp) for the alternatives (without it tie pixels are only counted).

    Returns (max abs errors of the pixels matched without a tie, fraction of
    pixels resolved through a tie, report) with report: ``choice`` {row:
    flips} of the pixels whose match took some tie the other way (feed it as
    ``flips`` to the oracle's gradient pass), ``entries`` [(kind, distance,
    taken other way)] of the primary tie entries, ``wide`` the rows resolved
    under the wide windows, ``unresolved`` rows with too many ties."""
    f_geo = res["flag_cut"] | res["flag_term"] | res["flag_branch"]
    g = _gpu_values(gpu_view, pix)
    last = _gpu_last_gid(gpu_view, pix, rast, v) if rast is not None else None
    n = pix.shape[0]
    row_err = _row_err(g, res, np.arange(n), np.arange(n))
    bad = ~f_geo & (row_err > tol)
    if last is not None:
        bad |= ~f_geo & (last != res["last_gid"])
    report = {"choice": {}, "entries": [], "unresolved": [], "wide": []}
    if oracle_ctx is None:
        assert not bad.any(), f"{bad.sum()} pixels differ (max error {row_err[bad].max():.3e})"
        report["unresolved"] = np.nonzero(f_geo)[0].tolist()
    else:
        P64, cam, geom, rp = oracle_ctx
        rows = np.nonzero(f_geo)[0]
        if rows.size:
            alts, ares, unres = render_alternatives(P64, cam, geom, pix, res["tie_list"], rp)
            report["unresolved"] = unres
            tl, td = res["tie_list"], res["tie_dist"]
            for r in rows:
                if r in unres:
                    continue
                fl = _resolve(g, last, r, res, r, alts, ares, tol, f"tie pixel {pix[r].tolist()}")
                if fl:
                    report["choice"][int(r)] = fl
                for (_, gid, kind), d in zip(tl[tl[:, 0] == r], td[tl[:, 0] == r]):
                    if kind <= 2:
                        report["entries"].append((TIE_KINDS[kind], float(d), (int(gid), TIE_KINDS[kind]) in fl))
        brows = np.nonzero(bad)[0]
        if brows.size:
            wide = (WIDE_CUTOFF_REL, WIDE_TERM_REL)
            sub = pix[brows]
            res_w = render_pixels(P64, cam, geom, sub, rp, windows=wide)
            alts, ares, unres = render_alternatives(P64, cam, geom, sub, res_w["tie_list"], rp, windows=wide)
            gs = {k: np.asarray(a)[brows] for k, a in g.items()}
            ls = None if last is None else last[brows]
            for i, r in enumerate(brows):
                assert i not in unres, f"pixel {pix[r].tolist()}: too many ties under the wide windows"
                fl = _resolve(gs, ls, i, res_w, i, alts, ares, tol, f"pixel {pix[r].tolist()} (wide windows)")
                if fl:
                    report["choice"][int(r)] = fl
            report["wide"] = brows.tolist()
    ok = ~f_geo & ~bad
    errs = {}
    for name in ("color", "alpha", "depth", "normal", "dist"):
        e = np.abs(np.asarray(g[name])[ok] - np.asarray(res[name])[ok])
        errs[name] = float(e.max()) if e.size else 0.0
    for name, e in errs.items():
        assert e <= tol, f"{name}: max abs error {e:.3e} > {tol}"
    return errs, float((f_geo | bad).mean()), report


GRAD_RTOL = 1e-3


def compare_grads(g, gref, excl=(), names=("means", "scales", "quats", "opac", "sh"), rtol=GRAD_RTOL):
    """The gradient bar: per tensor ||g - g_ref||_inf <= rtol ||g_ref||_inf,
    and |g - g_ref| <= rtol |g_ref| for every element with |g_ref| >=
    1e-2 ||g_ref||_inf; rows (surfels) in ``excl`` are left out."""
    report = {}
    for name, a, b in zip(names, g, gref):
        keep = np.ones(a.shape[0], bool)
        keep[np.asarray(excl, np.int64)] = False
        a, b = a[keep].reshape(-1), b[keep].reshape(-1)
        scale = np.abs(b).max()
        err = np.abs(a - b).max()
        big = np.abs(b) >= 1e-2 * scale
        rel = (np.abs(a - b)[big] / np.abs(b)[big]).max() if big.any() else 0.0
        report[name] = (float(err / max(scale, 1e-30)), float(rel))
    print("gradient errors (inf-norm relative, elementwise relative):", report, flush=True)
    for name, (e, r) in report.items():
        assert e <= rtol, f"{name}: inf-norm relative error {e:.2e}"
        assert r <= rtol, f"{name}: elementwise relative error {r:.2e}"
    return report


def clamp_tie_ids(res):
    """Surfels with an entry at the alpha clamp (within float32 reach): the
    value is continuous there but its derivative in the opacity is not."""
    tl = res["tie_list"]
    return np.unique(tl[tl[:, 2] == TIE_KINDS.index("clamp"), 1]) if len(tl) else np.zeros(0, np.int64)


def masked_loss_fn(mask_v, target_v, pix, HW, V, gamma, w_c):
    """The per-pixel masked L1 + background loss (Eq. 1, Eq. 2) of the
    pixels ``pix`` of one view, as a loss_fn for render_pixels: its sum over
    the chunks is (1/V) (w_c L1_v + gamma L_b,v) restricted to ``pix``."""
    m = torch.tensor(mask_v[pix[:, 1], pix[:, 0]], dtype=torch.float64)
    tgt = torch.tensor(np.asarray(target_v)[:, pix[:, 1], pix[:, 0]].T, dtype=torch.float64)

    def lf(out, rows):
        r = torch.as_tensor(rows)
        mm = m[r]
        l1 = (mm[:, None] * out["color"] - mm[:, None] * tgt[r]).abs().sum() / (3 * HW)
        lb = (out["alpha"] * (1 - mm)).sum() / HW
        return (w_c * l1 + gamma * lb) / V
    return lf


def masked_terms(res, mask_v, target_v, pix, HW):
    """(L1_v, L_b,v) of Eq. 2 / Eq. 1 summed over the pixels ``pix`` from the
    oracle's outputs (the view's terms when the rest of the view contributes
    nothing)."""
    m = mask_v[pix[:, 1], pix[:, 0]].astype(np.float64)
    tgt = np.asarray(target_v, np.float64)[:, pix[:, 1], pix[:, 0]].T
    l1 = float(np.abs(m[:, None] * res["color"] - m[:, None] * tgt).sum() / (3 * HW))
    lb = float((res["alpha"] * (1 - m)).sum() / HW)
    return l1, lb
