"""Parity at the full workload sizes, in the launch configuration the
benchmark uses: per-record bit-exact binning over every (view, surfel),
sampled tile lists, forward/backward on 64x64 crops and sampled pixels the
oracle evaluates one by one, central finite differences on a 200-surfel
subset, and the occlusion statistics of the shell scene over all 100 views."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from oracle.render import Params64, render_pixels
from paper_2501_08174_amd import scenes
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch, rasterize, prune_mask
from tests.gpu_helpers import clamp_tie_ids, compare_forward, compare_grads, crop_pixels, gpu_run, per_view
from tests.grouping import grouped_from_rectangles, instance_count, tile_list

pytestmark = pytest.mark.gpu
RP = oracle.RasterParams()
TIE_FRACTION = 1e-3     # largest fraction of compared pixels with a tie entry (each one still checked)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _geoms_parallel(sc, views=None):
    views = range(sc.v) if views is None else views
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        fut = {v: ex.submit(oracle.view_geometry64, sc.means, sc.scales, sc.quats, sc.opac, sc.cams[v], RP)
               for v in views}
        return {v: f.result() for v, f in fut.items()}


def _records_bit_exact(sc, rast, geoms):
    N = sc.n
    bad_total = 0
    for v, g in geoms.items():
        sl = slice(v * N, (v + 1) * N)
        tt = rast.tiles_touched[sl].cpu().numpy().view(np.uint32)
        dk = rast.depth_key[sl].cpu().numpy().view(np.uint32)
        rect = rast.rect[4 * v * N: 4 * (v + 1) * N].cpu().numpy().view(np.uint16).reshape(N, 4)
        ok = ~g["culled"]
        mism = (tt != g["tiles_touched"]) | (ok & (dk != g["depth_bits"])) | \
            (ok[:, None] & (rect.astype(np.int64) != g["rect"])).any(axis=1)
        bad = mism & ~g["grid_tie"]
        assert not bad.any(), f"view {v}: {bad.sum()} records differ: {np.nonzero(bad)[0][:5]}"
        bad_total += int(mism.sum())
    return bad_total


def _tile_list(g, tx_count, local_tile):
    ty, tx = divmod(local_tile, tx_count)
    sel = (~g["culled"]) & (g["tiles"][:, 0] <= tx) & (tx <= g["tiles"][:, 1]) & \
        (g["tiles"][:, 2] <= ty) & (ty <= g["tiles"][:, 3])
    ids = np.nonzero(sel)[0]
    return ids[np.lexsort((ids, g["depth_bits"][ids]))]


def _sampled_tiles(sc, run, geoms, n_tiles=48, seed=0):
    rast = run["rast"]
    views = rast.views
    rg = rast.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    vals = rast.vals.cpu().numpy().view(np.uint32)
    k64 = run["keys64"].cpu().numpy().view(np.uint64) if run["keys64"] is not None else None
    rng = np.random.default_rng(seed)
    for _ in range(n_tiles):
        v = int(rng.choice(list(geoms.keys())))
        h = views.host[v]
        t = int(rng.integers(0, h.tiles_x * h.tiles_y))
        want = _tile_list(geoms[v], h.tiles_x, t)
        tx, ty = t % h.tiles_x, t // h.tiles_x
        ids, pos = tile_list(vals, rg, h.tile_offset + t, (tx, ty))
        np.testing.assert_array_equal(ids, want)
        if k64 is not None:
            grp = h.group_offset + (ty // 4) * h.groups_x + tx // 4
            exp = (np.uint64(grp) << np.uint64(32)) | geoms[v]["depth_bits"][want].astype(np.uint64)
            np.testing.assert_array_equal(k64[pos], exp)
    # global properties: the groups' runs partition [0, n_inst) in group order
    n = run["status"][2]
    nz = np.unique(rg[rg[:, 1] > rg[:, 0]], axis=0)
    assert nz[0, 0] == 0 and nz[-1, 1] == n and np.all(nz[1:, 0] == nz[:-1, 1])


def _crop_forward(sc, rast, geoms, v, x0, y0, P64, w=64, h=64):
    """Forward parity on a crop under the tie protocol; returns (errors, tie
    pixels, compared pixels)."""
    pix = crop_pixels(x0, y0, w, h)
    res = render_pixels(P64, sc.cams[v], geoms[v], pix, RP)
    errs, frac, rep = compare_forward(per_view(rast, v), res, pix, rast, v,
                                      oracle_ctx=(P64, sc.cams[v], geoms[v], RP))
    assert not rep["unresolved"]
    return errs, int(round(frac * pix.shape[0])), pix.shape[0]


# --------------------------------------------------------------------------
# frame800-100k: one 800x800 view, 100k surfels, SH degree 3
# --------------------------------------------------------------------------

def _gpu_crop_grads(sc, x0, y0, w, h, gamma=0.5, w_c=1.0):
    """GPU gradients of the crop-restricted loss through the autograd path."""
    views = ViewBatch(sc.cams)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    p = Params.from_scene(sc)
    rast.plan_capacity(p)
    leaves = [t.clone().requires_grad_(True) for t in (p.means, p.scales, p.quats, p.opac, p.sh)]
    color, alpha, depth, normal, dist = rasterize(*leaves, rast)
    cam = sc.cams[0]
    H, W = cam.height, cam.width
    m = torch.tensor(sc.masks[0], dtype=torch.float32, device="cuda")
    tgt = torch.tensor(sc.targets[0], device="cuda")
    C = color.view(3, H, W)[:, y0:y0 + h, x0:x0 + w]
    A = alpha.view(H, W)[y0:y0 + h, x0:x0 + w]
    mc = m[y0:y0 + h, x0:x0 + w]
    L = w_c * (mc * C - mc * tgt[:, y0:y0 + h, x0:x0 + w]).abs().sum() / (3 * H * W) + \
        gamma * (A * (1 - mc)).sum() / (H * W)
    L.backward()
    torch.cuda.synchronize()
    return [t.grad.cpu().numpy().astype(np.float64) for t in leaves], float(L.item()), rast


def _oracle_crop_loss_fn(sc, x0, y0, w, h, gamma=0.5, w_c=1.0):
    cam = sc.cams[0]
    H, W = cam.height, cam.width
    pix = crop_pixels(x0, y0, w, h)
    m = torch.tensor(sc.masks[0][pix[:, 1], pix[:, 0]], dtype=torch.float64)
    tgt = torch.tensor(sc.targets[0][:, pix[:, 1], pix[:, 0]].T, dtype=torch.float64)

    def lf(out, rows):
        r = torch.as_tensor(rows)
        mm = m[r]
        return (w_c * (mm[:, None] * out["color"] - mm[:, None] * tgt[r]).abs().sum() / (3 * H * W)
                + gamma * (out["alpha"] * (1 - mm)).sum() / (H * W))
    return pix, lf


def test_frame800_crop_backward_and_fd_subset():
    """Gradients of the crop loss: GPU vs oracle autograd on every surfel,
    and GPU vs central finite differences of the FP64 oracle on 200
    surfels (seed 22) visible in the crop [368, 432)^2."""
    sc = scenes.make_frame800_100k()
    x0 = y0 = 368
    g, Lg, rast = _gpu_crop_grads(sc, x0, y0, 64, 64)
    geom = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, sc.cams[0], RP)
    pix, lf = _oracle_crop_loss_fn(sc, x0, y0, 64, 64)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 3, requires_grad=True)
    res0 = render_pixels(P64, sc.cams[0], geom, pix, RP)
    errs, frac, rep = compare_forward(per_view(rast, 0), res0, pix, rast, 0, oracle_ctx=(P64, sc.cams[0], geom, RP))
    assert not rep["unresolved"] and frac <= TIE_FRACTION
    choice = rep["choice"]          # ties taken the way the GPU took them, in every oracle pass below
    res = render_pixels(P64, sc.cams[0], geom, pix, RP, loss_fn=lf, flips=choice)
    gref = P64.grads()
    touched = np.unique(res["pairs"][0][:, 1])
    keep_rows = np.zeros(sc.n, bool)
    keep_rows[touched] = True
    clamp = clamp_tie_ids(res0)
    keep_rows[clamp] = False
    excl = np.nonzero(~keep_rows)[0]
    print(f"surfels blended in the crop {touched.size}; tie pixels {frac:.4f}, {len(choice)} taken the other way; "
          f"clamp-tie surfels left out {clamp.size}", flush=True)
    compare_grads(g, gref, excl)
    # finite differences on a 200-surfel subset, one random parameter each
    rng = np.random.default_rng(22)
    sub = rng.choice(touched, size=min(200, touched.size), replace=False)
    P0 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 3)
    names = ("means", "scales", "quats", "opac", "sh")
    widths = (3, 2, 4, 1, 48)
    checked, worst = 0, 0.0
    for gid in sub:
        k = int(rng.integers(0, 5))
        name = names[k]
        j = int(rng.integers(0, widths[k]))
        rect = geom["rect"][gid]
        fp = crop_pixels(max(rect[0], x0), max(rect[2], y0), min(rect[1], x0 + 63) - max(rect[0], x0) + 1,
                         min(rect[3], y0 + 63) - max(rect[2], y0) + 1)
        rows = (fp[:, 1] - y0) * 64 + (fp[:, 0] - x0)
        fl = {i: choice[int(r)] for i, r in enumerate(rows) if int(r) in choice}
        t = getattr(P0, name)
        flat = gid * widths[k] + j
        base = float(t.view(-1)[flat])
        hstep = 1e-6 * max(1.0, abs(base))
        vals, decs = [], []
        for sgn in (1, -1):
            with torch.no_grad():
                t.view(-1)[flat] = base + sgn * hstep
                r = render_pixels(P0, sc.cams[0], geom, fp, RP, keep_decisions=True, flips=fl,
                                  loss_fn=lambda out, rr: vals.append(float(lf(out, rows[rr]))) or None)
            # decisions that change the value: which entries blend, and their
            # branch and clamp (those of skipped entries do not matter)
            decs.append([d["blended"].tobytes() + (d["surf"] & d["blended"]).tobytes() +
                         (d["clamp"] & d["blended"]).tobytes() + d["first_stop"].tobytes()
                         for d in r["decisions"]])
        with torch.no_grad():
            t.view(-1)[flat] = base
        if decs[0] != decs[1]:
            continue
        fd = (sum(vals[: len(vals) // 2]) - sum(vals[len(vals) // 2:])) / (2 * hstep)
        gg = g[k].reshape(-1)[flat]
        scale = max(abs(fd), 1e-3 * np.abs(gref[k]).max())
        err = abs(gg - fd) / scale
        worst = max(worst, err)
        assert err <= 1e-3, (name, gid, j, gg, fd)
        checked += 1
        if checked % 50 == 0:
            print(f"  FD: {checked} checked, worst {worst:.2e}", flush=True)
    print(f"FD subset of {sub.size} surfels: {checked} parameters checked, "
          f"{sub.size - checked} with a decision change inside +-h; worst relative error {worst:.2e}")
    assert checked >= 150


# --------------------------------------------------------------------------
# ragged16-1m: 16 views 400..1600 px, 1M surfels (the benchmark workload)
# --------------------------------------------------------------------------

def test_ragged16_full_size():
    sc = scenes.make_ragged16_1m()
    run = gpu_run(sc, keys64=True, stats=True)
    rast = run["rast"]
    print("ragged16-1m: GPU pass done", flush=True)
    geoms = _geoms_parallel(sc)
    print("ragged16-1m: oracle geometry of 16 views done", flush=True)
    ex = _records_bit_exact(sc, rast, geoms)
    print("ragged16-1m records bit-exact; grid-tie exemptions", ex)
    vis, need, stored, status = run["status"]
    assert status == 0 and vis == sum(int((~g["culled"]).sum()) for g in geoms.values())
    assert need == instance_count(list(geoms.values()))
    # the whole sorted instance list, its 64-bit keys and every tile's range,
    # against the grouped layout built from the oracle's tile rectangles
    gl = [geoms[v] for v in range(sc.v)]
    keys, vals, ranges = grouped_from_rectangles(gl, sc.cams, RP.tile_w, RP.tile_h)
    print(f"ragged16-1m: oracle sorted list of {vals.size} instances built", flush=True)
    np.testing.assert_array_equal(rast.vals[:need].cpu().numpy().view(np.uint32), vals)
    np.testing.assert_array_equal(rast.ranges[: 2 * rast.views.T].cpu().numpy().view(np.uint32).reshape(-1, 2),
                                  ranges)
    np.testing.assert_array_equal(run["keys64"][:need].cpu().numpy().view(np.uint64), keys)
    del keys, vals, ranges
    print("ragged16-1m: whole sorted list, keys and ranges bit-exact", flush=True)
    _sampled_tiles(sc, run, geoms)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 3)
    rng = np.random.default_rng(3)
    ties, npix = 0, 0
    for v in (0, 5, 12):
        cam = sc.cams[v]
        x0 = int(rng.integers(0, cam.width - 64))
        y0 = int(rng.integers(0, cam.height - 64))
        errs, t, n = _crop_forward(sc, rast, geoms, v, cam.width // 2 - 32, cam.height // 2 - 32, P64)
        ties, npix = ties + t, npix + n
        print(f"ragged16-1m view {v} centre crop errors {errs} tie pixels {t}", flush=True)
        errs, t, n = _crop_forward(sc, rast, geoms, v, x0, y0, P64, w=32, h=32)
        ties, npix = ties + t, npix + n
        print(f"ragged16-1m view {v} crop ({x0},{y0}) errors {errs} tie pixels {t}", flush=True)
    assert ties <= TIE_FRACTION * npix, (ties, npix)


def test_wide8_crop():
    sc = scenes.make_wide8_3m()
    run = gpu_run(sc, stats=True)
    rast = run["rast"]
    geoms = _geoms_parallel(sc, views=[0])
    assert _records_bit_exact(sc, rast, geoms) == 0
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 3)
    errs, t, n = _crop_forward(sc, rast, geoms, 0, 948, 513, P64)
    print("wide8-3m crop errors", errs, "tie pixels", t)
    assert t <= TIE_FRACTION * n or t <= 2, t


# --------------------------------------------------------------------------
# shell100: occlusion pruning over 100 views of the shell scene
# --------------------------------------------------------------------------

def test_shell100_pruning():
    """Section 4.3 on the shell scene over 100 views (sr_prune_contrib, the
    whole pass): every interior surfel is inside the frustum of every view
    yet never blended (pruned); and every one of the 1.1M surfels has the
    oracle's statistics over all 100 views (the plain-C oracle loop): hits
    exact, maxima within 1e-5, mask and in-frustum flags exact; a surfel
    whose entries are exposed to a float32 tie of their pixel (a tie entry
    under the wide windows of the tie protocol - the pruning exemption of
    1e-6 on alpha - or a decision after one) has its hits within its
    exposure count of the oracle's, and is kept whenever the oracle blends
    it more often than that."""
    import os
    import time
    from oracle.prune_native import prune_stats_views64
    from oracle.render import WIDE_CUTOFF_REL, WIDE_TERM_REL
    from paper_2501_08174_amd.raster import prune_contrib
    sc = scenes.make_shell100()
    N = sc.n
    p = Params.from_scene(sc)
    print("shell100: scene ready", flush=True)
    st = prune_contrib(p, sc.cams, views_per_chunk=20)
    torch.cuda.synchronize()
    print("shell100: pruning pass over 100 views done", flush=True)
    mask = st.mask.cpu().numpy().astype(bool)
    h = st.hits.cpu().numpy().view(np.uint32).astype(np.int64)
    ma = st.max_alpha.cpu().numpy()
    mw = st.max_weight.cpu().numpy()
    infr = st.in_frustum.cpu().numpy().astype(bool)
    n_shell, n_inner = 300_000, 700_000
    inner = slice(n_shell, n_shell + n_inner)
    assert infr[inner].all()
    assert mask[inner].all() and (h[inner] == 0).all()
    assert np.array_equal(mask, h == 0)
    kept_shell = (~mask[:n_shell]).mean()
    print(f"pruned {mask.sum()} of {N}; shell kept {kept_shell:.3f}; exterior kept "
          f"{(~mask[n_shell + n_inner:]).mean():.3f}; in-frustum but pruned {(infr & mask).sum()}", flush=True)
    assert kept_shell > 0.5
    # the oracle over every view, ten views at a time
    t0 = time.time()
    workers = min(16, len(os.sched_getaffinity(0)))
    ref = None
    for v0 in range(0, sc.v, 10):
        r = prune_stats_views64(sc.means, sc.scales, sc.quats, sc.opac, sc.cams[v0:v0 + 10], RP, workers=workers,
                                windows=(WIDE_CUTOFF_REL, WIDE_TERM_REL))
        if ref is None:
            ref = r
        else:
            ref["hits"] += r["hits"]
            ref["tie"] += r["tie"]
            np.maximum(ref["max_alpha"], r["max_alpha"], out=ref["max_alpha"])
            np.maximum(ref["max_weight"], r["max_weight"], out=ref["max_weight"])
            ref["in_frustum"] |= r["in_frustum"]
        print(f"  oracle: views {v0}..{v0 + 9} done ({time.time() - t0:.0f}s)", flush=True)
    ref["prune"] = ref["max_alpha"] < RP.alpha_min
    np.testing.assert_array_equal(infr, ref["in_frustum"])
    tie = ref["tie"] > 0
    ok = ~tie
    np.testing.assert_array_equal(h[ok], ref["hits"][ok])
    np.testing.assert_allclose(ma[ok], ref["max_alpha"][ok], rtol=0, atol=1e-5)
    np.testing.assert_allclose(mw[ok], ref["max_weight"][ok], rtol=0, atol=1e-5)
    np.testing.assert_array_equal(mask[ok], ref["prune"][ok])
    # surfels exposed to ties: each exposed entry can move the count by one
    assert np.all(np.abs(h[tie] - ref["hits"][tie]) <= ref["tie"][tie].astype(np.int64))
    sure = tie & (ref["hits"] > ref["tie"])
    assert not mask[sure].any()
    print(f"oracle statistics matched for {ok.sum()} surfels exactly; {tie.sum()} exposed to ties, within their "
          f"exposure counts ({(h[tie] != ref['hits'][tie]).sum()} differing)", flush=True)


def test_ragged16_regularizers_full_size():
    """The 2DGS terms of Eq. 3 on the full config-3 forward (16 views,
    16.6 Mpx): per-view losses against the oracle over whole views; the
    gradients on sampled crops (the oracle evaluated on the crop grown by the
    two-pixel reach of the depth normals, rescaled to the whole-view means),
    pixels whose depth normals are ill-conditioned in float32 reported apart."""
    from paper_2501_08174_amd import _lib
    from oracle.regularizers import regularizer_view64
    sc = scenes.make_ragged16_1m()
    run = gpu_run(sc)
    rast, views = run["rast"], run["views"]
    wd, wn = 1000.0, 0.05
    P, V = views.P, views.V
    dA = torch.zeros(P, device="cuda")
    dD, dN, dS = torch.zeros(P, device="cuda"), torch.zeros(3 * P, device="cuda"), torch.zeros(P, device="cuda")
    loss = rast.regularizer_loss(wd, wn, dA, dD, dN, dS).cpu().numpy()
    torch.cuda.synchronize()
    print("ragged16-1m regularisers: GPU pass done", flush=True)
    rng = np.random.default_rng(9)
    for v in range(V):
        pv = per_view(rast, v)
        L_d, L_n = regularizer_view64(pv["alpha"], pv["depth"], pv["normal"], pv["dist"], sc.cams[v])
        assert abs(loss[v] - float(L_d)) <= 1e-4 * abs(float(L_d)) + 1e-7, (v, loss[v], float(L_d))
        assert abs(loss[V + v] - float(L_n)) <= 1e-4 * abs(float(L_n)) + 1e-7, (v, loss[V + v], float(L_n))
    print("ragged16-1m regularisers: 16 per-view losses match", flush=True)
    dA, dD, dN, dS = (t.cpu().numpy() for t in (dA, dD, dN, dS))
    for v in (0, 7, 13):
        cam = sc.cams[v]
        W, H = cam.width, cam.height
        pv = per_view(rast, v)
        o, HW = views.pix_offsets[v], W * H
        for (x0, y0) in [(0, 0), (int(rng.integers(2, W - 50)), int(rng.integers(2, H - 50)))]:
            xe0, ye0, xe1, ye1 = max(x0 - 2, 0), max(y0 - 2, 0), min(x0 + 48 + 2, W), min(y0 + 48 + 2, H)
            sub = {k: (pv[k][..., ye0:ye1, xe0:xe1]) for k in ("alpha", "depth", "normal", "dist")}
            cs = scenes.Camera(viewmat=cam.viewmat, fx=cam.fx, fy=cam.fy, cx=cam.cx - xe0, cy=cam.cy - ye0,
                               width=xe1 - xe0, height=ye1 - ye0, campos=cam.campos)
            ref = oracle.regularizer_loss64([sub["alpha"]], [sub["depth"]], [sub["normal"]], [sub["dist"]], [cs],
                                            wd, wn)["grads"][0]
            k = (xe1 - xe0) * (ye1 - ye0) / (HW * V)      # crop mean -> whole-view mean over V views
            cy, cx = slice(y0 - ye0, y0 - ye0 + 48), slice(x0 - xe0, x0 - xe0 + 48)
            # conditioning of the depth normals the crop's gradients use
            Pts = oracle.depth_points64(sub["alpha"], sub["depth"], cs).numpy()
            a = np.zeros_like(Pts); b = np.zeros_like(Pts)
            a[1:-1, 1:-1] = Pts[2:, 1:-1] - Pts[:-2, 1:-1]
            b[1:-1, 1:-1] = Pts[1:-1, 2:] - Pts[1:-1, :-2]
            cond = np.linalg.norm(np.cross(a, b), axis=-1) / np.maximum(
                np.linalg.norm(a, axis=-1) * np.linalg.norm(b, axis=-1), 1e-30)
            # pixels on the image border have no depth normal on either side
            jj = np.arange(ye0, ye1)[:, None]; ii = np.arange(xe0, xe1)[None, :]
            interior = (ii >= 1) & (ii <= W - 2) & (jj >= 1) & (jj <= H - 2)
            inner_e = np.zeros(cond.shape, bool); inner_e[1:-1, 1:-1] = True
            bad = (cond < 1e-2) & interior & inner_e
            near = bad.copy()
            near[1:] |= bad[:-1]; near[:-1] |= bad[1:]; near[:, 1:] |= bad[:, :-1]; near[:, :-1] |= bad[:, 1:]
            keep = ~near[cy, cx]
            gy = np.arange(y0, y0 + 48)[:, None] * W + np.arange(x0, x0 + 48)[None, :]
            got = {"alpha": dA[o + gy], "depth": dD[o + gy], "dist": dS[o + gy],
                   "normal": np.stack([dN[3 * o + c * HW + gy] for c in range(3)])}
            for name in ("alpha", "depth", "dist", "normal"):
                r = ref[name][..., cy, cx] * k
                gg = got[name]
                if name == "normal":
                    r, gg = r[:, keep], gg[:, keep]
                else:
                    r, gg = r[keep], gg[keep]
                scale = np.abs(r).max()
                err = np.abs(gg - r).max() / max(scale, 1e-30)
                assert err <= 1e-3, (v, x0, y0, name, err)
            print(f"ragged16-1m view {v} crop ({x0},{y0}): gradients match; ill-conditioned pixels apart: "
                  f"{int((~keep).sum())}", flush=True)
