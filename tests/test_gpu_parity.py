"""Parity of the HIP path (through the C ABI) with the FP64 oracle on small
and ragged scenes: bit-exact binning, forward outputs within 1e-4, gradients
within 1e-3 relative, losses, pruning statistics, batched vs per-view."""
import numpy as np
import pytest
import torch

import oracle
from oracle.render import Params64, render_pixels
from paper_2501_08174_amd import scenes
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch, rasterize, prune_mask
from tests.gpu_helpers import (clamp_tie_ids, compare_binning, compare_forward, compare_grads, crop_pixels,
                               geometry, gpu_run, per_view)

pytestmark = pytest.mark.gpu

RP = oracle.RasterParams()
TIE_FRACTION = 1e-3     # largest fraction of compared pixels with a tie entry (each one still checked)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _full(cam):
    return crop_pixels(0, 0, cam.width, cam.height)


def _ragged_scene(seed=31, n=300, deg=0):
    return scenes.make_random_scene(seed, n, n_views=3, width=[61, 40, 17], height=[37, 64, 90],
                                    sh_degree=deg, scale_range=(0.02, 0.3))


# --------------------------------------------------------------------------
# binning
# --------------------------------------------------------------------------

def _wide_depth_scene():
    """Random scene plus surfels on view 0's optical axis from depth 0.25
    to 50000: visible depth keys spanning more than 2^27 (every byte of
    the key differs between the nearest and the farthest surfel)."""
    sc = scenes.make_random_scene(33, 2000, n_views=2, width=[100, 129], height=[77, 50], scale_range=(0.01, 0.3))
    depths = np.array([0.25, 0.3, 0.5, 20000.0, 35000.0, 50000.0])
    k = depths.size
    sc.means[:k] = np.stack([np.zeros(k), np.zeros(k), depths - 4.0], axis=1).astype(np.float32)
    sc.scales[:k] = np.stack([depths * 0.02, depths * 0.03], axis=1).astype(np.float32)
    sc.opac[:k] = 0.9
    return sc


@pytest.mark.parametrize("make", [lambda: _ragged_scene(), lambda: scenes.make_frame64_1k(),
                                  lambda: scenes.make_random_scene(32, 2000, n_views=2, width=[100, 129],
                                                                   height=[77, 50], scale_range=(0.01, 0.6)),
                                  _wide_depth_scene])
def test_binning_bit_exact(make):
    sc = make()
    run = gpu_run(sc, keys64=True)
    geoms = geometry(sc)
    keys = np.concatenate([g["depth_bits"][~g["culled"]] for g in geoms]).astype(np.int64)
    print(f"visible depth-key range {keys.max() - keys.min()}")
    if make is _wide_depth_scene:
        assert not geoms[0]["culled"][:6].any() and keys.max() - keys.min() >= (1 << 27)
    exempt = compare_binning(sc, run, geoms)
    print(f"binning exact; grid-tie exemptions: {exempt}")
    assert exempt == 0


def _projection_records(sc, n, shade):
    """Projection records (tiles, depth key, rectangle, geometry and, when
    shading, appearance) of the first n surfels of sc, projected alone."""
    views = ViewBatch(sc.cams)
    rast = Rasterizer(n, views, sc.sh_degree, sh_stride=sc.sh.shape[1], shade=shade)
    p = Params.from_scene(sc)
    p = Params(p.means[:n].contiguous(), p.scales[:n].contiguous(), p.quats[:n].contiguous(),
               p.opac[:n].contiguous(), p.sh[:n].contiguous())
    rast.preprocess(p)
    torch.cuda.synchronize()
    V = sc.v
    out = {"tiles": rast.tiles_touched[: V * n].cpu().numpy().view(np.uint32).reshape(V, n),
           "key": rast.depth_key[: V * n].cpu().numpy().view(np.uint32).reshape(V, n),
           "rect": rast.rect[: 4 * V * n].cpu().numpy().view(np.uint16).reshape(V, n, 4),
           "geom": rast.geom[: V * n * 16].cpu().numpy().view(np.uint32).reshape(V, n, 16),
           "in_frustum": rast.in_frustum[:n].cpu().numpy()}
    if shade:
        out["app"] = rast.app[: V * n * 8].cpu().numpy().view(np.uint32).reshape(V, n, 8)
    return out


@pytest.mark.parametrize("deg,shade", [(3, True), (1, True), (0, False)])
def test_projection_kernels_agree(deg, shade):
    """The projection has a one-thread-per-surfel kernel (looping over the
    views; batches of 196608 surfels and more) and a one-thread-per-(surfel,
    view) kernel (smaller batches; with four views its staged variant).
    The same surfels projected in a batch of 200003 and in a batch of their
    first 60001 give bit-identical records (every visible record's geometry
    and appearance too), and the large batch's binning records equal the
    oracle's."""
    sc = scenes.make_random_scene(71, 200_003, n_views=4, width=[333, 64, 1000, 500], height=[201, 999, 77, 500],
                                  sh_degree=deg, scale_range=(0.002, 0.05))
    big = _projection_records(sc, sc.n, shade)
    small = _projection_records(sc, 60_001, shade)
    m = 60_001
    for k in ("tiles", "key", "rect"):
        np.testing.assert_array_equal(big[k][:, :m], small[k], err_msg=k)
    vis = small["tiles"] != 0
    assert vis.sum() > 1000 and (~vis).sum() > 100, (vis.sum(), (~vis).sum())
    np.testing.assert_array_equal(big["geom"][:, :m][vis], small["geom"][vis])
    if shade:
        np.testing.assert_array_equal(big["app"][:, :m][vis], small["app"][vis])
    np.testing.assert_array_equal(big["in_frustum"][:m], small["in_frustum"])
    rp = oracle.RasterParams()
    for v, cam in enumerate(sc.cams):
        g = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp)
        ok = ~g["culled"]
        mism = (big["tiles"][v] != g["tiles_touched"]) | (ok & (big["key"][v] != g["depth_bits"])) | \
            (ok[:, None] & (big["rect"][v].astype(np.int64) != g["rect"])).any(axis=1)
        bad = mism & ~g["grid_tie"]
        assert not bad.any(), f"view {v}: {bad.sum()} records differ, e.g. {np.nonzero(bad)[0][:5]}"
        print(f"view {v}: {int(ok.sum())} visible of {sc.n}, grid-tie exemptions {int(mism.sum())}")
    np.testing.assert_array_equal(big["in_frustum"].astype(bool),
                                  np.any([big["tiles"][v] != 0 for v in range(sc.v)], axis=0))


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 8)])
def test_every_tile_shape_bins_and_renders(tile):
    """Binning bit-exact and forward parity for each compiled tile shape."""
    sc = _ragged_scene(38, 400, 3)
    rp = oracle.RasterParams(tile_w=tile[0], tile_h=tile[1])
    run = gpu_run(sc, keys64=True, tile=tile)
    geoms = geometry(sc, rp)
    assert compare_binning(sc, run, geoms, rp) == 0
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 3)
    ref = gpu_run(sc)
    for v, cam in enumerate(sc.cams):
        pix = _full(cam)
        res = render_pixels(P64, cam, geoms[v], pix, rp)
        errs, flagged, _ = compare_forward(per_view(run["rast"], v), res, pix, run["rast"], v,
                                           oracle_ctx=(P64, cam, geoms[v], rp))
        a, b = per_view(run["rast"], v), per_view(ref["rast"], v)
        # the blend order does not depend on the tile shape: identical images
        for k in ("color", "alpha", "depth", "normal", "dist", "T_final"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"{tile} view {v} {k}")


def _quat_of(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix (Shepperd's method)."""
    t = R[0, 0] + R[1, 1] + R[2, 2]
    if t > 0.0:
        s = 2.0 * np.sqrt(t + 1.0)
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif R[1, 1] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = 2.0 * np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    return np.array(q)


def _extreme_scene(seed=45):
    """Needles (scales 1000:1), surfels whose normal is perpendicular to
    view 0's ray through their centre (seen edge-on), sub-pixel surfels (the
    low-pass disc decides) and large ones: the most degenerate conics the
    per-wave culling bounds meet."""
    sc = scenes.make_random_scene(seed, 800, n_views=3, width=[70, 96, 33], height=[45, 64, 80],
                                  scale_range=(0.01, 0.3))
    rng = np.random.default_rng(seed)
    idx = rng.permutation(sc.means.shape[0])
    needle, edge, tiny, large = idx[:200], idx[200:400], idx[400:550], idx[550:600]
    sc.scales[needle] = np.stack([rng.uniform(0.1, 0.4, needle.size), rng.uniform(1e-4, 4e-4, needle.size)], 1)
    sc.scales[tiny] = rng.uniform(5e-5, 3e-4, (tiny.size, 2))
    sc.scales[large] = rng.uniform(0.4, 0.9, (large.size, 2))
    c0 = sc.cams[0].campos.astype(np.float64)
    for g in edge:
        d = sc.means[g].astype(np.float64) - c0
        d /= np.linalg.norm(d)
        nrm = np.cross(d, rng.normal(size=3))
        nrm /= np.linalg.norm(nrm)
        tu = np.cross(nrm, rng.normal(size=3))
        tu /= np.linalg.norm(tu)
        tv = np.cross(nrm, tu)
        R = np.stack([tu, tv, nrm], axis=1)
        q = _quat_of(R)
        assert np.allclose(np.stack([c[0] for c in oracle.rotation_columns64(q[None])], axis=1), R, atol=1e-12)
        sc.quats[g] = q
    return sc


@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_extreme_shapes_bin_and_render(tile):
    """Needles, edge-on, sub-pixel and large surfels: binning bit-exact and
    forward parity on whole frames (the per-wave culling must never drop an
    entry that blends)."""
    sc = _extreme_scene()
    rp = oracle.RasterParams(tile_w=tile[0], tile_h=tile[1])
    run = gpu_run(sc, keys64=True, tile=tile)
    geoms = geometry(sc, rp)
    assert compare_binning(sc, run, geoms, rp) == 0
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    ties, npix = 0, 0
    for v, cam in enumerate(sc.cams):
        pix = _full(cam)
        res = render_pixels(P64, cam, geoms[v], pix, rp)
        errs, flagged, rep = compare_forward(per_view(run["rast"], v), res, pix, run["rast"], v,
                                             oracle_ctx=(P64, cam, geoms[v], rp))
        print(f"{tile} view {v} errors {errs} tie pixels {flagged} taken the other way {len(rep['choice'])}")
        ties += flagged * pix.shape[0]
        npix += pix.shape[0]
    assert ties <= TIE_FRACTION * npix, (ties, npix)


# --------------------------------------------------------------------------
# forward
# --------------------------------------------------------------------------

def test_forward_frame64_full_frame():
    sc = scenes.make_frame64_1k()
    run = gpu_run(sc)
    geoms = geometry(sc)
    pix = _full(sc.cams[0])
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    res = render_pixels(P64, sc.cams[0], geoms[0], pix, RP)
    errs, flagged, rep = compare_forward(per_view(run["rast"], 0), res, pix, run["rast"], 0,
                                         oracle_ctx=(P64, sc.cams[0], geoms[0], RP))
    print("frame64-1k errors", errs, "tie pixels", flagged, "taken the other way", len(rep["choice"]))
    assert flagged <= TIE_FRACTION


def test_work_counts_match_oracle():
    """sr_render_count: blended pairs equal the oracle's per-pixel blend
    counts (pixels with a tie flag aside); the wave-step counts bound the
    pixel counts."""
    sc = _ragged_scene(41, 500, 0)
    run = gpu_run(sc)
    geoms = geometry(sc)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    nb, nb_flagged = 0, 0
    for v, cam in enumerate(sc.cams):
        res = render_pixels(P64, cam, geoms[v], _full(cam), RP)
        fl = res["flag_cut"] | res["flag_term"] | res["flag_clamp"]
        nb += int(res["nblend"][~fl].sum())
        nb_flagged += int(res["nblend"][fl].sum())
    R, B, WS, WB, RB = run["rast"].count_pairs(waves=True)
    upto = int(run["rast"].n_contrib[: run["views"].P].to(torch.int64).sum().item())
    print("reached", R, "blended", B, "oracle blended", nb, "+ flagged", nb_flagged, "wave steps", WS, WB,
          "backward pairs", RB, "list entries up to the last blend", upto)
    assert B >= nb
    if nb_flagged == 0:
        assert B == nb
    assert B <= R <= 64 * WS
    assert WB <= WS and B <= 64 * WB and WB > 0
    # the backward revisits the tested entries up to each pixel's last blend:
    # at least the blended ones, at most every list entry up to it
    assert B <= RB <= min(R, upto)


@pytest.mark.parametrize("deg", [0, 3])
def test_forward_multiview_ragged(deg):
    sc = _ragged_scene(33, 400, deg)
    run = gpu_run(sc)
    geoms = geometry(sc)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, deg)
    ties, npix = 0, 0
    for v, cam in enumerate(sc.cams):
        pix = _full(cam)
        res = render_pixels(P64, cam, geoms[v], pix, RP)
        errs, flagged, rep = compare_forward(per_view(run["rast"], v), res, pix, run["rast"], v,
                                             oracle_ctx=(P64, cam, geoms[v], RP))
        print(f"view {v} errors {errs} tie pixels {flagged} taken the other way {len(rep['choice'])}")
        ties += flagged * pix.shape[0]
        npix += pix.shape[0]
    assert ties <= TIE_FRACTION * npix, (ties, npix)


def test_batched_equals_per_view_bitwise():
    sc = _ragged_scene(34, 500, 3)
    run = gpu_run(sc)
    for v in range(sc.v):
        one = scenes.Scene(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree, [sc.cams[v]],
                           [sc.masks[v]])
        r1 = gpu_run(one)
        a, b = per_view(run["rast"], v), per_view(r1["rast"], 0)
        for k in ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"view {v} {k}")


# --------------------------------------------------------------------------
# backward
# --------------------------------------------------------------------------

def _weights(sc, rng):
    w = []
    for c in sc.cams:
        n = c.width * c.height
        w.append({"c": rng.normal(size=(n, 3)), "a": rng.normal(size=n), "d": rng.normal(size=n) * 0.3,
                  "n": rng.normal(size=(n, 3)), "s": rng.normal(size=n)})
    return w


def _gpu_grads(sc, w, tile=(16, 16), bwd_batch=0):
    views = ViewBatch(sc.cams, tile=tile)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1], bwd_batch=bwd_batch)
    p = Params.from_scene(sc)
    rast.plan_capacity(p)
    leaves = [t.clone().requires_grad_(True) for t in (p.means, p.scales, p.quats, p.opac, p.sh)]
    color, alpha, depth, normal, dist = rasterize(*leaves, rast)
    P = views.P
    gc = torch.zeros(3 * P, device="cuda")
    ga, gd, gn, gs = (torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda"),
                      torch.zeros(3 * P, device="cuda"), torch.zeros(P, device="cuda"))
    for v, c in enumerate(sc.cams):
        n = c.width * c.height
        o = views.pix_offsets[v]
        f = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
        gc[3 * o: 3 * (o + n)] = f(w[v]["c"].T.reshape(-1))
        gn[3 * o: 3 * (o + n)] = f(w[v]["n"].T.reshape(-1))
        ga[o: o + n] = f(w[v]["a"])
        gd[o: o + n] = f(w[v]["d"])
        gs[o: o + n] = f(w[v]["s"])
    L = (color * gc).sum() + (alpha * ga).sum() + (depth * gd).sum() + (normal * gn).sum() + (dist * gs).sum()
    L.backward()
    torch.cuda.synchronize()
    return [t.grad.cpu().numpy().astype(np.float64) for t in leaves], rast


def _oracle_grads(sc, w, geoms, rast):
    """Oracle autograd of the weighted sum of the five outputs over whole
    views, every tie taken the way the GPU took it (its forward outputs,
    still in ``rast``, against the oracle's correct results); returns the
    gradients and the surfels left out (entries at the alpha clamp, where
    the derivative in the opacity jumps)."""
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree, requires_grad=True)
    flagged = []
    for v, cam in enumerate(sc.cams):
        pix = _full(cam)
        res = render_pixels(P64, cam, geoms[v], pix, RP)
        _, frac, rep = compare_forward(per_view(rast, v), res, pix, rast, v, oracle_ctx=(P64, cam, geoms[v], RP))
        assert not rep["unresolved"]
        wt = {k: torch.tensor(a) for k, a in w[v].items()}

        def lf(out, rows, wt=wt):
            r = torch.as_tensor(rows)
            return ((out["color"] * wt["c"][r]).sum() + (out["alpha"] * wt["a"][r]).sum() +
                    (out["depth"] * wt["d"][r]).sum() + (out["normal"] * wt["n"][r]).sum() +
                    (out["dist"] * wt["s"][r]).sum())
        render_pixels(P64, cam, geoms[v], pix, RP, loss_fn=lf, flips=rep["choice"])
        flagged.append(clamp_tie_ids(res))
    return P64.grads(), np.unique(np.concatenate(flagged))


_compare_grads = compare_grads


@pytest.mark.parametrize("deg", [0, 3])
def test_backward_matches_oracle_autograd(deg):
    sc = scenes.make_random_scene(40 + deg, 150, n_views=2, width=[48, 37], height=[40, 51], sh_degree=deg,
                                  spread=0.6, scale_range=(0.03, 0.3))
    rng = np.random.default_rng(7)
    w = _weights(sc, rng)
    g, rast = _gpu_grads(sc, w)
    gref, excl = _oracle_grads(sc, w, geometry(sc), rast)
    print("surfels left out (an entry at the alpha clamp):", len(excl))
    compare_grads(g, gref, excl)


def test_extreme_shapes_gradients():
    """The backward on the needle / edge-on / sub-pixel / large scene against
    the oracle's autograd at the gradient bar: the culling bits the backward
    reads and the pair gradients near degenerate conics."""
    sc = _extreme_scene()
    w = _weights(sc, np.random.default_rng(9))
    g, rast = _gpu_grads(sc, w)
    gref, excl = _oracle_grads(sc, w, geometry(sc), rast)
    print("surfels left out (an entry at the alpha clamp):", len(excl))
    compare_grads(g, gref, excl)


# every compiled (tile shape, backward LDS batch)
BWD_VARIANTS = ([((16, 16), b) for b in (32, 64, 128, 256)] + [((32, 8), b) for b in (32, 64, 128, 256)] +
                [((16, 8), b) for b in (32, 64, 128)] + [((8, 8), b) for b in (32, 64)])


@pytest.fixture(scope="module")
def _bwd_case():
    """A scene, upstream weights of all five outputs and the oracle's
    gradients (ties taken as the GPU's forward took them: the forward does
    not depend on the tile shape or the batch)."""
    sc = scenes.make_random_scene(46, 200, n_views=2, width=[48, 37], height=[40, 51], sh_degree=3,
                                  spread=0.6, scale_range=(0.03, 0.3))
    w = _weights(sc, np.random.default_rng(8))
    _, rast = _gpu_grads(sc, w)
    gref, excl = _oracle_grads(sc, w, geometry(sc), rast)
    return sc, w, gref, excl


@pytest.mark.parametrize("tile,batch", BWD_VARIANTS, ids=[f"{t[0]}x{t[1]}-b{b}" for t, b in BWD_VARIANTS])
def test_backward_every_lds_batch(_bwd_case, tile, batch):
    """The backward compositing with every compiled LDS batch and tile shape
    (the autotuner's search space) against the oracle's gradients."""
    from paper_2501_08174_amd import _lib
    assert _lib.lib().sr_bwd_batch_supported(tile[0], tile[1], batch) == 1
    sc, w, gref, excl = _bwd_case
    g, _ = _gpu_grads(sc, w, tile=tile, bwd_batch=batch)
    compare_grads(g, gref, excl)


def test_gradient_marks():
    """The compositing backward marks (bit 31 of tiles_touched) exactly the
    records it gives a gradient; the projection backward with the marks
    reads only those, clears the marks and the accumulator, and gives the
    gradients of the unmarked read of every record."""
    import ctypes
    from paper_2501_08174_amd import _lib
    from paper_2501_08174_amd._lib import SrConfig
    from paper_2501_08174_amd.raster import _ptr
    # large surfels: about half of the visible records are occluded everywhere
    sc = scenes.make_random_scene(47, 3000, n_views=3, width=[90, 64, 120], height=[70, 100, 33], sh_degree=3,
                                  scale_range=(0.05, 0.4))
    rng = np.random.default_rng(48)
    views = ViewBatch(sc.cams)
    mask = torch.tensor(rng.integers(0, 2, views.P).astype(np.uint8), device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    p = Params.from_scene(sc)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    rast.plan_capacity(p)
    VN = sc.v * sc.n

    def step(marked):
        g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
        rast.preprocess(p)
        rast.bin()
        rast.train_step_raster(mask, target, 0.5, 1.0, schedule=False)
        torch.cuda.synchronize()
        tt = rast.tiles_touched[:VN].cpu().numpy().view(np.uint32).copy()
        rec = rast.grad_rec[: VN * _lib.SR_GRAD_STRIDE].cpu().numpy().reshape(VN, -1)
        has = (rec != 0).any(axis=1)
        if marked:
            rast.backward_project(p, g)
        else:
            cfg = SrConfig.from_buffer_copy(rast.cfg)
            _lib.call("sr_backward_project", rast.ctx.ptr, ctypes.byref(cfg), rast.N, views.V, views.host_ptr,
                      _ptr(views.dev), _ptr(p.means), _ptr(p.scales), _ptr(p.quats), _ptr(p.sh), _ptr(rast.geom),
                      _ptr(rast.app), _ptr(rast.tiles_touched), _ptr(rast.grad_rec), _ptr(g.means),
                      _ptr(g.scales), _ptr(g.quats), _ptr(g.opac), _ptr(g.sh), None, None, None)
        torch.cuda.synchronize()
        after = rast.tiles_touched[:VN].cpu().numpy().view(np.uint32)
        return tt, has, after, [t.cpu().numpy() for t in (g.means, g.scales, g.quats, g.opac, g.sh)]

    tt, has, after, g_marked = step(True)
    marks = (tt >> 31) == 1
    np.testing.assert_array_equal(marks, has)
    unmarked_visible = int((~has & ((tt & 0x7FFFFFFF) != 0)).sum())
    assert has.sum() > 1000 and unmarked_visible > 1000, (int(has.sum()), unmarked_visible)
    np.testing.assert_array_equal(after, tt & 0x7FFFFFFF)
    assert not rast.grad_rec.any().item()
    tt2, has2, after2, g_all = step(False)
    np.testing.assert_array_equal(has2, has)
    np.testing.assert_array_equal(after2, tt2)          # the unmarked read leaves the marks
    for a, b in zip(g_marked, g_all):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-5 * max(float(np.abs(b).max()), 1e-30))
    print(f"{int(has.sum())} of {int(((tt & 0x7FFFFFFF) != 0).sum())} visible records hold gradients")


def test_large_surfels_across_tile_groups():
    """Surfels whose rectangles span many 4x4-tile groups next to small ones,
    on views whose tile grids are not multiples of the group: bit-exact
    grouped binning, forward outputs and parameter gradients."""
    sc = scenes.make_random_scene(47, 160, n_views=2, width=[150, 97], height=[130, 111], spread=0.8,
                                  scale_range=(0.05, 1.5))
    geoms = geometry(sc)
    run = gpu_run(sc, keys64=True)
    compare_binning(sc, run, geoms)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree)
    for v, cam in enumerate(sc.cams):
        pix = _full(cam)
        res = render_pixels(P64, cam, geoms[v], pix, RP)
        errs, flagged, _ = compare_forward(per_view(run["rast"], v), res, pix, run["rast"], v,
                                           oracle_ctx=(P64, cam, geoms[v], RP))
        print(f"view {v} errors {errs} tie pixels {flagged}")
    # some entries cover several groups, and some groups hold entries of many tiles
    rast = run["rast"]
    vals = rast.vals[: run["status"][2]].cpu().numpy().view(np.uint32)
    sub = vals >> np.uint32(24)
    spans = ((sub >> 2) & 3) - (sub & 3) + 1
    assert (spans == 4).any() and (spans == 1).any()
    rng = np.random.default_rng(8)
    w = _weights(sc, rng)
    g, rast = _gpu_grads(sc, w)
    gref, excl = _oracle_grads(sc, w, geoms, rast)
    print("surfels left out (an entry at the alpha clamp):", len(excl))
    compare_grads(g, gref, excl)


# --------------------------------------------------------------------------
# losses (Eq. 1, Eq. 2)
# --------------------------------------------------------------------------

def test_background_and_masked_l1_loss():
    sc = _ragged_scene(35, 300, 0)
    run = gpu_run(sc)
    rast = run["rast"]
    views = rast.views
    rng = np.random.default_rng(3)
    masks = [rng.integers(0, 2, size=(c.height, c.width)).astype(np.uint8) for c in sc.cams]
    targets = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cams]
    mask = torch.tensor(np.concatenate([m.reshape(-1) for m in masks]), device="cuda")
    target = torch.tensor(np.concatenate([t.reshape(-1) for t in targets]), device="cuda")
    dA = torch.zeros_like(rast.alpha)
    dC = torch.zeros_like(rast.color)
    loss = rast.loss(mask, target, gamma=0.5, w_c=1.0, dL_dalpha=dA, dL_dcolor=dC)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    V = sc.v
    tot = 0.0
    for v, c in enumerate(sc.cams):
        pv = per_view(rast, v)
        lb = oracle.background_loss64(pv["alpha"], masks[v])
        l1 = oracle.masked_l1_64(pv["color"], targets[v], masks[v])
        assert abs(loss[v] - lb) <= 1e-6 * max(1, lb)
        assert abs(loss[V + v] - l1) <= 1e-6 * max(1, l1)
        tot += (l1 + 0.5 * lb) / V
        HW = c.width * c.height
        o = views.pix_offsets[v]
        np.testing.assert_allclose(dA[o:o + HW].cpu().numpy(), 0.5 * (1 - masks[v].reshape(-1)) / (HW * V),
                                   rtol=1e-6)
        d = pv["color"] * masks[v][None] - targets[v] * masks[v][None]
        np.testing.assert_allclose(dC[3 * o:3 * (o + HW)].cpu().numpy(), (np.sign(d) / (3 * HW * V)).reshape(-1),
                                   rtol=1e-6)
    assert abs(loss[2 * V] - tot) <= 1e-6


# --------------------------------------------------------------------------
# occlusion-aware pruning (Section 4.3)
# --------------------------------------------------------------------------

def test_prune_stats_match_oracle():
    sc = _ragged_scene(36, 600, 0)
    run = gpu_run(sc, stats=True)
    hits, ma, mw = (t.cpu().numpy() for t in run["stats"])
    geoms = geometry(sc)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    pairs, tie_ids = [], []
    for v, cam in enumerate(sc.cams):
        res = render_pixels(P64, cam, geoms[v], _full(cam), RP)
        pairs.append(res["pairs"])
        tie_ids.append(res["tie_ids"])
    st = oracle.prune_stats64(sc.n, pairs, [g["culled"] for g in geoms])
    keep = np.ones(sc.n, bool)
    keep[np.unique(np.concatenate(tie_ids))] = False  # surfels at a tie entry
    np.testing.assert_array_equal(hits.view(np.uint32)[keep], st["hits"][keep])
    np.testing.assert_allclose(ma[keep], st["max_alpha"][keep], atol=1e-5)
    np.testing.assert_allclose(mw[keep], st["max_weight"][keep], atol=1e-5)
    mask = prune_mask(run["stats"][1]).cpu().numpy().astype(bool)
    np.testing.assert_array_equal(mask[keep], st["prune"][keep])
    inf = run["rast"].in_frustum[: sc.n].cpu().numpy().astype(bool)
    np.testing.assert_array_equal(inf, st["in_frustum"])
    print(f"pruned {mask.sum()} of {sc.n}; exempt {(~keep).sum()}")


def test_usage_counts_alone():
    """hits alone (no maxima): the usage record of Section 4.3 taken in the
    forward and in the fused training step equals the full statistics' hits
    and the oracle's, accumulates across calls, and leaves every forward
    output bit-identical."""
    sc = _ragged_scene(36, 600, 0)
    geoms = geometry(sc)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    pairs, tie_ids = [], []
    for v, cam in enumerate(sc.cams):
        res = render_pixels(P64, cam, geoms[v], _full(cam), RP)
        pairs.append(res["pairs"])
        tie_ids.append(res["tie_ids"])
    ref = oracle.prune_stats64(sc.n, pairs, [g["culled"] for g in geoms])
    keep = np.ones(sc.n, bool)
    keep[np.unique(np.concatenate(tie_ids))] = False
    views = ViewBatch(sc.cams)
    rng = np.random.default_rng(4)
    masks = torch.tensor(np.concatenate([rng.integers(0, 2, c.width * c.height) for c in sc.cams]).astype(np.uint8),
                         device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    p = Params.from_scene(sc)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    rast.plan_capacity(p)
    rast.preprocess(p)
    rast.bin()
    outs = ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib")
    for fused in (False, True):
        full = (torch.zeros(sc.n, dtype=torch.int32, device="cuda"), torch.zeros(sc.n, device="cuda"),
                torch.zeros(sc.n, device="cuda"))
        hits = torch.full((sc.n,), 7, dtype=torch.int32, device="cuda")     # cleared by the call
        res = []
        for st in (full, hits):
            if fused:
                rast.train_step_raster(masks, target, 0.5, 1.0, stats=st)
            else:
                rast.forward(stats=st)
            torch.cuda.synchronize()
            res.append({k: getattr(rast, k).clone() for k in outs})
        for k in outs:
            assert torch.equal(res[0][k], res[1][k]), (fused, k)
        h = hits.cpu().numpy()
        np.testing.assert_array_equal(h, full[0].cpu().numpy())
        np.testing.assert_array_equal(h.view(np.uint32)[keep], ref["hits"][keep])
        # accumulate: a second call adds the same counts
        if fused:
            rast.train_step_raster(masks, target, 0.5, 1.0, stats=hits, accumulate=True)
        else:
            rast.forward(stats=hits, accumulate=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(hits.cpu().numpy(), 2 * h)
    print(f"used {(h > 0).sum()} of {sc.n}; exempt {(~keep).sum()}")


def test_cost_ordered_dispatch():
    """The fused step records each tile's cost (the largest n_contrib of its
    pixels); sr_tile_order sorts the tiles by descending cost, equal costs by
    ascending id; launched in that order the step gives bit-identical forward
    outputs, usage counts and losses, and the gradients up to the rounding
    order of float atomics."""
    sc = scenes.make_random_scene(44, 4000, n_views=3, width=[150, 97, 64], height=[80, 121, 64], sh_degree=3,
                                  scale_range=(0.01, 0.4))
    rng = np.random.default_rng(6)
    views = ViewBatch(sc.cams)
    mask = torch.tensor(rng.integers(0, 2, views.P).astype(np.uint8), device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    p = Params.from_scene(sc)
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    grads = (g.means, g.scales, g.quats, g.opac, g.sh)
    hits = torch.zeros(sc.n, dtype=torch.int32, device="cuda")
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    rast.plan_capacity(p)
    outs = ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib")

    def run(schedule):
        for t in grads:
            t.zero_()
        rast.preprocess(p)
        rast.bin()
        loss = rast.train_step_raster(mask, target, 0.5, 1.0, stats=hits, schedule=schedule)
        rast.backward_project(p, g)
        torch.cuda.synchronize()
        return ({k: getattr(rast, k).clone() for k in outs}, hits.clone(), loss.clone(), [t.clone() for t in grads])

    ref = run(False)
    run(True)                                   # first scheduled call: default order, costs recorded
    T = views.T
    cost = rast.tile_cost.cpu().numpy().astype(np.int64)
    ncon = rast.n_contrib[: views.P].cpu().numpy().astype(np.int64)
    want = np.zeros(T, np.int64)
    for v in range(views.V):
        c = views.host[v]
        img = ncon[c.pix_offset: c.pix_offset + c.width * c.height].reshape(c.height, c.width)
        for ty in range(c.tiles_y):
            for tx in range(c.tiles_x):
                want[c.tile_offset + ty * c.tiles_x + tx] = img[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].max()
    np.testing.assert_array_equal(cost, want)
    assert len(np.unique(cost)) > 3
    got = run(True)                             # ordered by the recorded costs
    order = rast.tile_order.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(order, np.lexsort((np.arange(T), -_cost_class(cost))))
    for k in outs:
        assert torch.equal(got[0][k], ref[0][k]), k
    assert torch.equal(got[1], ref[1])
    assert torch.equal(got[2], ref[2])
    for x, y in zip(got[3], ref[3]):
        assert float((x - y).abs().max().item()) <= 1e-5 * float(y.abs().max().item()) + 1e-12
    print(f"{T} tiles, costs {cost.min()}..{cost.max()}, heaviest first: {order[:5].tolist()}")

    # the separate launches: the forward records the same costs, forward and
    # backward launch in the order of the last recorded costs; the backward
    # also with depth, normal and distortion gradients (the Eq. 3 path)
    P = views.P
    rg = np.random.default_rng(16)
    dD = torch.tensor(rg.normal(size=P).astype(np.float32), device="cuda")
    dN = torch.tensor(rg.normal(size=3 * P).astype(np.float32), device="cuda")
    dS = torch.tensor(rg.normal(size=P).astype(np.float32), device="cuda")

    def run_sep(schedule, geo=False):
        for t in grads:
            t.zero_()
        rast.preprocess(p)
        rast.bin()
        rast.forward(stats=hits, schedule=schedule)
        dA = torch.zeros_like(rast.alpha)
        dC = torch.zeros_like(rast.color)
        loss = rast.loss(mask, target, 0.5, 1.0, dA, dC)
        if geo:
            rast.backward_raster(dC=dC, dA=dA, dD=dD, dN=dN, dS=dS, schedule=schedule)
        else:
            rast.backward_raster(dC=dC, dA=dA, schedule=schedule)
        rast.backward_project(p, g)
        torch.cuda.synchronize()
        order = None if rast.last_order is None else rast.last_order.cpu().numpy().astype(np.int64)
        return ({k: getattr(rast, k).clone() for k in outs}, hits.clone(), loss.clone(), [t.clone() for t in grads],
                order)

    for geo in (False, True):
        ref_sep = run_sep(False, geo)
        run_sep(True, geo)                          # records this forward's costs
        got_sep = run_sep(True, geo)                # launched in the order of those costs
        order = got_sep[4]
        assert order is not None and not np.array_equal(order, np.arange(T))
        np.testing.assert_array_equal(np.sort(order), np.arange(T))
        np.testing.assert_array_equal(order, np.lexsort((np.arange(T), -_cost_class(want))))
        np.testing.assert_array_equal(rast.tile_cost.cpu().numpy().astype(np.int64), want)
        for k in outs:
            assert torch.equal(got_sep[0][k], ref_sep[0][k]), k
            assert torch.equal(got_sep[0][k], ref[0][k]), k      # separate and fused forwards agree
        assert torch.equal(got_sep[1], ref_sep[1])
        assert torch.equal(got_sep[2], ref_sep[2])
        for x, y in zip(got_sep[3], ref_sep[3]):
            assert float((x - y).abs().max().item()) <= 1e-5 * float(y.abs().max().item()) + 1e-12
        print(f"separate launches{' with depth/normal/distortion gradients' if geo else ''}: ordered "
              f"forward and backward match the default order")


def _cost_class(c):
    """The logarithmic cost class of sr_tile_order, written out: c below 16,
    above that 16 classes per octave."""
    c = np.asarray(c, dtype=np.int64)
    e = np.floor(np.log2(np.maximum(c, 1))).astype(np.int64)
    # the float log2 of a 32-bit integer is exact enough to give its msb, but
    # check it against the integer definition
    assert np.all((c < 16) | ((1 << e) <= c) & (c < (1 << (e + 1))))
    return np.where(c < 16, c, (e - 3) * 16 + ((c >> np.maximum(e - 4, 0)) & 15))


def test_tile_order_sort_edge_cases():
    """sr_tile_order alone: a ragged tile count (not a multiple of any block
    size), many equal costs, large costs; the order equals numpy's stable
    sort by descending cost class."""
    import ctypes
    from paper_2501_08174_amd import _lib
    from paper_2501_08174_amd.raster import _ctx
    rng = np.random.default_rng(12)
    for T in (1, 7, 100003):
        cost = rng.integers(0, 40, size=T).astype(np.int64)           # many ties
        big = rng.random(T) < 0.01
        cost[big] = rng.integers(1 << 4, 1 << 32, size=int(big.sum()))   # up to the full 32 bits
        n = ctypes.c_size_t(0)
        _lib.call("sr_tile_order_workspace_size", T, ctypes.byref(n))
        ws = torch.zeros(max(n.value, 1), dtype=torch.uint8, device="cuda")
        c = torch.tensor(cost.astype(np.uint32).view(np.int32), device="cuda")
        out = torch.full((T,), -1, dtype=torch.int32, device="cuda")
        _lib.call("sr_tile_order", _ctx(c), T, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64),
                                      np.lexsort((np.arange(T), -_cost_class(cost))))
    _lib.call("sr_tile_order", _ctx(c), 0, None, None, 0, None, None)      # empty: a no-op


def test_prune_pass_culling_keeps_statistics():
    """sr_prune_contrib (no shading) with per-wave culling by the pixel
    rectangles, without it, and the statistics of the shaded forward: the
    same hits and maxima (the oracle's tie surfels aside)."""
    sc = _ragged_scene(37, 600, 0)
    run = gpu_run(sc, stats=True)
    ref = [t.cpu().numpy() for t in run["stats"]]
    views = ViewBatch(sc.cams)
    rast = Rasterizer(sc.n, views, 0, shade=False)
    p = Params.from_scene(sc)
    rast.plan_capacity(p)
    rast.preprocess(p)
    rast.bin()
    rast.check_capacity()
    out = {}
    for cull in (True, False):
        st = (torch.zeros(sc.n, dtype=torch.int32, device="cuda"), torch.zeros(sc.n, device="cuda"),
              torch.zeros(sc.n, device="cuda"))
        rast.prune_stats(*st, cull=cull)
        out[cull] = [t.cpu().numpy() for t in st]
    geoms = geometry(sc)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    tie_ids = [render_pixels(P64, cam, geoms[v], _full(cam), RP)["tie_ids"] for v, cam in enumerate(sc.cams)]
    keep = np.ones(sc.n, bool)
    keep[np.unique(np.concatenate(tie_ids))] = False
    for cull in (True, False):
        for a, b in zip(out[cull], ref):
            np.testing.assert_array_equal(a[keep], b[keep])
    assert (ref[0] > 0).sum() > 50


def test_prune_occluded_surfel_scene():
    from tests.oracle_scenes import front_camera, scene_from
    ID = [1.0, 0.0, 0.0, 0.0]
    cam = front_camera(40)
    means = [[0, 0, 0.0], [0, 0, 0.05], [0, 0, 0.1], [0, 0, 0.5], [0, 0, -5.0], [30.0, 0, 0.5],
             [0.2, 0.1, -0.5]]
    sc = scene_from(means, [(5, 5)] * 3 + [(0.2, 0.2)] * 4, [ID] * 7, [0.99, 0.99, 0.99, 0.9, 0.9, 0.9, 0.002],
                    [(1, 1, 1)] * 7, [cam])
    run = gpu_run(sc, stats=True)
    hits = run["stats"][0].cpu().numpy()
    inf = run["rast"].in_frustum[:7].cpu().numpy()
    assert list(inf) == [1, 1, 1, 1, 0, 0, 0]
    assert all(hits[:3] > 0) and hits[3] == 0 and all(hits[4:] == 0)


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

def test_edge_cases_empty_and_tiny():
    from tests.oracle_scenes import front_camera, scene_from
    ID = [1.0, 0.0, 0.0, 0.0]
    # every surfel culled: background everywhere, no instances
    cam = front_camera(20)
    cam.bg = np.array([0.25, 0.5, 0.75], np.float32)
    sc = scene_from([[0, 0, -6.0], [0, 0, -4.1]], [(0.1, 0.1)] * 2, [ID] * 2, [0.9, 0.9], [(1, 1, 1)] * 2, [cam])
    run = gpu_run(sc, capacity=16)
    pv = per_view(run["rast"], 0)
    assert run["status"] == (0, 0, 0, 0)
    assert np.all(pv["alpha"] == 0) and np.all(pv["n_contrib"] == 0)
    np.testing.assert_array_equal(pv["color"], np.broadcast_to(cam.bg[:, None, None], pv["color"].shape))
    # 1x1 and 1xH views next to a regular one
    sc = scenes.make_random_scene(37, 50, n_views=3, width=[1, 1, 33], height=[1, 29, 18],
                                  scale_range=(0.1, 0.5))
    run = gpu_run(sc, keys64=True)
    compare_binning(sc, run, geometry(sc))


def test_capacity_overflow_flags_outputs():
    """A binning over its capacity sets the context's status word: the
    compositing calls after it compute nothing and flag their outputs
    (forward and fused step: NaN images and losses, n_contrib 0, no
    statistics, no gradients; the prune mask prunes nothing);
    sr_read_status reports SR_ERR_CAPACITY with the instance count needed
    and clears the word; re-planned, the same rasterizer renders exactly as
    a fresh one."""
    import ctypes
    from paper_2501_08174_amd import _lib
    from paper_2501_08174_amd.raster import _ptr, _stream
    sc = _ragged_scene(39, 500, 3)
    n = sc.n
    views = ViewBatch(sc.cams)
    rast = Rasterizer(n, views, 3, sh_stride=16)
    p = Params.from_scene(sc)
    need = rast.plan_capacity(p)
    assert need > 200
    rast.set_capacity(100)
    rast.preprocess(p)
    rast.bin()
    vis, need2, stored, st = rast.status()
    assert st == 1 and stored == 100 and need2 == need
    outs = ("color", "alpha", "depth", "normal", "dist", "T_final")
    stats = (torch.full((n,), 5, dtype=torch.int32, device="cuda"), torch.ones(n, device="cuda"),
             torch.ones(n, device="cuda"))
    rast.forward(stats=stats)
    torch.cuda.synchronize()
    for k in outs:
        assert torch.isnan(getattr(rast, k)[: views.P * (3 if k in ("color", "normal") else 1)]).all(), k
    assert int(rast.n_contrib[: views.P].abs().max().item()) == 0
    assert all(float(t.abs().max().item()) == 0 for t in stats)          # cleared, nothing added
    rng = np.random.default_rng(10)
    mask = torch.tensor(rng.integers(0, 2, views.P).astype(np.uint8), device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    loss = rast.train_step_raster(mask, target, 0.5, 1.0, stats=stats[0])
    rast.backward_project(p, g)
    dC = torch.ones_like(rast.color)
    rast.backward_raster(dC=dC, dA=torch.ones_like(rast.alpha))
    rast.backward_project(p, g)
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    _lib.call("sr_prune_mask", rast.ctx.ptr, n, _ptr(stats[1]), float(1 / 255), _ptr(out), _stream())
    torch.cuda.synchronize()
    assert torch.isnan(loss).all()
    assert torch.isnan(rast.alpha[: views.P]).all()
    assert all(float(t.abs().max().item()) == 0 for t in (g.means, g.scales, g.quats, g.opac, g.sh))
    assert int(stats[0].abs().max().item()) == 0 and int(out.max().item()) == 0
    bits, needed = rast.ctx.read_status(clear=False)
    assert bits == _lib.SR_STATUS_CAPACITY and needed == need
    with pytest.raises(_lib.SurfelRasterError) as e:
        rast.check_capacity()
    assert e.value.code == _lib.SR_ERR_CAPACITY and str(need) in str(e.value)
    assert rast.ctx.read_status() == (0, 0)
    # re-planned: identical to a fresh rasterizer
    rast.set_capacity(need + 1024)
    rast.preprocess(p)
    rast.bin()
    rast.forward()
    torch.cuda.synchronize()
    ref = gpu_run(sc)["rast"]
    for k in outs + ("n_contrib",):
        assert torch.equal(getattr(rast, k), getattr(ref, k)), k


def test_prune_pass_chunks_accumulation_and_overflow():
    """sr_prune_contrib, the whole pass: the same statistics, in-frustum
    flags and mask for any number of views per chunk and as the stage calls
    (projection, binning, sr_prune_stats over all views at once);
    in_frustum equals the oracle's; accumulation over two calls doubles the
    counts and keeps the maxima; a capacity below the need sets the status
    word and leaves the mask all zero."""
    import ctypes
    from paper_2501_08174_amd import _lib
    from paper_2501_08174_amd.raster import PruneStats, _ptr, _stream, make_config, prune_contrib
    sc = _ragged_scene(36, 600, 0)
    sc.opac[:40] = 0.002            # below the cutoff everywhere: culled, never blended, pruned
    n = sc.n
    p = Params.from_scene(sc)
    runs = {vpc: prune_contrib(p, sc.cams, views_per_chunk=vpc) for vpc in (1, 2, 3)}
    views = ViewBatch(sc.cams)
    rast = Rasterizer(n, views, 0, shade=False)
    rast.plan_capacity(p)
    rast.preprocess(p)
    rast.bin()
    ref = (torch.zeros(n, dtype=torch.int32, device="cuda"), torch.zeros(n, device="cuda"),
           torch.zeros(n, device="cuda"))
    rast.prune_stats(*ref)
    rast.check_capacity()
    geoms = geometry(sc)
    inf_oracle = np.zeros(n, bool)
    for gm in geoms:
        inf_oracle |= ~gm["culled"]
    for vpc, st in runs.items():
        for a, b in zip((st.hits, st.max_alpha, st.max_weight), ref):
            assert torch.equal(a, b), vpc
        np.testing.assert_array_equal(st.in_frustum.cpu().numpy().astype(bool), inf_oracle)
        np.testing.assert_array_equal(st.mask.cpu().numpy().astype(bool), ref[0].cpu().numpy() == 0)
    assert (ref[0] > 0).sum() > 50 and (ref[0][:40] == 0).all() and not inf_oracle[:40].any()
    acc = prune_contrib(p, sc.cams, views_per_chunk=2, stats=runs[1])
    torch.cuda.synchronize()
    assert torch.equal(acc.hits, 2 * ref[0]) and torch.equal(acc.max_alpha, ref[1])
    np.testing.assert_array_equal(acc.in_frustum.cpu().numpy().astype(bool), inf_oracle)
    # overflow: capacity 10 for every chunk
    ctx = _lib.Context(torch.cuda.current_device())
    cfg = make_config(0, None, views.tile)
    b = ctypes.c_size_t(0)
    _lib.call("sr_prune_workspace_size", ctypes.byref(cfg), _lib.SR_PRIM_SURFEL, n, views.V, views.host_ptr, 2, 10,
              ctypes.byref(b))
    ws = torch.zeros(b.value, dtype=torch.uint8, device="cuda")
    st = PruneStats(*[torch.zeros(n, dtype=dt, device="cuda") for dt in (torch.int32, torch.float32, torch.float32,
                                                                         torch.uint8, torch.uint8)])
    _lib.call("sr_prune_contrib", ctx.ptr, ctypes.byref(cfg), _lib.SR_PRIM_SURFEL, n, _ptr(p.means), _ptr(p.scales),
              _ptr(p.quats), _ptr(p.opac), views.V, views.host_ptr, _ptr(views.dev), 2, float(1 / 255), 10, _ptr(ws),
              b.value, _ptr(st.hits), _ptr(st.max_alpha), _ptr(st.max_weight), _ptr(st.in_frustum), _ptr(st.mask),
              _stream())
    bits, needed = ctx.read_status()
    assert bits == _lib.SR_STATUS_CAPACITY and needed > 10
    assert int(st.mask.max().item()) == 0 and int(st.hits.max().item()) == 0


# --------------------------------------------------------------------------
# fused training step vs the separate calls
# --------------------------------------------------------------------------

def test_fused_train_step_matches_separate_calls():
    """sr_train_step_raster = sr_render_forward (+statistics) +
    sr_background_loss + sr_backward_raster, in one launch: identical forward
    outputs and statistics, equal losses and gradients (atomic order aside)."""
    sc = _ragged_scene(39, 500, 3)
    rng = np.random.default_rng(9)
    views = ViewBatch(sc.cams)
    masks = torch.tensor(np.concatenate([rng.integers(0, 2, c.width * c.height) for c in sc.cams]).astype(np.uint8),
                         device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    p = Params.from_scene(sc)
    out = []
    for fused in (False, True):
        rast = Rasterizer(sc.n, views, 3, sh_stride=16)
        rast.plan_capacity(p)
        rast.preprocess(p)
        rast.bin()
        st = (torch.zeros(sc.n, dtype=torch.int32, device="cuda"), torch.zeros(sc.n, device="cuda"),
              torch.zeros(sc.n, device="cuda"))
        g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
        if fused:
            loss = rast.train_step_raster(masks, target, 0.5, 1.0, stats=st)
        else:
            rast.forward(stats=st)
            dA = torch.zeros_like(rast.alpha)
            dC = torch.zeros_like(rast.color)
            loss = rast.loss(masks, target, 0.5, 1.0, dA, dC)
            rast.backward_raster(dC=dC, dA=dA)
        rast.backward_project(p, g)
        torch.cuda.synchronize()
        out.append(dict(fwd={k: getattr(rast, k).cpu().numpy() for k in
                             ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib")},
                        stats=[t.cpu().numpy() for t in st], loss=loss.cpu().numpy().copy(),
                        grads=[t.cpu().numpy().astype(np.float64) for t in (g.means, g.scales, g.quats, g.opac,
                                                                             g.sh)]))
    a, b = out
    for k in a["fwd"]:
        np.testing.assert_array_equal(a["fwd"][k], b["fwd"][k], err_msg=k)
    for x, y in zip(a["stats"], b["stats"]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_allclose(a["loss"], b["loss"], rtol=1e-5, atol=1e-7)
    for x, y in zip(a["grads"], b["grads"]):
        np.testing.assert_allclose(x, y, rtol=1e-4, atol=1e-6 * np.abs(y).max())
