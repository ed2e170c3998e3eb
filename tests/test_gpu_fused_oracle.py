"""The fused training step (sr_train_step_raster: forward, occlusion
statistics, masked L1 + background loss gradients and backward in one
launch) against the FP64 oracle: forward outputs under the tie protocol,
per-view losses (Eq. 1, Eq. 2), the statistics of Section 4.3 and all five
parameter gradients.  At the full benchmark sizes the step runs on whole
views with the loss restricted to a 64x64 crop through the mask (every
non-zero upstream gradient inside the crop), so the oracle renders only
the crop."""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle.render import Params64, render_pixels
from paper_2501_08174_amd import scenes
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch
from tests.gpu_helpers import (clamp_tie_ids, compare_forward, compare_grads, crop_pixels, masked_loss_fn,
                               masked_terms, per_view)
from tests.test_gpu_parity import BWD_VARIANTS, _extreme_scene

pytestmark = pytest.mark.gpu
RP = oracle.RasterParams()
TIE_FRACTION = 1e-3     # largest fraction of compared pixels with a tie entry


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _fused(sc, masks, targets, gamma, w_c, level, tile=(16, 16), bwd_batch=0):
    """One fused step on the GPU: level 0 no statistics, 1 the usage counts,
    2 counts and both maxima.  Returns the rasterizer (outputs), the loss
    vector, the statistics and the five parameter gradients."""
    views = ViewBatch(sc.cams, tile=tile)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1], bwd_batch=bwd_batch)
    p = Params.from_scene(sc)
    rast.plan_capacity(p)
    rast.preprocess(p)
    rast.bin()
    mask = torch.tensor(np.concatenate([m.reshape(-1) for m in masks]).astype(np.uint8), device="cuda")
    target = torch.tensor(np.concatenate([t.reshape(-1) for t in targets]).astype(np.float32), device="cuda")
    n = sc.n
    st = None
    if level == 1:
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
    elif level == 2:
        st = (torch.zeros(n, dtype=torch.int32, device="cuda"), torch.zeros(n, device="cuda"),
              torch.zeros(n, device="cuda"))
    loss = rast.train_step_raster(mask, target, gamma, w_c, stats=st, schedule=False)
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    rast.backward_project(p, g)
    rast.check_capacity()
    torch.cuda.synchronize()
    stats = None
    if level == 1:
        stats = (st.cpu().numpy().view(np.uint32),)
    elif level == 2:
        stats = (st[0].cpu().numpy().view(np.uint32), st[1].cpu().numpy(), st[2].cpu().numpy())
    grads = [t.cpu().numpy().astype(np.float64) for t in (g.means, g.scales, g.quats, g.opac, g.sh)]
    return rast, loss.cpu().numpy().astype(np.float64), stats, grads


def _ragged(seed=61, n=500, deg=3):
    return scenes.make_random_scene(seed, n, n_views=3, width=[61, 40, 33], height=[37, 64, 50], sh_degree=deg,
                                    scale_range=(0.02, 0.3))


@pytest.mark.parametrize("level,make", [(1, _ragged), (2, _ragged), (1, _extreme_scene)],
                         ids=["ragged-counts", "ragged-full", "degenerate-counts"])
def test_fused_step_matches_oracle_small(level, make):
    """Ragged three-view scene (and the scene of needles, edge-on, sub-pixel
    and large surfels), whole views: outputs, per-view losses, statistics
    and gradients of the fused launch against the oracle."""
    sc = make()
    rng = np.random.default_rng(62)
    masks = [rng.integers(0, 2, size=(c.height, c.width)).astype(np.uint8) for c in sc.cams]
    targets = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cams]
    gamma, w_c = 0.5, 1.0
    rast, loss, stats, g = _fused(sc, masks, targets, gamma, w_c, level)
    V = sc.v
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree, requires_grad=True)
    geoms = [oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, c, RP) for c in sc.cams]
    pairs, excl, tot, ties, npix = [], [], 0.0, 0, 0
    for v, cam in enumerate(sc.cams):
        HW = cam.width * cam.height
        pix = crop_pixels(0, 0, cam.width, cam.height)
        res = render_pixels(P64, cam, geoms[v], pix, RP)
        errs, frac, rep = compare_forward(per_view(rast, v), res, pix, rast, v, oracle_ctx=(P64, cam, geoms[v], RP))
        assert not rep["unresolved"]
        ties += int(round(frac * pix.shape[0]))
        npix += pix.shape[0]
        # the gradient pass takes every tie the way the GPU took it
        lf = masked_loss_fn(masks[v], targets[v], pix, HW, V, gamma, w_c)
        resg = render_pixels(P64, cam, geoms[v], pix, RP, loss_fn=lf, flips=rep["choice"])
        pairs.append(resg["pairs"])
        excl.append(clamp_tie_ids(res))
        l1, lb = masked_terms(resg, masks[v], targets[v], pix, HW)
        assert abs(loss[v] - lb) <= 1e-5 * max(lb, 1e-3), (v, loss[v], lb)
        assert abs(loss[V + v] - l1) <= 1e-5 * max(l1, 1e-3), (v, loss[V + v], l1)
        tot += (w_c * l1 + gamma * lb) / V
        print(f"view {v}: errors {errs}, tie pixels {frac:.4f}, ties taken the other way {len(rep['choice'])}")
    assert abs(loss[2 * V] - tot) <= 1e-5 * tot
    assert ties <= TIE_FRACTION * npix or ties <= 2, (ties, npix)
    st = oracle.prune_stats64(sc.n, pairs)
    np.testing.assert_array_equal(stats[0], st["hits"])
    if level == 2:
        np.testing.assert_allclose(stats[1], st["max_alpha"], atol=1e-5, rtol=0)
        np.testing.assert_allclose(stats[2], st["max_weight"], atol=1e-5, rtol=0)
    excl = np.unique(np.concatenate(excl))
    print(f"surfels used {(st['hits'] > 0).sum()} of {sc.n}; clamp-tie surfels left out of the gradients "
          f"{excl.size}")
    compare_grads(g, P64.grads(), excl)


@pytest.fixture(scope="module")
def _small_ref():
    """The ragged three-view scene's masked losses, statistics and gradients
    from the oracle (ties taken as the GPU's forward took them)."""
    sc = _ragged(seed=63, n=400)
    rng = np.random.default_rng(64)
    masks = [rng.integers(0, 2, size=(c.height, c.width)).astype(np.uint8) for c in sc.cams]
    targets = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in sc.cams]
    gamma, w_c = 0.5, 1.0
    rast, _, _, _ = _fused(sc, masks, targets, gamma, w_c, 2)
    V = sc.v
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree, requires_grad=True)
    pairs, excl, losses = [], [], np.zeros(2 * V + 1)
    for v, cam in enumerate(sc.cams):
        HW = cam.width * cam.height
        pix = crop_pixels(0, 0, cam.width, cam.height)
        geom = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, RP)
        res = render_pixels(P64, cam, geom, pix, RP)
        _, _, rep = compare_forward(per_view(rast, v), res, pix, rast, v, oracle_ctx=(P64, cam, geom, RP))
        assert not rep["unresolved"]
        lf = masked_loss_fn(masks[v], targets[v], pix, HW, V, gamma, w_c)
        resg = render_pixels(P64, cam, geom, pix, RP, loss_fn=lf, flips=rep["choice"])
        pairs.append(resg["pairs"])
        excl.append(clamp_tie_ids(res))
        l1, lb = masked_terms(resg, masks[v], targets[v], pix, HW)
        losses[v], losses[V + v] = lb, l1
        losses[2 * V] += (w_c * l1 + gamma * lb) / V
    st = oracle.prune_stats64(sc.n, pairs)
    return sc, masks, targets, gamma, w_c, losses, st, P64.grads(), np.unique(np.concatenate(excl))


@pytest.mark.parametrize("tile,batch", BWD_VARIANTS, ids=[f"{t[0]}x{t[1]}-b{b}" for t, b in BWD_VARIANTS])
def test_fused_step_every_lds_batch(_small_ref, tile, batch):
    """The fused step (full statistics) with every compiled tile shape and
    backward LDS batch: losses, statistics and gradients against the
    oracle."""
    sc, masks, targets, gamma, w_c, losses, st, gref, excl = _small_ref
    _, loss, stats, g = _fused(sc, masks, targets, gamma, w_c, 2, tile=tile, bwd_batch=batch)
    np.testing.assert_allclose(loss, losses, rtol=1e-5, atol=1e-8)
    np.testing.assert_array_equal(stats[0], st["hits"])
    np.testing.assert_allclose(stats[1], st["max_alpha"], atol=1e-5, rtol=0)
    np.testing.assert_allclose(stats[2], st["max_weight"], atol=1e-5, rtol=0)
    compare_grads(g, gref, excl)


def _crop_runs(sc, v, x0, y0, w=64, h=64, level=1):
    """Two fused launches whose every non-zero upstream gradient lies in the
    crop [x0, x0+w) x [y0, y0+h) of view v: (w_c = 1, gamma = 0, mask 1
    only inside the crop) and (w_c = 0, gamma = 0.5, mask 0 only inside the
    crop, 1 everywhere in the other views).  Their gradients add up to the
    gradient of the crop loss sum_crop (|C - I| / (3 H W) + 0.5 A / (H W)) / V,
    which one oracle pass over the crop gives (the oracle's cost grows with
    the crop's list lengths: thousands of entries per pixel at 3M surfels);
    each run's loss terms are checked on their own."""
    t0 = time.time()
    V = sc.v
    cam = sc.cams[v]
    HW = cam.width * cam.height
    inside = np.zeros((cam.height, cam.width), bool)
    inside[y0:y0 + h, x0:x0 + w] = True
    m1 = [inside.astype(np.uint8) if u == v else np.zeros((c.height, c.width), np.uint8)
          for u, c in enumerate(sc.cams)]
    m2 = [(~inside).astype(np.uint8) if u == v else np.ones((c.height, c.width), np.uint8)
          for u, c in enumerate(sc.cams)]
    gpu = []
    for masks, gamma, w_c in ((m1, 0.0, 1.0), (m2, 0.5, 0.0)):
        rast, loss, _, g = _fused(sc, masks, sc.targets, gamma, w_c, level)
        gpu.append((per_view(rast, v), loss, g, rast))
        del rast
    print(f"  GPU: two fused launches done ({time.time() - t0:.0f}s)", flush=True)
    geom = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, RP)
    P64 = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree, requires_grad=True)
    pix = crop_pixels(x0, y0, w, h)
    ones = np.ones((cam.height, cam.width), np.uint8)
    l1f = masked_loss_fn(ones, sc.targets[v], pix, HW, V, 0.0, 1.0)
    lbf = masked_loss_fn(np.zeros_like(ones), sc.targets[v], pix, HW, V, 0.5, 0.0)
    lf = lambda out, rows: l1f(out, rows) + lbf(out, rows)
    # the gradient pass is also the forward: rendered again only if a tie
    # has to be taken the other way
    res = render_pixels(P64, cam, geom, pix, RP, loss_fn=lf)
    print(f"  oracle forward + gradients of the crop done ({time.time() - t0:.0f}s)", flush=True)
    choice = None
    for k, (pv, loss, g, rast) in enumerate(gpu):
        errs, frac, rep = compare_forward(pv, res, pix, rast, v, oracle_ctx=(P64, cam, geom, RP))
        assert not rep["unresolved"]
        assert frac <= TIE_FRACTION or frac * pix.shape[0] <= 2, frac
        assert choice is None or rep["choice"] == choice      # both launches take the same decisions
        choice = rep["choice"]
        print(f"  run {k}: forward errors {errs}, tie pixels {frac:.4f} ({len(choice)} taken the other way)",
              flush=True)
    excl = clamp_tie_ids(res)
    if choice:
        P64.zero_grad()
        res = render_pixels(P64, cam, geom, pix, RP, loss_fn=lf, flips=choice)
    l1, _ = masked_terms(res, ones, sc.targets[v], pix, HW)
    _, lb = masked_terms(res, np.zeros_like(ones), sc.targets[v], pix, HW)
    (_, loss1, g1, _), (_, loss2, g2, _) = gpu
    assert abs(loss1[V + v] - l1) <= 1e-5 * l1 and abs(loss1[2 * V] - l1 / V) <= 1e-5 * l1 / V, (loss1, l1)
    assert abs(loss2[v] - lb) <= 1e-5 * lb and abs(loss2[2 * V] - 0.5 * lb / V) <= 1e-5 * lb / V, (loss2, lb)
    compare_grads([a + b for a, b in zip(g1, g2)], P64.grads(), excl)
    print(f"  clamp-tie surfels left out of the gradients: {excl.size} ({time.time() - t0:.0f}s)")


def test_fused_step_ragged16_crop():
    """ragged16-1m (16 views 400-1600 px, 1M surfels, SH 3) in the
    benchmark's launch configuration; loss restricted to the 64x64 crop at
    the centre of view 0."""
    sc = scenes.make_ragged16_1m()
    cam = sc.cams[0]
    _crop_runs(sc, 0, cam.width // 2 - 32, cam.height // 2 - 32, level=1)


def test_fused_step_wide8_crop_full_stats():
    """wide8-3m (8 views 1960x1090, 3M surfels, SH 3) with the full
    statistics in the same launch (the fused training-step workload); loss
    restricted to the 64x64 crop of view 0 at (948, 513)."""
    sc = scenes.make_wide8_3m()
    _crop_runs(sc, 0, 948, 513, level=2)
