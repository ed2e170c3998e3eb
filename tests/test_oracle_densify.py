"""Pins of the oracle's density-control statistic (the loss gradient with
respect to a screen-space translation of each surfel): the analytic
derivative of a single fronto-parallel surfel, central finite differences on
a random scene (cases whose blend decisions change under the step are
skipped), and the accumulation over views."""
import numpy as np
import pytest
import torch

import oracle
from oracle.render import Params64, render_pixels
from paper_2501_08174_amd import scenes
from tests.oracle_scenes import front_camera, scene_from

ID = [1.0, 0.0, 0.0, 0.0]


def _full(cam):
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1)


@pytest.mark.parametrize("s", [(0.3, 0.2), (0.15, 0.25)])
def test_fronto_parallel_analytic_translation_gradient(rp, s):
    cam = front_camera(40)
    mu = np.array([0.05, -0.03, 0.2])
    o = 0.6
    sc = scene_from(mu, s, ID, o, (0.5, 0.5, 0.5), [cam])
    g = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp)
    P = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    pix = _full(cam)
    w = np.random.default_rng(1).normal(size=pix.shape[0])
    wt = torch.tensor(w)
    shift = torch.zeros((1, 2), dtype=torch.float64, requires_grad=True)
    res = render_pixels(P, cam, g, pix, rp, loss_fn=lambda out, rows: (out["alpha"] * wt[rows]).sum(),
                        screen_shift=shift)
    got = shift.grad.numpy()[0]
    # analytic: alpha(x) = o G(x - delta), G = max(G_s, G_f) on blended, unclamped pixels
    mu32 = sc.means[0].astype(np.float64)
    su, sv = sc.scales[0].astype(np.float64)
    Z = mu32[2] + 4.0
    fx, cx = float(cam.fx), float(cam.cx)
    ccx, ccy = fx * mu32[0] / Z + cx, fx * mu32[1] / Z + cx
    x = pix[:, 0] + 0.5 - ccx
    y = pix[:, 1] + 0.5 - ccy
    ku, kv = Z / (fx * su), Z / (fx * sv)
    u, v = x * ku, y * kv
    Gs = np.exp(-(u * u + v * v) / 2)
    Gf = np.exp(-(x * x + y * y))
    surf = Gs >= Gf
    dGx = np.where(surf, Gs * u * ku, Gf * 2 * x)
    dGy = np.where(surf, Gs * v * kv, Gf * 2 * y)
    o32 = float(sc.opac[0])                     # the stored (float32) opacity
    a = o32 * np.maximum(Gs, Gf)
    on = (res["alpha"] > 0) & (a < 0.99)
    ref = np.array([(w * o32 * dGx)[on].sum(), (w * o32 * dGy)[on].sum()])
    assert not res["flag_cut"].any() or res["flag_cut"].mean() < 0.01
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12)


def test_finite_differences_and_accumulation(rp):
    sc = scenes.make_random_scene(61, 40, n_views=2, width=[30, 26], height=[24, 29], spread=0.5,
                                  scale_range=(0.05, 0.3))
    geoms = [oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, c, rp) for c in sc.cams]
    P = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
    rng = np.random.default_rng(4)
    ws = [torch.tensor(rng.normal(size=(c.width * c.height, 3))) for c in sc.cams]
    lfs = [lambda out, rows, w=w: (out["color"] * w[rows]).sum() for w in ws]
    pixs = [_full(c) for c in sc.cams]
    total, count, per_view, flagged = oracle.screen_grad_stats64(P, sc.cams, geoms, pixs, rp, lfs)
    for v in range(2):
        assert np.all(per_view[v][geoms[v]["culled"]] == 0)
    ref_total = sum(np.where(~geoms[v]["culled"], np.linalg.norm(per_view[v], axis=1), 0) for v in range(2))
    np.testing.assert_allclose(total, ref_total, rtol=1e-14)
    np.testing.assert_array_equal(count, sum((~g["culled"]).astype(int) for g in geoms))

    def loss(v, shift):
        with torch.no_grad():
            r = render_pixels(P, sc.cams[v], geoms[v], pixs[v], rp, screen_shift=torch.tensor(shift),
                              keep_decisions=True)
        L = float((torch.tensor(r["color"]) * ws[v]).sum())
        return L, np.concatenate([d["blended"].reshape(-1) for d in r["decisions"]])

    h, checked = 1e-6, 0
    for v in range(2):
        vis = np.nonzero(np.abs(per_view[v]).sum(axis=1) > 1e-3)[0][:6]
        for gid in vis:
            for ax in range(2):
                sp = np.zeros((sc.n, 2)); sm = np.zeros((sc.n, 2))
                sp[gid, ax] = h; sm[gid, ax] = -h
                Lp, dp = loss(v, sp)
                Lm, dm = loss(v, sm)
                if dp.shape != dm.shape or not np.array_equal(dp, dm):
                    continue
                fd = (Lp - Lm) / (2 * h)
                assert abs(fd - per_view[v][gid, ax]) <= 1e-5 * max(1.0, abs(fd)), (v, gid, ax, fd)
                checked += 1
    assert checked >= 12
