"""Pins of the oracle's median depth (the 2DGS surface depth variant of the
normal consistency term): stacked surfels in closed form, a single surfel,
the derivative with respect to the median entry's depth, and the median
variant of the regulariser against planes and finite differences."""
import math

import numpy as np
import torch

import oracle
from oracle.render import Params64, render_pixels, render_view
from paper_2501_08174_amd import scenes
from tests.oracle_scenes import centre_on_pixel, front_camera, scene_from

ID = [1.0, 0.0, 0.0, 0.0]


def test_stacked_surfels_median(rp):
    """Three stacked fronto surfels at the centre pixel: the median entry is
    the last one that starts with T > 1/2 (T before each: 1, 1 - a1,
    (1 - a1)(1 - a2))."""
    cam = front_camera(32)
    for ops, want in [((0.4, 0.3, 0.5), 1), ((0.6, 0.3, 0.5), 0), ((0.1, 0.2, 0.3), 2)]:
        depths = [4.1, 4.3, 4.5]
        means = [centre_on_pixel(cam, 16, 16, d) for d in depths]
        sc = scene_from(means, [(0.5, 0.5)] * 3, [ID] * 3, ops, [(0.5, 0.5, 0.5)] * 3, [cam])
        g = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp)
        P = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0)
        res = render_pixels(P, cam, g, np.array([[16, 16]]), rp)
        # alphas at the centre pixel: o * exp(-u^2/2) with the float32 centre offset
        T, med = 1.0, -1
        for k in range(3):
            p = sc.means[k].astype(np.float64) + np.array([0, 0, 4.0])
            ctr = np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])
            u = (np.array([16.5, 16.5]) - ctr) * p[2] / (float(cam.fx) * float(sc.scales[k, 0]))
            a = float(sc.opac[k]) * math.exp(-(u @ u) / 2)
            if T > 0.5:
                med = k
            T *= 1 - a
        assert med == want
        assert res["median_gid"][0] == want
        p = sc.means[want].astype(np.float64) + np.array([0, 0, 4.0])
        assert abs(res["median_depth"][0] - p[2]) < 1e-9


def test_single_surfel_median_and_its_derivative(rp):
    cam = front_camera(24)
    sc = scene_from([centre_on_pixel(cam, 12, 12, 4.2)], [(0.3, 0.3)], [ID], 0.8, (0.5, 0.5, 0.5), [cam])
    g = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp)
    P = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, 0, requires_grad=True)
    jj, ii = np.meshgrid(np.arange(24), np.arange(24), indexing="ij")
    pix = np.stack([ii.ravel(), jj.ravel()], axis=1)
    res = render_pixels(P, cam, g, pix, rp,
                        loss_fn=lambda out, rows: out["median_depth"].sum())
    on = res["alpha"] > 0
    assert np.all(res["median_depth"][on] == res["depth"][on] / res["alpha"][on]) or \
        np.allclose(res["median_depth"][on], res["depth"][on] / res["alpha"][on], rtol=1e-12)
    assert np.all(res["median_depth"][~on] == 0)
    # fronto-parallel: the median depth of a blended pixel is p_z = mu_z + 4,
    # so d(sum median)/d mu_z = number of blended pixels
    gm = P.grads()[0][0]
    assert abs(gm[2] - on.sum()) < 1e-9 * on.sum()


def _plane_depth(cam, n, d):
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    r = np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy, np.ones(ii.shape)], -1)
    return d / (r @ np.asarray(n, np.float64))


def test_median_regulariser_plane_and_fd():
    cam = scenes.make_camera(np.eye(3), np.zeros(3), 13, 11)
    n = np.array([0.2, -0.1, -1.0]); n /= np.linalg.norm(n)
    z = _plane_depth(cam, n, -3.0)
    rng = np.random.default_rng(2)
    A = rng.uniform(0.3, 1.0, z.shape)
    D = rng.uniform(0.5, 2.0, z.shape)                 # ignored by the median variant
    N = np.moveaxis(A[..., None] * n, -1, 0)
    S = np.zeros(z.shape)
    r = oracle.regularizer_loss64([A], [D], [N], [S], [cam], 1.0, 0.5, medians=[z])
    border = np.ones(z.shape, bool); border[1:-1, 1:-1] = False
    assert abs(r["per_view"][0][1] - A[border].sum() / A.size) < 1e-12
    assert np.all(r["grads"][0]["depth"] == 0)
    zz = z + 0.05 * rng.standard_normal(z.shape)
    r = oracle.regularizer_loss64([A], [D], [N], [S], [cam], 1.0, 0.5, medians=[zz])
    f = lambda m: oracle.regularizer_loss64([A], [D], [N], [S], [cam], 1.0, 0.5, medians=[m])["total"]
    h = 1e-6
    for (j, i) in [(0, 0), (3, 4), (5, 6), (10, 12)]:
        mp, mm = zz.copy(), zz.copy()
        mp[j, i] += h; mm[j, i] -= h
        fd = (f(mp) - f(mm)) / (2 * h)
        assert abs(fd - r["grads"][0]["median"][j, i]) <= 1e-6 * max(1.0, abs(fd))
