"""Pins of the oracle's 3D-Gaussian pruning path: the EWA covariance of an
on-axis isotropic Gaussian in closed form, the projected covariance against
an explicit matrix product (including the clamped field-of-view Jacobian),
rotation invariance of isotropic Gaussians, conservativeness of the pixel
rectangle against dense evaluation, stacked-Gaussian compositing weights and
the culls."""
import math

import numpy as np
import pytest

import oracle
from oracle.gauss3d import prune_pixels3d, view_geometry3d64
from paper_2501_08174_amd import scenes


def _cam(W=48, H=40, pos=(0.0, 0.0, 0.0)):
    return scenes.make_camera(np.eye(3), np.asarray(pos, float), W, H)


def _g(mu, s, q, o, cam, rp):
    return view_geometry3d64(np.asarray(mu, np.float32).reshape(-1, 3), np.asarray(s, np.float32).reshape(-1, 3),
                             np.asarray(q, np.float32).reshape(-1, 4), np.asarray(o, np.float32).reshape(-1),
                             cam, rp)


def test_on_axis_isotropic_closed_form(rp):
    cam = _cam()
    Z, s, o = 3.0, 0.2, 0.8
    g = _g([0.0, 0.0, Z], [s, s, s], [1, 0, 0, 0], o, cam, rp)
    f = float(np.float32(cam.fx))
    s32 = float(np.float32(s))
    var = (f * s32 / Z) ** 2 + 0.3
    np.testing.assert_allclose(g["cov2"][0], [var, 0.0, var], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(g["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-14)
    assert tuple(g["center"][0]) == (float(np.float32(cam.cx)), float(np.float32(cam.cy)))
    # blended alphas at every pixel in closed form
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    pix = np.stack([ii.ravel(), jj.ravel()], axis=1)
    res = prune_pixels3d(g, pix, rp)
    rows, a = res["pairs"][0][:, 0], res["pairs"][1]
    d2 = (pix[rows, 0] + 0.5 - cam.cx) ** 2 + (pix[rows, 1] + 0.5 - cam.cy) ** 2
    o32 = float(np.float32(o))
    np.testing.assert_allclose(a, np.minimum(0.99, o32 * np.exp(-d2 / (2 * var))), rtol=1e-13)
    # every pixel above the cutoff blends it
    d2_all = (pix[:, 0] + 0.5 - cam.cx) ** 2 + (pix[:, 1] + 0.5 - cam.cy) ** 2
    want = o32 * np.exp(-d2_all / (2 * var)) >= rp.alpha_min
    got = np.zeros(pix.shape[0], bool); got[rows] = True
    assert np.array_equal(got | res["flagged"], want | res["flagged"])


@pytest.mark.parametrize("mu", [(0.4, -0.3, 2.5), (6.0, 0.5, 2.0), (-0.2, -9.0, 3.0)])
def test_projected_covariance_matches_matrix_product(rp, mu):
    rng = np.random.default_rng(int(abs(mu[0]) * 10))
    cam = _cam()
    s = rng.uniform(0.05, 0.4, 3)
    q = rng.standard_normal(4)
    g = _g(mu, s, q, 0.7, cam, rp)
    m = np.float32(mu).astype(np.float64); s32 = np.float32(s).astype(np.float64)
    q32 = np.float32(q).astype(np.float64); q32 /= np.linalg.norm(q32)
    w, x, y, z = q32
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    Sig = R @ np.diag(s32 ** 2) @ R.T
    f, cx = float(np.float32(cam.fx)), float(np.float32(cam.cx))
    X, Y, Zc = m
    lim = 1.3 * cam.width / (2 * f), 1.3 * cam.height / (2 * f)
    tx = np.clip(X / Zc, -lim[0], lim[0]) * Zc
    ty = np.clip(Y / Zc, -lim[1], lim[1]) * Zc
    J = np.array([[f / Zc, 0, -f * tx / Zc ** 2], [0, f / Zc, -f * ty / Zc ** 2]])
    C2 = J @ Sig @ J.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(g["cov2"][0], [C2[0, 0], C2[0, 1], C2[1, 1]], rtol=1e-12)
    assert abs(g["center"][0][0] - (f * X / Zc + cx)) < 1e-12


def test_isotropic_rotation_invariance(rp):
    cam = _cam()
    rng = np.random.default_rng(3)
    qs = rng.standard_normal((6, 4))
    mus = np.tile([[0.3, 0.2, 2.8]], (6, 1))
    g = _g(mus, np.full((6, 3), 0.15), qs, np.full(6, 0.5), cam, rp)
    assert np.abs(g["cov2"] - g["cov2"][0]).max() < 1e-12
    assert np.all(g["rect"] == g["rect"][0])


def test_rectangle_is_conservative(rp):
    """No pixel centre outside the rectangle reaches the cutoff (dense check
    over a margin of 8 pixels around every rectangle)."""
    rng = np.random.default_rng(5)
    n = 200
    cam = _cam(64, 56)
    mus = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.2, 1.2, n), rng.uniform(1.0, 4.0, n)], 1)
    s = np.exp(rng.uniform(math.log(0.02), math.log(0.3), (n, 3)))
    g = _g(mus, s, rng.standard_normal((n, 4)), rng.uniform(0.01, 1.0, n), cam, rp)
    checked = 0
    for k in np.nonzero(~g["culled"])[0]:
        i0, i1, j0, j1 = g["rect"][k]
        jj, ii = np.meshgrid(np.arange(j0 - 8, j1 + 9), np.arange(i0 - 8, i1 + 9), indexing="ij")
        out = (ii < i0) | (ii > i1) | (jj < j0) | (jj > j1)
        inside_img = (ii >= 0) & (ii < cam.width) & (jj >= 0) & (jj < cam.height)
        dx = ii + 0.5 - g["center"][k, 0]; dy = jj + 0.5 - g["center"][k, 1]
        c = g["conic"][k]
        qv = (c[0] * dx * dx + 2 * c[1] * dx * dy) + c[2] * dy * dy
        a = g["opac"][k] * np.exp(-0.5 * qv)
        assert not np.any((a >= rp.alpha_min) & out & inside_img), k
        checked += 1
    assert checked > 100


def test_stacked_gaussians_and_culls(rp):
    cam = _cam()
    o = np.array([0.5, 0.6, 0.7, 0.9, 0.002, 0.5], np.float32)
    mus = [[0, 0, 2.0], [0, 0, 2.5], [0, 0, 3.0], [0, 0, -1.0], [0, 0, 2.2], [40.0, 0, 2.0]]
    g = _g(mus, np.full((6, 3), 0.3), np.tile([1.0, 0, 0, 0], (6, 1)), o, cam, rp)
    assert list(g["cull_reason"]) == [0, 0, 0, 1, 2, 4]
    pix = np.array([[24, 20]])
    res = prune_pixels3d(g, pix, rp)
    ids = res["pairs"][0][:, 1]
    assert list(ids) == [0, 1, 2]
    a = res["pairs"][1]
    w = res["pairs"][2]
    np.testing.assert_allclose(w, a * np.concatenate([[1.0], np.cumprod(1 - a)[:-1]]), rtol=1e-15)
    st = oracle.prune_stats64(6, [res["pairs"]], [g["culled"]])
    assert list(st["hits"]) == [1, 1, 1, 0, 0, 0]
    assert list(st["in_frustum"]) == [True, True, True, False, False, False]
