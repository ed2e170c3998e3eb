"""Pins of the oracle's 2DGS regularisers (Eq. 3's L_d and L_n): geometric
facts of the depth normals (planes, spheres, orientation), closed forms of
the losses and of their direct gradients, and central finite differences of
the gradients that flow through the depth normals."""
import numpy as np
import pytest

import oracle
from paper_2501_08174_amd import scenes


def _cam(W, H, f=None):
    return scenes.make_camera(np.eye(3), np.zeros(3), W, H, fx=f)


def _rays(cam):
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy, np.ones(ii.shape)], -1)


def _plane_depth(cam, n, d):
    """Depth map (z) of the plane n . X = d along every pixel ray."""
    r = _rays(cam)
    return d / (r @ np.asarray(n, np.float64))


@pytest.mark.parametrize("n", [(0.0, 0.0, -1.0), (0.3, -0.2, -1.0), (-0.5, 0.4, -0.8)])
def test_plane_gives_its_normal_towards_the_camera(n):
    cam = _cam(23, 17)
    n = np.asarray(n) / np.linalg.norm(n)
    z = _plane_depth(cam, n, -3.0)           # n . X = -3: plane in front, n towards the camera
    assert np.all(z > 0)
    A = np.full(z.shape, 0.7)
    Nd = oracle.depth_normal64(A, A * z, cam).numpy()
    inner = Nd[1:-1, 1:-1].reshape(-1, 3)
    assert np.abs(inner - n).max() < 1e-12
    assert np.all(Nd[0] == 0) and np.all(Nd[-1] == 0) and np.all(Nd[:, 0] == 0) and np.all(Nd[:, -1] == 0)


def test_sphere_normals_to_second_order():
    """Points of a sphere: central differences give the outward normal with
    an O(h^2) error; halving the pixel size quarters it."""
    errs = []
    for W in (64, 128):
        cam = _cam(W, W, f=W * 1.2)
        r = _rays(cam)
        c = np.array([0.0, 0.0, 4.0]); R = 1.5
        # nearest intersection of the ray t r with |X - c| = R
        a = (r * r).sum(-1); b = -2 * (r @ c); cc = c @ c - R * R
        t = (-b - np.sqrt(b * b - 4 * a * cc)) / (2 * a)
        X = t[..., None] * r
        ref = (X - c) / R
        Nd = oracle.depth_normal64(np.ones(t.shape), t, cam).numpy()
        k = W // 4
        errs.append(np.abs(Nd[W // 2 - k:W // 2 + k, W // 2 - k:W // 2 + k] - ref[W // 2 - k:W // 2 + k,
                                                                                  W // 2 - k:W // 2 + k]).max())
    assert errs[0] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_zero_alpha_pixels_sit_at_the_camera_centre():
    cam = _cam(5, 4)
    A = np.ones((4, 5)); A[1, 2] = 0.0
    D = np.full((4, 5), 2.0)
    P = oracle.depth_points64(A, D, cam).numpy()
    assert np.all(P[1, 2] == 0)
    assert P[0, 0, 2] == 2.0


def test_loss_closed_forms_and_direct_gradients():
    """Rendered normals equal to alpha times the plane normal: every interior
    pixel's L_n term vanishes, the border ones are A; L_d is the mean
    distortion; dL/d dist and dL/dN are the constants of the definition."""
    cams = [_cam(11, 9), _cam(6, 8)]
    rng = np.random.default_rng(0)
    As, Ds, Ns, Ss, n = [], [], [], [], np.array([0.1, -0.2, -1.0]) / np.linalg.norm([0.1, -0.2, -1.0])
    for cam in cams:
        z = _plane_depth(cam, n, -2.5)
        A = rng.uniform(0.2, 1.0, z.shape)
        As.append(A); Ds.append(A * z); Ns.append(np.moveaxis(A[..., None] * n, -1, 0)); Ss.append(rng.uniform(0, 1, z.shape))
    wd, wn = 1000.0, 0.05
    r = oracle.regularizer_loss64(As, Ds, Ns, Ss, cams, wd, wn)
    for v, cam in enumerate(cams):
        A = As[v]
        border = np.ones(A.shape, bool); border[1:-1, 1:-1] = False
        L_d, L_n = r["per_view"][v]
        assert abs(L_d - Ss[v].mean()) < 1e-15
        assert abs(L_n - A[border].sum() / A.size) < 1e-12
        HW, V = A.size, len(cams)
        g = r["grads"][v]
        np.testing.assert_allclose(g["dist"], wd / (HW * V), rtol=1e-14)
        Nd = oracle.depth_normal64(A, Ds[v], cam).numpy()
        np.testing.assert_allclose(g["normal"], np.moveaxis(-wn * Nd / (HW * V), -1, 0), atol=1e-15)
    tot = sum(wd * a + wn * b for a, b in r["per_view"]) / len(cams)
    assert abs(r["total"] - tot) <= 1e-14 * abs(tot)


def test_gradients_through_the_depth_normals_match_finite_differences():
    cam = _cam(7, 6)
    rng = np.random.default_rng(3)
    H, W = 6, 7
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    z = 3.0 + 0.3 * np.sin(0.7 * ii) + 0.2 * np.cos(0.9 * jj) + 0.05 * rng.standard_normal((H, W))
    A = rng.uniform(0.3, 1.0, (H, W)); A[2, 3] = 0.0
    D = A * z
    N = rng.standard_normal((3, H, W)) * 0.5
    S = rng.uniform(0, 0.1, (H, W))
    wd, wn = 3.0, 0.7
    r = oracle.regularizer_loss64([A], [D], [N], [S], [cam], wd, wn)
    f = lambda A_, D_: oracle.regularizer_loss64([A_], [D_], [N], [S], [cam], wd, wn)["total"]
    h = 1e-6
    for (j, i) in [(0, 0), (1, 1), (2, 2), (3, 3), (2, 4), (4, 5), (5, 6), (1, 3)]:
        for name, X in (("depth", D), ("alpha", A)):
            if name == "alpha" and A[j, i] == 0.0:
                continue
            Xp, Xm = X.copy(), X.copy()
            Xp[j, i] += h; Xm[j, i] -= h
            fd = (f(Xp, D) - f(Xm, D)) / (2 * h) if name == "alpha" else (f(A, Xp) - f(A, Xm)) / (2 * h)
            an = r["grads"][0][name][j, i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, j, i, fd, an)


def test_tiny_images_have_no_depth_normals():
    for H, W in [(1, 1), (2, 5), (5, 2), (2, 2)]:
        cam = _cam(W, H)
        A = np.full((H, W), 0.5)
        r = oracle.regularizer_loss64([A], [A * 2], [np.ones((3, H, W))], [np.zeros((H, W))], [cam], 1.0, 1.0)
        assert abs(r["per_view"][0][1] - 0.5) < 1e-15
        assert np.all(r["grads"][0]["depth"] == 0)
