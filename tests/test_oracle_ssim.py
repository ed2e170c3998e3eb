"""Pins of the oracle's masked SSIM / D-SSIM and PSNR: the window's
definition, identity and symmetry, the closed form on constant images away
from the borders, the zero-padding border of a constant image, masked-out
images, a direct double-loop evaluation of one pixel, and central finite
differences of the D-SSIM gradient."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle.ssim import C1, C2, ssim_map64


def test_window():
    g = oracle.gaussian_1d64().numpy()
    assert g.shape == (11,) and abs(g.sum() - 1) < 1e-15
    assert np.allclose(g, g[::-1], atol=0)
    ref = np.exp(-np.arange(-5, 6) ** 2 / (2 * 1.5 ** 2))
    assert np.allclose(g, ref / ref.sum(), rtol=1e-15)
    w = oracle.window_2d64().numpy()
    assert abs(w.sum() - 1) < 1e-14 and w.argmax() == 60


def test_identity_symmetry_and_masked_out():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.uniform(size=(3, 19, 23)))
    y = torch.tensor(rng.uniform(size=(3, 19, 23)))
    assert torch.allclose(ssim_map64(x, x), torch.ones_like(x), atol=1e-12)
    assert torch.allclose(ssim_map64(x, y), ssim_map64(y, x), atol=0)
    assert float(ssim_map64(x, y).mean()) < 0.5
    z = np.zeros((19, 23))
    assert abs(float(oracle.masked_ssim64(x.numpy(), y.numpy(), z)) - 1.0) < 1e-15


def test_constant_images_closed_form():
    """Constant a and b: interior pixels (the window inside the image) have
    zero variances, so SSIM = (2ab + C1) / (a^2 + b^2 + C1); at a border the
    zero padding lowers the means by the clipped window weight."""
    H, W, a, b = 17, 20, 0.7, 0.3
    x = torch.full((3, H, W), a, dtype=torch.float64)
    y = torch.full((3, H, W), b, dtype=torch.float64)
    m = ssim_map64(x, y).numpy()
    ref = (2 * a * b + C1) / (a * a + b * b + C1)
    assert np.abs(m[:, 5:-5, 5:-5] - ref).max() < 1e-12
    # corner pixel: the window sees the quarter (incl. the centre row and
    # column) of the Gaussian; the means are the clipped weight times a, b
    g = oracle.gaussian_1d64().numpy()
    wsum = g[5:].sum() ** 2
    mx, my = a * wsum, b * wsum
    sx = a * a * wsum - mx * mx
    sy = b * b * wsum - my * my
    sxy = a * b * wsum - mx * my
    corner = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))
    assert abs(m[0, 0, 0] - corner) < 1e-12


def test_one_pixel_by_direct_summation():
    rng = np.random.default_rng(1)
    x = rng.uniform(size=(3, 14, 15)); y = rng.uniform(size=(3, 14, 15))
    m = ssim_map64(torch.tensor(x), torch.tensor(y)).numpy()
    g = oracle.gaussian_1d64().numpy()
    for (c, j, i) in [(0, 0, 0), (1, 7, 7), (2, 13, 3), (0, 4, 14)]:
        sums = np.zeros(5)
        for dj in range(-5, 6):
            for di in range(-5, 6):
                jj, ii = j + dj, i + di
                if 0 <= jj < 14 and 0 <= ii < 15:
                    w = g[dj + 5] * g[di + 5]
                    xv, yv = x[c, jj, ii], y[c, jj, ii]
                    sums += w * np.array([xv, yv, xv * xv, yv * yv, xv * yv])
        mx, my, ex2, ey2, exy = sums
        sx, sy, sxy = ex2 - mx * mx, ey2 - my * my, exy - mx * my
        ref = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sx + sy + C2))
        assert abs(m[c, j, i] - ref) < 1e-13


def test_psnr():
    c = np.zeros((3, 4, 5)); t = np.full((3, 4, 5), 0.1); m = np.ones((4, 5))
    assert abs(oracle.masked_psnr64(c, t, m) - 20.0) < 1e-12
    m[:, :] = 0
    assert oracle.masked_psnr64(c, t, m) == math.inf


def test_dssim_gradient_finite_differences():
    rng = np.random.default_rng(2)
    H, W = 9, 12
    cols = [rng.uniform(size=(3, H, W)), rng.uniform(size=(3, 7, 6))]
    tgts = [rng.uniform(size=(3, H, W)), rng.uniform(size=(3, 7, 6))]
    masks = [(rng.uniform(size=(H, W)) > 0.3).astype(np.uint8), np.ones((7, 6), np.uint8)]
    r = oracle.dssim_loss64(cols, tgts, masks, 0.2)
    assert abs(r["total"] - sum(0.2 * (1 - s) for s in r["ssim"]) / 2) < 1e-15
    h = 1e-6
    f = lambda cs: oracle.dssim_loss64(cs, tgts, masks, 0.2)["total"]
    for v, (c, j, i) in [(0, (0, 0, 0)), (0, (1, 4, 6)), (0, (2, 8, 11)), (1, (1, 3, 2))]:
        cp = [x.copy() for x in cols]; cm = [x.copy() for x in cols]
        cp[v][c, j, i] += h; cm[v][c, j, i] -= h
        fd = (f(cp) - f(cm)) / (2 * h)
        an = r["grads"][v][c, j, i]
        assert abs(fd - an) <= 1e-7 + 1e-6 * abs(an), (v, c, j, i, fd, an)
    # masked-out pixels receive no gradient
    assert np.all(r["grads"][0][:, masks[0] == 0] == 0)
