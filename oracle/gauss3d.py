"""Occlusion-aware pruning statistics for 3D Gaussians (oracle; test
infrastructure only).

Appendix B applies the pruning of Section 4.3 to 3DGS: the renderer again
records, over all views, whether each Gaussian contributed to the colour of
at least one pixel, now with 3D Gaussians splatted as 2D Gaussians (EWA
splatting).  The projection and
compositing details are those of 3DGS; the readings (listed with reasons in
the design notes) are

  covariance  Sigma = (R(q/|q|) S)(R S)^T, S = diag(s_1, s_2, s_3); camera
              space W = R_v R S, Sigma_c = W W^T
  projection  p = R_v mu + t_v; centre c = (f_x p_x/p_z + c_x, f_y p_y/p_z + c_y);
              Jacobian J of the perspective map at (t_x, t_y, p_z) with t/p_z
              clamped to 1.3 tan(fov/2) per axis (tan(fov_x/2) = W/(2 f_x));
              Sigma_2 = J Sigma_c J^T + 0.3 I (the low-pass dilation)
  cutoff      o exp(-q/2) >= alpha_min with q = d^T Sigma_2^-1 d, d = x - c:
              q <= 2 L, L = ln(o / alpha_min); the pixel rectangle is the
              bounding box of q <= ceil_grid(2 L) (half extents
              sqrt(r2 Sigma_2,xx), sqrt(r2 Sigma_2,yy)), pixel centres inside,
              clipped to the image; ceil_grid rounds up to 2^-16
  culls       p_z <= z_near, o < alpha_min, det(Sigma_2) <= 0 (or NaN), empty
              rectangle
  compositing a = min(alpha_max, o exp(-q/2)); skip a < alpha_min; stop before
              blending k when T (1 - a_k) < t_min; lists in ascending
              (float32 p_z, id) like the surfel path

Binning quantities are float64 expressions evaluated elementwise in the
written order (no fused multiply-add; IEEE division and square root) so that
the GPU reproduces them bit for bit; the logarithm is the only library
routine and is rounded up to the 2^-16 grid (values within 1e-9 of a grid
point are reported in grid_tie).
"""
from __future__ import annotations

import numpy as np

from .geometry import GRID, RasterParams, _rot_apply, rotation_columns64
from .render import TIE_CLAMP, TIE_CUTOFF_REL, TIE_TERM_REL

DILATION = 0.3
FOV_CLAMP = 1.3


def view_geometry3d64(means, scales, quats, opac, cam, rp: RasterParams = RasterParams()):
    """Per-Gaussian float64 projection of one view (all arrays over N):
    p (N,3); cov2 (N,3) = (a, b, c) of Sigma_2; conic (N,3); center (N,2);
    L (N,); culled, cull_reason (0 none, 1 near, 2 opacity, 3 degenerate,
    4 empty rect); rect (N,4) inclusive [i_lo, i_hi, j_lo, j_hi]; tiles (N,4);
    tiles_touched (N,); depth_bits (N,) uint32; grid_tie (N,)."""
    mu = np.asarray(means, np.float64)
    s = np.asarray(scales, np.float64)
    o = np.asarray(opac, np.float64)
    N = mu.shape[0]
    vm = np.asarray(cam.viewmat, np.float64)
    Rv, tv = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = (float(np.float32(cam.fx)), float(np.float32(cam.fy)),
                      float(np.float32(cam.cx)), float(np.float32(cam.cy)))
    znear = float(np.float32(cam.znear))
    Wd, Hd = int(cam.width), int(cam.height)
    amin = float(np.float32(rp.alpha_min))

    c0, c1, c2 = rotation_columns64(quats)              # columns of R(q)
    # columns of W = R_v R S
    w0 = _rot_apply(Rv, c0) * s[:, 0:1]
    w1 = _rot_apply(Rv, c1) * s[:, 1:2]
    w2 = _rot_apply(Rv, c2) * s[:, 2:3]
    p = _rot_apply(Rv, mu)
    for i in range(3):
        p[:, i] = p[:, i] + tv[i]
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    limx = FOV_CLAMP * (Wd / (2.0 * fx))
    limy = FOV_CLAMP * (Hd / (2.0 * fy))
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        tx = np.minimum(limx, np.maximum(-limx, x / z)) * z
        ty = np.minimum(limy, np.maximum(-limy, y / z)) * z
        j00 = fx / z
        j02 = -(fx * tx) / (z * z)
        j11 = fy / z
        j12 = -(fy * ty) / (z * z)
        # rows of U = J W: U_0k = j00 W_0k + j02 W_2k, U_1k = j11 W_1k + j12 W_2k
        cols = (w0, w1, w2)
        u0 = np.stack([j00 * wk[:, 0] + j02 * wk[:, 2] for wk in cols], axis=1)
        u1 = np.stack([j11 * wk[:, 1] + j12 * wk[:, 2] for wk in cols], axis=1)
        dot = lambda a, b: (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1]) + a[:, 2] * b[:, 2]
        ca = dot(u0, u0) + DILATION
        cb = dot(u0, u1)
        cc = dot(u1, u1) + DILATION
        det = ca * cc - cb * cb
        conic = np.stack([cc / det, -cb / det, ca / det], axis=1)
        L = np.log(o / amin)
        r2 = np.ceil(2.0 * L * GRID) / GRID
        frac = 2.0 * L * GRID - np.floor(2.0 * L * GRID)
        grid_tie = np.minimum(frac, 1 - frac) < 1e-9 * (2.0 * L * GRID + 1.0)
        ccx = (fx * x) / z + cx
        ccy = (fy * y) / z + cy
        ex = np.sqrt(r2 * ca)
        ey = np.sqrt(r2 * cc)
        ilo = np.maximum(np.ceil((ccx - ex) - 0.5), 0.0)
        ihi = np.minimum(np.floor((ccx + ex) - 0.5), Wd - 1.0)
        jlo = np.maximum(np.ceil((ccy - ey) - 0.5), 0.0)
        jhi = np.minimum(np.floor((ccy + ey) - 0.5), Hd - 1.0)
        c_rect = ~((ilo <= ihi) & (jlo <= jhi))
        c_degen = ~(det > 0.0)

    reason = np.zeros(N, np.int8)
    reason[c_rect] = 4
    reason[c_degen] = 3
    reason[o < amin] = 2
    reason[z <= znear] = 1
    culled = reason != 0
    rect = np.zeros((N, 4), np.int64)
    ok = ~culled
    rect[ok, 0] = ilo[ok].astype(np.int64)
    rect[ok, 1] = ihi[ok].astype(np.int64)
    rect[ok, 2] = jlo[ok].astype(np.int64)
    rect[ok, 3] = jhi[ok].astype(np.int64)
    tiles = np.zeros((N, 4), np.int64)
    tiles[:, 0] = rect[:, 0] // rp.tile_w
    tiles[:, 1] = rect[:, 1] // rp.tile_w
    tiles[:, 2] = rect[:, 2] // rp.tile_h
    tiles[:, 3] = rect[:, 3] // rp.tile_h
    tt = (tiles[:, 1] - tiles[:, 0] + 1) * (tiles[:, 3] - tiles[:, 2] + 1)
    tt[culled] = 0
    depth_bits = np.where(culled, np.uint32(0xFFFFFFFF), np.float32(z).view(np.uint32)).astype(np.uint32)
    return dict(p=p, cov2=np.stack([ca, cb, cc], axis=1), conic=conic, center=np.stack([ccx, ccy], axis=1),
                L=L, opac=o, culled=culled, cull_reason=reason, rect=rect, tiles=tiles,
                tiles_touched=tt.astype(np.int64), depth_bits=depth_bits, grid_tie=grid_tie & ok)


def prune_pixels3d(geom, pix: np.ndarray, rp: RasterParams = RasterParams()):
    """Front-to-back compositing decisions of the pixels ``pix`` (P,2) (no
    shading).  Returns the blended pairs (pixel row, id, a, omega), a per
    pixel tie flag and the ids of the tie entries (a cutoff, clamp or
    termination decision within the tie windows)."""
    ok = ~geom["culled"]
    rect = geom["rect"]
    rows, gids, avals, wvals, tie_ids = [], [], [], [], []
    flagged = np.zeros(pix.shape[0], bool)
    if pix.shape[0] == 0:
        return {"pairs": (np.zeros((0, 2), np.int64), np.zeros(0), np.zeros(0)), "flagged": flagged,
                "tie_ids": np.zeros(0, np.int64)}
    # candidates: rectangles meeting the bounding box of the pixels
    i0, i1, j0, j1 = pix[:, 0].min(), pix[:, 0].max(), pix[:, 1].min(), pix[:, 1].max()
    ok = ok & (rect[:, 0] <= i1) & (rect[:, 1] >= i0) & (rect[:, 2] <= j1) & (rect[:, 3] >= j0)
    cand_all = np.nonzero(ok)[0]
    order = np.lexsort((cand_all, geom["depth_bits"][cand_all]))
    cand_all = cand_all[order]
    r = rect[cand_all]
    for k, (i, j) in enumerate(pix):
        sel = (r[:, 0] <= i) & (i <= r[:, 1]) & (r[:, 2] <= j) & (j <= r[:, 3])
        ids = cand_all[sel]
        if ids.size == 0:
            continue
        dx = (i + 0.5) - geom["center"][ids, 0]
        dy = (j + 0.5) - geom["center"][ids, 1]
        con = geom["conic"][ids]
        q = (con[:, 0] * dx * dx + 2.0 * con[:, 1] * dx * dy) + con[:, 2] * dy * dy
        a_raw = geom["opac"][ids] * np.exp(-0.5 * q)
        a = np.minimum(rp.alpha_max, a_raw)
        T = 1.0
        ties = []                     # entries whose own decision sits on a threshold
        for n, gid in enumerate(ids):
            if abs(a_raw[n] - rp.alpha_min) <= TIE_CUTOFF_REL * rp.alpha_min:
                ties.append(gid)
            if a[n] < rp.alpha_min:
                continue
            if abs(a_raw[n] - rp.alpha_max) <= TIE_CLAMP:
                ties.append(gid)
            Tn = T * (1.0 - a[n])
            if abs(Tn - rp.t_min) <= TIE_TERM_REL * rp.t_min:
                ties.append(gid)
            if Tn < rp.t_min:
                break
            rows.append(k); gids.append(gid); avals.append(a[n]); wvals.append(a[n] * T)
            T = Tn
        if ties:
            flagged[k] = True
            tie_ids.append(np.asarray(ties, np.int64))
    pairs = (np.stack([np.asarray(rows, np.int64), np.asarray(gids, np.int64)], axis=1) if rows
             else np.zeros((0, 2), np.int64), np.asarray(avals), np.asarray(wvals))
    return {"pairs": pairs, "flagged": flagged,
            "tie_ids": np.unique(np.concatenate(tie_ids)) if tie_ids else np.zeros(0, np.int64)}
