"""Surfel projection, culling, conservative pixel rectangles and tile binning
in float64 (oracle; test infrastructure only).

What it follows
  * Section 4.3 of the paper: during preprocessing every Gaussian inside the
    viewing frustum is projected to the image and assigned the pixels it can
    contribute to; a Gaussian outside is disqualified and assigned to no
    pixel; each pixel then blends its assigned Gaussians front to back.
  * Section 3.1: a surfel has a position, a shape (two tangent scales and a
    rotation) and an appearance.
The numerical details the paper leaves to the 2DGS/3DGS renderers are fixed
here as explicit readings (they are listed with reasons in the design notes):

  surfel frame      R(q/|q|) with columns (t_u, t_v, n); quaternion (w,x,y,z)
  camera space      p = R_v mu + t_v, a_u = s_u R_v t_u, a_v = s_v R_v t_v,
                    n_c = R_v n, negated when n_c . p > 0
  splat matrix      M = K [a_u a_v p] with K the pinhole intrinsics
  cutoff radii      L = ln(o / alpha_min), r_s^2 = ceil_grid(2L),
                    r_f^2 = ceil_grid(L), ceil_grid rounds up to 2^-16
  culling           (i) p_z <= znear, (ii) o < alpha_min, (iii) the cutoff
                    disc is not strictly in front of the camera,
                    (iv) empty pixel rectangle
  rectangle         extent of the projected disc u^2+v^2 <= r_s^2 (dual
                    conic) united with the low-pass disc |x - c| <= r_f,
                    pixels whose centres lie inside, clipped to the image
  key               (global tile id << 32) | bits(float32(p_z)); ties by id

Every float64 expression is evaluated elementwise with numpy in the order
written (no fused multiply-add, IEEE division and square root), so that an
implementation that evaluates the same expressions in the same order obtains
the same bits.  Only the natural logarithm is a library routine on both sides;
its result is rounded up to the 2^-16 grid, and values within 1e-9 of a grid
point are reported in ``grid_tie`` so that a test can exempt them.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GRID = 65536.0


@dataclass(frozen=True)
class RasterParams:
    """Renderer constants.  The defaults are the float32 values of 1/255,
    0.99 and 1e-4 (alpha cutoff, alpha clamp, transmittance stop)."""
    tile_w: int = 16
    tile_h: int = 16
    alpha_min: float = float(np.float32(1.0 / 255.0))
    alpha_max: float = float(np.float32(0.99))
    t_min: float = float(np.float32(1e-4))


def rotation_columns64(quats: np.ndarray):
    """Columns (t_u, t_v, n) of the rotation matrix of q/|q|, float64,
    each (N,3).  Textbook unit-quaternion rotation matrix."""
    q = np.asarray(quats, np.float64)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    nrm = np.sqrt(((w * w + x * x) + y * y) + z * z)
    w = w / nrm
    x = x / nrm
    y = y / nrm
    z = z / nrm
    r00 = 1.0 - 2.0 * (y * y + z * z)
    r01 = 2.0 * (x * y - w * z)
    r02 = 2.0 * (x * z + w * y)
    r10 = 2.0 * (x * y + w * z)
    r11 = 1.0 - 2.0 * (x * x + z * z)
    r12 = 2.0 * (y * z - w * x)
    r20 = 2.0 * (x * z - w * y)
    r21 = 2.0 * (y * z + w * x)
    r22 = 1.0 - 2.0 * (x * x + y * y)
    tu = np.stack([r00, r10, r20], axis=1)
    tv = np.stack([r01, r11, r21], axis=1)
    n = np.stack([r02, r12, r22], axis=1)
    return tu, tv, n


def _rot_apply(Rv: np.ndarray, a: np.ndarray) -> np.ndarray:
    """R_v a for a (N,3), row by row as ((r0 a0 + r1 a1) + r2 a2)."""
    out = np.empty_like(a)
    for i in range(3):
        out[:, i] = (Rv[i, 0] * a[:, 0] + Rv[i, 1] * a[:, 1]) + Rv[i, 2] * a[:, 2]
    return out


def _ceil_grid(x: np.ndarray) -> np.ndarray:
    return np.ceil(x * GRID) / GRID


def _conic_dot(rs2, a, b):
    """<a,b> = r_s^2 (a0 b0 + a1 b1) - a2 b2 (dual conic of the disc)."""
    return rs2 * (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1]) - a[:, 2] * b[:, 2]


def view_geometry64(means, scales, quats, opac, cam, rp: RasterParams = RasterParams()):
    """Per-surfel float64 projection of one view.

    Returns a dict of arrays over all N surfels:
      p, au, av, nc (N,3); M (N,3,3) rows m1,m2,m3; center (N,2);
      culled (N,) bool; cull_reason (N,) int8 (0 none, 1 near, 2 opacity,
      3 disc behind, 4 empty rect); flip (N,) bool; rs2, rf2 (N,);
      rect (N,4) int64 [i_lo, i_hi, j_lo, j_hi] (inclusive pixel range,
      valid where not culled); tiles (N,4) [tx_lo, tx_hi, ty_lo, ty_hi];
      tiles_touched (N,) int64 (0 where culled); depth_bits (N,) uint32
      (bits of float32(p_z)); grid_tie (N,) bool.
    """
    mu = np.asarray(means, np.float64)
    s = np.asarray(scales, np.float64)
    o = np.asarray(opac, np.float64)
    N = mu.shape[0]
    vm = np.asarray(cam.viewmat, np.float64)
    Rv, tv = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = (float(np.float32(cam.fx)), float(np.float32(cam.fy)),
                      float(np.float32(cam.cx)), float(np.float32(cam.cy)))
    znear = float(np.float32(cam.znear))
    W, H = int(cam.width), int(cam.height)
    amin = float(np.float32(rp.alpha_min))

    tu, tvv, n = rotation_columns64(quats)
    p = _rot_apply(Rv, mu)
    for i in range(3):
        p[:, i] = p[:, i] + tv[i]
    au = _rot_apply(Rv, tu) * s[:, 0:1]
    av = _rot_apply(Rv, tvv) * s[:, 1:2]
    nc = _rot_apply(Rv, n)
    dotnp = (nc[:, 0] * p[:, 0] + nc[:, 1] * p[:, 1]) + nc[:, 2] * p[:, 2]
    flip = dotnp > 0.0
    nc = np.where(flip[:, None], -nc, nc)

    # splat matrix M = K [a_u a_v p]; columns j = (a_u, a_v, p)
    X = np.stack([au[:, 0], av[:, 0], p[:, 0]], axis=1)
    Y = np.stack([au[:, 1], av[:, 1], p[:, 1]], axis=1)
    Z = np.stack([au[:, 2], av[:, 2], p[:, 2]], axis=1)
    m1 = fx * X + cx * Z
    m2 = fy * Y + cy * Z
    m3 = Z
    M = np.stack([m1, m2, m3], axis=1)

    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        L = np.log(o / amin)
        rs2 = _ceil_grid(2.0 * L)
        rf2 = _ceil_grid(L)
        # grid points straddled by a one-ulp change of the logarithm
        frac_s = 2.0 * L * GRID - np.floor(2.0 * L * GRID)
        frac_f = L * GRID - np.floor(L * GRID)
        grid_tie = (np.minimum(frac_s, 1 - frac_s) < 1e-9 * (2.0 * L * GRID + 1.0)) | \
                   (np.minimum(frac_f, 1 - frac_f) < 1e-9 * (L * GRID + 1.0))

        pz = p[:, 2]
        c_near = pz <= znear
        c_opac = o < amin
        c_disc = (pz * pz) <= rs2 * (au[:, 2] * au[:, 2] + av[:, 2] * av[:, 2])

        d13 = _conic_dot(rs2, m1, m3)
        d11 = _conic_dot(rs2, m1, m1)
        d23 = _conic_dot(rs2, m2, m3)
        d22 = _conic_dot(rs2, m2, m2)
        d33 = _conic_dot(rs2, m3, m3)
        sdx = np.sqrt(np.maximum(d13 * d13 - d11 * d33, 0.0))
        sdy = np.sqrt(np.maximum(d23 * d23 - d22 * d33, 0.0))
        xa = (d13 - sdx) / d33
        xb = (d13 + sdx) / d33
        ya = (d23 - sdy) / d33
        yb = (d23 + sdy) / d33
        ccx = m1[:, 2] / m3[:, 2]
        ccy = m2[:, 2] / m3[:, 2]
        rf = np.sqrt(rf2)
        xmin = np.minimum(np.minimum(xa, xb), ccx - rf)
        xmax = np.maximum(np.maximum(xa, xb), ccx + rf)
        ymin = np.minimum(np.minimum(ya, yb), ccy - rf)
        ymax = np.maximum(np.maximum(ya, yb), ccy + rf)
        ilo = np.maximum(np.ceil(xmin - 0.5), 0.0)
        ihi = np.minimum(np.floor(xmax - 0.5), W - 1.0)
        jlo = np.maximum(np.ceil(ymin - 0.5), 0.0)
        jhi = np.minimum(np.floor(ymax - 0.5), H - 1.0)
        # '!(lo <= hi)' also rejects NaN
        c_rect = ~((ilo <= ihi) & (jlo <= jhi))

    reason = np.zeros(N, np.int8)
    reason[c_rect] = 4
    reason[c_disc] = 3
    reason[c_opac] = 2
    reason[c_near] = 1
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
    depth_bits = pz.astype(np.float32).view(np.uint32).copy()
    return dict(p=p, au=au, av=av, nc=nc, M=M, center=np.stack([ccx, ccy], axis=1),
                culled=culled, cull_reason=reason, flip=flip, rs2=rs2, rf2=rf2,
                rect=rect, tiles=tiles, tiles_touched=tt.astype(np.int64),
                depth_bits=depth_bits, grid_tie=grid_tie & ~c_opac)


def tile_layout(cams, rp: RasterParams = RasterParams()):
    """Per view (tiles_x, tiles_y, tile_offset) and the total tile count;
    tile ids are global across the views, view-major then row-major."""
    out, off = [], 0
    for c in cams:
        tx = (int(c.width) + rp.tile_w - 1) // rp.tile_w
        ty = (int(c.height) + rp.tile_h - 1) // rp.tile_h
        out.append((tx, ty, off))
        off += tx * ty
    return out, off


def instances64(geom, view_tile_offset: int, tiles_x: int):
    """Unsorted (key, id) instances of one view: for every surfel that is
    not culled, one entry per tile of its tile rectangle."""
    ok = np.nonzero(~geom["culled"])[0]
    t = geom["tiles"][ok]
    counts = geom["tiles_touched"][ok]
    total = int(counts.sum())
    gid = np.repeat(ok, counts)
    start = np.repeat(np.cumsum(counts) - counts, counts)
    local = np.arange(total) - start
    w = np.repeat(t[:, 1] - t[:, 0] + 1, counts)
    tx = np.repeat(t[:, 0], counts) + local % w
    ty = np.repeat(t[:, 2], counts) + local // w
    tile = view_tile_offset + ty * tiles_x + tx
    keys = (tile.astype(np.uint64) << np.uint64(32)) | geom["depth_bits"][gid].astype(np.uint64)
    return keys, gid.astype(np.uint32)


def bin64(geoms, cams, rp: RasterParams = RasterParams()):
    """Sorted instance list and per-tile ranges over all views: one instance
    per (tile, surfel) of the surfel's tile rectangle; keys (uint64) = global
    tile id << 32 | depth bits ascending, ties by surfel id ascending
    (np.lexsort); vals = surfel ids; ranges (T,2) uint32 with [start, end)
    of every global tile, [0,0) when empty."""
    lay, total_tiles = tile_layout(cams, rp)
    ks, vs = [], []
    for g, (tx, ty, off) in zip(geoms, lay):
        k, v = instances64(g, off, tx)
        ks.append(k)
        vs.append(v)
    keys = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
    vals = np.concatenate(vs) if vs else np.zeros(0, np.uint32)
    order = np.lexsort((vals, keys))
    keys, vals = keys[order], vals[order]
    ranges = np.zeros((total_tiles, 2), np.uint32)
    if keys.size:
        tile = (keys >> np.uint64(32)).astype(np.int64)
        first = np.ones(keys.size, bool)
        first[1:] = tile[1:] != tile[:-1]
        last = np.ones(keys.size, bool)
        last[:-1] = tile[1:] != tile[:-1]
        idx = np.arange(keys.size, dtype=np.int64)
        ranges[tile[first], 0] = idx[first]
        ranges[tile[last], 1] = idx[last] + 1
    return keys, vals, ranges
