"""The library's 4x4-tile-group instance layout, derived from the oracle's
plain per-tile lists (test-side transform; no renderer arithmetic).

The HIP binning stores one instance per (tile group, surfel) whose tile
rectangle meets the group, sorted by (global group id, float32 depth, id),
with the surfel's tile rectangle clipped to the group packed above a 24-bit
id: value = id | (x_lo | x_hi << 2 | y_lo << 4 | y_hi << 6) << 24.  A tile's
own front-to-back list is the entries of its group's run whose
sub-rectangle contains the tile.  These helpers

  * build that layout from the per-tile lists of ``oracle.bin64``
    (``grouped_from_tile_lists``), so that the GPU's sorted array, keys and
    ranges can be compared with it bit for bit;
  * build the same layout directly from the oracle's per-surfel tile
    rectangles (``grouped_from_rectangles``), vectorised, for full-size
    workloads where the per-tile lists would hold hundreds of millions of
    entries; a CPU test checks that the two constructions agree;
  * expand a grouped run back to one tile's list (``tile_list``), so the
    GPU's runs can be checked against the oracle's per-tile lists.
"""
from __future__ import annotations

import numpy as np

GROUP = 4
ID_BITS = 24
ID_MASK = np.uint32((1 << ID_BITS) - 1)


def group_layout(cams, tile_w: int, tile_h: int, group: int = GROUP):
    """Per view (tiles_x, tiles_y, tile_offset, groups_x, groups_y,
    group_offset); tile and group ids are global across the views,
    view-major then row-major."""
    out, toff, goff = [], 0, 0
    for c in cams:
        tx = (int(c.width) + tile_w - 1) // tile_w
        ty = (int(c.height) + tile_h - 1) // tile_h
        gx, gy = (tx + group - 1) // group, (ty + group - 1) // group
        out.append((tx, ty, toff, gx, gy, goff))
        toff += tx * ty
        goff += gx * gy
    return out


def _pack(ids, xlo, xhi, ylo, yhi):
    sub = (np.asarray(xlo) | (np.asarray(xhi) << 2) | (np.asarray(ylo) << 4) | (np.asarray(yhi) << 6))
    return np.asarray(ids, np.uint32) | (sub.astype(np.uint32) << np.uint32(ID_BITS))


def _tile_ranges(granges, lay, group):
    """Per global tile, the [start, end) of its group's run."""
    T = sum(tx * ty for tx, ty, *_ in lay)
    ranges = np.zeros((T, 2), np.uint32)
    for tx, ty, toff, gx, gy, goff in lay:
        t = np.arange(tx * ty)
        gid = goff + (t // tx // group) * gx + (t % tx) // group
        ranges[toff + t] = granges[gid]
    return ranges


def _group_runs(gkeys, ngroups):
    granges = np.zeros((ngroups, 2), np.uint32)
    if gkeys.size:
        first = np.ones(gkeys.size, bool)
        first[1:] = gkeys[1:] != gkeys[:-1]
        last = np.ones(gkeys.size, bool)
        last[:-1] = gkeys[1:] != gkeys[:-1]
        idx = np.arange(gkeys.size, dtype=np.int64)
        granges[gkeys[first], 0] = idx[first]
        granges[gkeys[last], 1] = idx[last] + 1
    return granges


def grouped_from_tile_lists(keys, vals, ranges, cams, tile_w: int, tile_h: int, group: int = GROUP):
    """The grouped layout from the per-tile sorted lists of ``oracle.bin64``
    (keys = tile << 32 | depth bits, vals = surfel ids, ranges per tile):
    the entries of a group are the surfels of its tiles' lists, once each,
    in (depth, id) order; the sub-rectangle is the bounding box of the
    group's tiles whose lists hold the surfel.  Returns (keys64, vals,
    ranges) as the library writes them."""
    lay = group_layout(cams, tile_w, tile_h, group)
    gk, gv = [], []
    for tx, ty, toff, gx, gy, goff in lay:
        for g in range(gx * gy):
            grow, gcol = divmod(g, gx)
            ent = {}
            for sy in range(group):
                for sx in range(group):
                    cx, cy = gcol * group + sx, grow * group + sy
                    if cx >= tx or cy >= ty:
                        continue
                    s, e = (int(x) for x in ranges[toff + cy * tx + cx])
                    for k in range(s, e):
                        sid = int(vals[k])
                        d = int(keys[k]) & 0xFFFFFFFF
                        if sid in ent:
                            dd, x0, x1, y0, y1 = ent[sid]
                            assert dd == d, "a surfel has one depth per view"
                            ent[sid] = (d, min(x0, sx), max(x1, sx), min(y0, sy), max(y1, sy))
                        else:
                            ent[sid] = (d, sx, sx, sy, sy)
            for sid, (d, x0, x1, y0, y1) in sorted(ent.items(), key=lambda kv: (kv[1][0], kv[0])):
                gk.append(((goff + g) << 32) | d)
                gv.append(int(_pack(sid, x0, x1, y0, y1)))
    keys64 = np.asarray(gk, np.uint64)
    gvals = np.asarray(gv, np.uint32)
    ngroups = sum(gx * gy for *_, gx, gy, _ in lay)
    granges = _group_runs((keys64 >> np.uint64(32)).astype(np.int64), ngroups)
    return keys64, gvals, _tile_ranges(granges, lay, group)


def grouped_from_rectangles(geoms, cams, tile_w: int, tile_h: int, group: int = GROUP):
    """The same layout built directly from the oracle's per-surfel tile
    rectangles (``geoms[v]['tiles']``, culled surfels excluded) and depth
    bits, vectorised; the instances of a view are generated in ascending
    surfel id, so a stable sort on the 64-bit key leaves equal keys in id
    order."""
    lay = group_layout(cams, tile_w, tile_h, group)
    ks, vs = [], []
    for geom, (tx, ty, toff, gx, gy, goff) in zip(geoms, lay):
        ok = np.nonzero(~geom["culled"])[0]
        t = geom["tiles"][ok]
        g0x, g1x, g0y, g1y = t[:, 0] // group, t[:, 1] // group, t[:, 2] // group, t[:, 3] // group
        counts = (g1x - g0x + 1) * (g1y - g0y + 1)
        total = int(counts.sum())
        rep = lambda a: np.repeat(a, counts)
        gid = rep(ok)
        local = np.arange(total) - rep(np.cumsum(counts) - counts)
        w = rep(g1x - g0x + 1)
        gxx = rep(g0x) + local % w
        gyy = rep(g0y) + local // w
        ox, oy = group * gxx, group * gyy
        xlo = np.maximum(rep(t[:, 0]), ox) - ox
        xhi = np.minimum(rep(t[:, 1]), ox + group - 1) - ox
        ylo = np.maximum(rep(t[:, 2]), oy) - oy
        yhi = np.minimum(rep(t[:, 3]), oy + group - 1) - oy
        ks.append(((goff + gyy * gx + gxx).astype(np.uint64) << np.uint64(32)) |
                  geom["depth_bits"][gid].astype(np.uint64))
        vs.append(_pack(gid, xlo, xhi, ylo, yhi))
    keys = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
    vals = np.concatenate(vs) if vs else np.zeros(0, np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    ngroups = sum(gx * gy for *_, gx, gy, _ in lay)
    granges = _group_runs((keys >> np.uint64(32)).astype(np.int64), ngroups)
    return keys, vals, _tile_ranges(granges, lay, group)


def instance_count(geoms, group: int = GROUP):
    """Instances of grouped binning: per visible record, the tile groups its
    tile rectangle meets."""
    n = 0
    for g in geoms:
        t = g["tiles"][~g["culled"]]
        n += int(((t[:, 1] // group - t[:, 0] // group + 1) * (t[:, 3] // group - t[:, 2] // group + 1)).sum())
    return n


def tile_list(vals, ranges, t: int, tile_xy, group: int = GROUP):
    """Surfel ids of tile t (tile coordinates tile_xy within its view) from
    grouped lists: the entries of its group's run whose sub-rectangle
    contains the tile, in run order, with their run positions."""
    s, e = (int(x) for x in ranges[t])
    v = np.asarray(vals[s:e], np.uint32)
    sub = v >> np.uint32(ID_BITS)
    x, y = tile_xy[0] % group, tile_xy[1] % group
    inside = ((sub & 3) <= x) & (x <= ((sub >> 2) & 3)) & (((sub >> 4) & 3) <= y) & (y <= ((sub >> 6) & 3))
    return (v & ID_MASK)[inside], np.arange(s, e)[inside]


def expand_to_tile_lists(vals, ranges, cams, tile_w: int, tile_h: int, group: int = GROUP):
    """Every tile's list expanded from grouped runs, as per-tile (keys-free)
    arrays: returns (ids concatenated in global tile order, per-tile
    [start, end)), comparable with ``oracle.bin64``'s vals and ranges."""
    lay = group_layout(cams, tile_w, tile_h, group)
    out, rng = [], []
    pos = 0
    for tx, ty, toff, *_ in lay:
        for t in range(tx * ty):
            ids, _ = tile_list(vals, ranges, toff + t, (t % tx, t // tx), group)
            out.append(ids)
            rng.append((pos, pos + ids.size) if ids.size else (0, 0))
            pos += ids.size
    ids = np.concatenate(out) if out else np.zeros(0, np.uint32)
    return ids, np.asarray(rng, np.uint32).reshape(-1, 2)
