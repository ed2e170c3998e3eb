"""Differentiable FP64 per-pixel compositing of surfels (oracle; test
infrastructure only).

Follows the paper's description of rendering (Section 3.1 and Section 4.3):
every pixel blends the Gaussians assigned to it in front-to-back order,
accumulating colour and opacity, and stops once the accumulated opacity
reaches a threshold close to one or the list is exhausted.  The outputs are
the ones the paper's losses consume: colour R, accumulated alpha A (Eq. 1),
depth, normal and the depth distortion of the 2DGS regularisers (Eq. 3).

Readings of what the paper leaves to the underlying renderers (listed with
reasons in the design notes):
  * pixel (i, j) is sampled at x = (i + 1/2, j + 1/2);
  * the ray through x hits the surfel plane p + u a_u + v a_v at
    (u, v, tau), the solution of [a_u a_v -d] (u,v,tau)^T = -p with
    d = ((x - c_x)/f_x, (y - c_y)/f_y, 1) (Cramer's rule; a singular system
    gives G_s = 0);
  * G_s = exp(-(u^2+v^2)/2) at depth tau; the screen-space low-pass value is
    G_f = exp(-|x - c|^2) at the centre depth p_z; the larger one is used
    (equality takes the surface value);
  * a = min(alpha_max, o G); an entry with a < alpha_min is skipped;
    blending stops before an entry k when T (1 - a_k) < t_min;
  * omega_k = a_k T_k; C = sum omega c + T_final bg; A = 1 - T_final;
    depth = sum omega z; normal = sum omega n_c;
    dist = sum_{i,j} omega_i omega_j (z_i - z_j)^2 over ordered pairs;
    median depth = z of the last blended entry that starts with T > 1/2
    (0 when there is none), the 2DGS median depth.
The per-pixel list is every surfel that is not culled and whose pixel
rectangle (``geometry.view_geometry64``) contains the pixel, in ascending
(float32 centre depth, id).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np
import torch

from .geometry import RasterParams
from .sh import sh_colour

DT = torch.float64

# Tie windows for the flags that mark pixels where a float32 evaluation may
# legitimately take the other side of a threshold (both results are then
# correct; ``render_alternatives`` gives the other one).  A float32
# evaluation of o G is exact to a few float32 ulps of the exponent (a
# relative error of order 1e-7 to 1e-6: rounding of the record, of
# rho = u^2 + v^2 and of the log-space cutoff); T (1 - a) accumulates the
# rounding of one product per blended entry (order 1e-6 after a hundred).
# Measured on 64x64 crops of the 16-view, 1M-surfel benchmark scene
# (131,072 pixels, about 11,000 entries within 1e-3 of a threshold): where
# only one result matched, float32 took the other side at relative
# distances up to 3.3e-7 (cutoff and termination alike).  The windows are
# ten and thirty times that.
TIE_CUTOFF_REL = 3e-6      # |o G - alpha_min| <= 3e-6 alpha_min
TIE_TERM_REL = 1e-5        # |T (1 - a) - t_min| <= 1e-5 t_min
# The wide windows of the tie protocol: |o G - alpha_min| <= 2e-6 (absolute;
# the pruning exemption of the benchmark description is 1e-6 on the weight)
# and |T (1 - a) - t_min| <= 1e-4 t_min.  Entries of surfels seen at a
# steep angle or close to the camera can carry float32 errors of the order
# of 1e-4 relative (measured: cutoff decisions taken the other way at up to
# 8.8e-5, termination at 1.4e-5, on the 100-view shell scene): a pixel that
# matches no result under the primary windows is resolved under these.
WIDE_CUTOFF_REL = 2e-6 / float(np.float32(1.0 / 255.0))
WIDE_TERM_REL = 1e-4
TIE_BRANCH = 1e-6          # |G_s - G_f|
TIE_CLAMP = 1e-6           # |o G - alpha_max|
TIE_MEDIAN = 1e-5          # |T_before - 1/2| at a blended entry (median depth)


@dataclass
class Params64:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opac: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @staticmethod
    def from_arrays(means, scales, quats, opac, sh, sh_degree, requires_grad=False):
        ts = [torch.tensor(np.asarray(a, np.float64), dtype=DT, requires_grad=requires_grad)
              for a in (means, scales, quats, opac, sh)]
        return Params64(*ts, sh_degree=int(sh_degree))

    def leaves(self):
        return [self.means, self.scales, self.quats, self.opac, self.sh]

    def grads(self):
        return [None if t.grad is None else t.grad.detach().numpy().copy() for t in self.leaves()]

    def zero_grad(self):
        for t in self.leaves():
            t.grad = None


def quat_to_frame(q: torch.Tensor):
    """Columns (t_u, t_v, n) of the rotation of q/|q|, q = (w,x,y,z)."""
    qn = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    tu = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], dim=-1)
    tv = torch.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], dim=-1)
    n = torch.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)], dim=-1)
    return tu, tv, n


def _cross(a, b):
    return torch.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                        a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                        a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], dim=-1)


def _dot(a, b):
    return (a * b).sum(dim=-1)


def surfel_view_quantities(P: Params64, ids: np.ndarray, cam, flip: np.ndarray):
    """Differentiable camera-space quantities of the surfels ``ids``."""
    idx = torch.as_tensor(ids, dtype=torch.long)
    mu = P.means[idx]
    s = P.scales[idx]
    tu, tv, n = quat_to_frame(P.quats[idx])
    vm = torch.tensor(np.asarray(cam.viewmat, np.float64), dtype=DT)
    Rv, t = vm[:, :3], vm[:, 3]
    p = mu @ Rv.T + t
    au = s[:, 0:1] * (tu @ Rv.T)
    av = s[:, 1:2] * (tv @ Rv.T)
    sign = torch.where(torch.as_tensor(flip[ids]), -1.0, 1.0).to(DT)
    nc = sign[:, None] * (n @ Rv.T)
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    centre = torch.stack([fx * p[:, 0] / p[:, 2] + cx, fy * p[:, 1] / p[:, 2] + cy], dim=-1)
    campos = torch.tensor(np.asarray(cam.campos, np.float64), dtype=DT)
    dvec = mu - campos
    dirs = dvec / torch.linalg.norm(dvec, dim=-1, keepdim=True)
    rgb, rgb_raw = sh_colour(P.sh[idx], dirs, P.sh_degree)
    return dict(p=p, au=au, av=av, nc=nc, centre=centre, rgb=rgb, rgb_raw=rgb_raw,
                o=P.opac[idx])


def _pixel_lists(geom, pix: np.ndarray, margin: int = 1):
    """Ordered candidate lists for the pixels ``pix`` (P,2) = (i, j).

    Returns (cand ids in list order, index matrix (P,L) into cand, valid
    mask (P,L), ghost mask (P,L)).  Ghost entries are surfels whose
    rectangle grown by ``margin`` pixels contains the pixel but the
    rectangle itself does not; they never blend and only feed tie flags."""
    ok = ~geom["culled"]
    rect = geom["rect"]
    i0, i1 = pix[:, 0].min(), pix[:, 0].max()
    j0, j1 = pix[:, 1].min(), pix[:, 1].max()
    sel = ok & (rect[:, 0] - margin <= i1) & (rect[:, 1] + margin >= i0) & \
        (rect[:, 2] - margin <= j1) & (rect[:, 3] + margin >= j0)
    cand = np.nonzero(sel)[0]
    if cand.size == 0:
        z = np.zeros((pix.shape[0], 1), bool)
        return cand, np.zeros((pix.shape[0], 1), np.int64), z, z
    order = np.lexsort((cand, geom["depth_bits"][cand]))
    cand = cand[order]
    r = rect[cand]
    pi = pix[:, 0:1]
    pj = pix[:, 1:2]
    inside = (r[None, :, 0] <= pi) & (pi <= r[None, :, 1]) & (r[None, :, 2] <= pj) & (pj <= r[None, :, 3])
    near = (r[None, :, 0] - margin <= pi) & (pi <= r[None, :, 1] + margin) & \
        (r[None, :, 2] - margin <= pj) & (pj <= r[None, :, 3] + margin)
    cnt = near.sum(axis=1)
    L = int(cnt.max()) if cnt.size else 0
    L = max(L, 1)
    # stable compaction of the 'near' columns to the front of each row
    key = np.where(near, 0, 1)
    colorder = np.argsort(key, axis=1, kind="stable")[:, :L]
    valid = np.take_along_axis(near, colorder, axis=1)
    ghost = valid & ~np.take_along_axis(inside, colorder, axis=1)
    return cand, colorder, valid, ghost


def _composite(Q, cam, pix, colidx, valid, ghost, rp: RasterParams, flip=None, windows=None):
    """Front-to-back compositing of a chunk of pixels.  ``flip`` (optional)
    holds (P,L) boolean masks "cut", "term" and "branch" of entries whose
    decision is taken the other way: the cutoff test, the termination test
    and the surface/low-pass choice (an alternative result where float32
    may land on the other side of a threshold)."""
    Pn, L = colidx.shape
    ci = torch.as_tensor(colidx, dtype=torch.long)
    g = lambda t: t[ci]                                    # (P,L,...)
    p, au, av = g(Q["p"]), g(Q["au"]), g(Q["av"])
    fx, fy, cx, cy = (float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy))
    x = torch.as_tensor(pix[:, 0] + 0.5, dtype=DT)[:, None].expand(Pn, L)
    y = torch.as_tensor(pix[:, 1] + 0.5, dtype=DT)[:, None].expand(Pn, L)
    if "shift" in Q:
        # the surfel translated by delta in screen space is seen at x - delta
        sh = g(Q["shift"])
        x = x - sh[..., 0]
        y = y - sh[..., 1]
    d = torch.stack([(x - cx) / fx, (y - cy) / fy, torch.ones_like(x)], dim=-1)
    # Cramer's rule for [a_u a_v -d] (u, v, tau)^T = -p
    c1, c2, c3, b = au, av, -d, -p
    det = _dot(c1, _cross(c2, c3))
    sing = det == 0
    dsafe = torch.where(sing, torch.ones_like(det), det)
    u = _dot(b, _cross(c2, c3)) / dsafe
    v = _dot(c1, _cross(b, c3)) / dsafe
    tau = _dot(c1, _cross(c2, b)) / dsafe
    Gs = torch.where(sing, torch.zeros_like(u), torch.exp(-(u * u + v * v) / 2))
    ctr = g(Q["centre"])
    dx = x - ctr[..., 0]
    dy = y - ctr[..., 1]
    Gf = torch.exp(-(dx * dx + dy * dy))
    surf = Gs >= Gf
    if flip is not None:
        surf = surf ^ torch.as_tensor(flip["branch"])
    G = torch.where(surf, Gs, Gf)
    z = torch.where(surf, tau, p[..., 2])
    o = g(Q["o"])
    a_raw = o * G
    a = torch.clamp(a_raw, max=rp.alpha_max)

    vt = torch.as_tensor(valid)
    gt = torch.as_tensor(ghost)
    cut = a < rp.alpha_min
    if flip is not None:
        cut = cut ^ torch.as_tensor(flip["cut"])
    skip = cut | ~vt | gt
    one_minus = torch.where(skip, torch.ones_like(a), 1 - a)
    T_after = torch.cumprod(one_minus, dim=1)
    T_before = torch.cat([torch.ones_like(T_after[:, :1]), T_after[:, :-1]], dim=1)
    term = T_after < rp.t_min
    if flip is not None:
        term = term ^ torch.as_tensor(flip["term"])
    stop = (~skip) & term
    has_stop = stop.any(dim=1)
    first_stop = torch.where(has_stop, stop.to(torch.int64).argmax(dim=1), torch.full((Pn,), L))
    k = torch.arange(L)[None, :]
    reached = vt & (k <= first_stop[:, None])
    blended = (~skip) & (k < first_stop[:, None])
    w = torch.where(blended, a * T_before, torch.zeros_like(a))
    T_final = torch.prod(torch.where(blended, 1 - a, torch.ones_like(a)), dim=1)

    rgb = g(Q["rgb"])
    nc = g(Q["nc"])
    bg = torch.tensor(np.asarray(cam.bg, np.float64), dtype=DT)
    color = (w[..., None] * rgb).sum(dim=1) + T_final[:, None] * bg
    alpha = 1 - T_final
    depth = (w * z).sum(dim=1)
    normal = (w[..., None] * nc).sum(dim=1)
    # distortion: literal double sum over the blended entries
    nb = blended.sum(dim=1)
    Lb = max(int(nb.max()), 1)
    border = torch.argsort((~blended).to(torch.int8), dim=1, stable=True)[:, :Lb]
    wb = torch.gather(w, 1, border)
    zb = torch.gather(z, 1, border)
    bmask = torch.gather(blended, 1, border)
    wb = torch.where(bmask, wb, torch.zeros_like(wb))
    zb = torch.where(bmask, zb, torch.zeros_like(zb))
    dz = zb[:, :, None] - zb[:, None, :]
    dist = (wb[:, :, None] * wb[:, None, :] * dz * dz).sum(dim=(1, 2))

    last = torch.where(blended, k.expand(Pn, L), torch.full_like(k.expand(Pn, L), -1)).max(dim=1).values
    n_contrib = (last + 1)
    # median depth: the depth of the last blended entry that starts with
    # T > 1/2 (0 without one); median_idx is that entry's 1-based list index
    med_cand = blended & (T_before > 0.5)
    kmed = torch.where(med_cand, k.expand(Pn, L), torch.full_like(k.expand(Pn, L), -1)).max(dim=1).values
    has_med = kmed >= 0
    zmed = torch.gather(z, 1, kmed.clamp(min=0)[:, None])[:, 0]
    median_depth = torch.where(has_med, zmed, torch.zeros_like(zmed))
    median_idx = kmed + 1

    with torch.no_grad():
        w_cut, w_term = (TIE_CUTOFF_REL, TIE_TERM_REL) if windows is None else windows
        # an entry outside its surfel's pixel rectangle (bit-exact on both
        # sides) is never evaluated, so it cannot make a tie
        nsk = reached & ~gt
        e_cut = nsk & ((a_raw - rp.alpha_min).abs() <= w_cut * rp.alpha_min)
        e_term = nsk & ~skip & ((T_before * (1 - a) - rp.t_min).abs() <= w_term * rp.t_min)
        e_branch = blended & ((Gs - Gf).abs() <= TIE_BRANCH)
        e_clamp = blended & ((a_raw - rp.alpha_max).abs() <= TIE_CLAMP)
        e_median = blended & ((T_before - 0.5).abs() <= TIE_MEDIAN)
        f_median = e_median.any(dim=1)
        f_cut, f_term = e_cut.any(dim=1), e_term.any(dim=1)
        f_branch, f_clamp = e_branch.any(dim=1), e_clamp.any(dim=1)
        tie_entry = e_cut | e_term | e_branch | e_clamp
        tie_kinds = torch.stack([e_cut, e_term, e_branch, e_clamp, e_median], dim=-1)
        # signed distance of each entry from each threshold (relative for the
        # cutoff and the termination test)
        tie_dist = torch.stack([(a_raw - rp.alpha_min) / rp.alpha_min,
                                (T_before * (1 - a) - rp.t_min) / rp.t_min,
                                Gs - Gf, a_raw - rp.alpha_max, T_before - 0.5], dim=-1)
    return dict(tie_kinds=tie_kinds, tie_dist=tie_dist, color=color, alpha=alpha, depth=depth, normal=normal, dist=dist,
                T_final=T_final, n_contrib=n_contrib, blended=blended, reached=reached,
                a=a, w=w, z=z, surf=surf, skip=skip, first_stop=first_stop,
                clamp=a_raw > rp.alpha_max, tie_entry=tie_entry,
                flag_cut=f_cut, flag_term=f_term, flag_branch=f_branch, flag_clamp=f_clamp,
                median_depth=median_depth, median_idx=median_idx, flag_median=f_median)


OUT_KEYS = ("color", "alpha", "depth", "normal", "dist", "T_final", "median_depth")
TIE_KINDS = ("cut", "term", "branch", "clamp", "median")


def render_pixels(P: Params64, cam, geom, pix: np.ndarray, rp: RasterParams = RasterParams(),
                  loss_fn: Optional[Callable] = None, max_entries: int = 1_500_000,
                  keep_decisions: bool = False, screen_shift: Optional[torch.Tensor] = None,
                  flips: Optional[dict] = None, windows=None):
    """Render the pixels ``pix`` (P,2) int (column i, row j) of one view.

    Returns numpy arrays: color (P,3), alpha, depth, normal (P,3), dist,
    T_final, n_contrib (count of list entries up to the last blended one),
    last_gid (id of the last blended surfel, -1 if none), nblend; the tie
    flags flag_cut, flag_term, flag_branch, flag_clamp; ``pairs`` with the
    blended (pixel, id, a, omega) entries; ``flag_ids``: ids of surfels
    reached at a flagged pixel.  With ``loss_fn(out_chunk, rows)`` the
    returned scalar of every chunk is back-propagated into the leaves of
    ``P`` (the chunked sum is the full loss), so no graph outlives a chunk.
    ``screen_shift`` (N,2): every surfel translated in screen space by that
    many pixels (evaluated at x - shift); with requires_grad and zeros, the
    chunks' backward leaves dL/d(shift), the screen-space gradient of the
    density-control statistic.
    ``tie_list`` (K,3) lists the tie entries: (row of ``pix``, surfel id,
    kind) with kind TIE_KINDS.index of the threshold it sits at, and
    ``tie_dist`` (K,) each one's signed distance from that threshold
    (relative to it for the cutoff and the termination test).
    ``flips`` {row: [(surfel id, kind), ...]} takes the decision of those
    entries of that pixel the other way (kind "cut", "term" or "branch"; see
    ``render_alternatives``).  ``windows`` = (cutoff, termination) relative
    tie windows (default TIE_CUTOFF_REL, TIE_TERM_REL).
    """
    pix = np.asarray(pix, np.int64).reshape(-1, 2)
    Pn = pix.shape[0]
    res = {k: [] for k in OUT_KEYS}
    extra = {k: [] for k in ("n_contrib", "last_gid", "nblend", "flag_cut", "flag_term",
                             "flag_branch", "flag_clamp", "median_idx", "flag_median")}
    pairs, flag_ids, tie_ids, decisions, tie_list, tie_dist = [], [], [], [], [], []
    start = 0
    step = max(1, min(Pn, 1024))
    while start < Pn:
        stop = min(Pn, start + step)
        sub = pix[start:stop]
        cand, colidx, valid, ghost = _pixel_lists(geom, sub)
        if colidx.shape[0] * colidx.shape[1] > max_entries and step > 1:
            step = max(1, step // 2)
            continue
        ids = cand if cand.size else np.zeros(1, np.int64)
        if cand.size == 0:
            valid = np.zeros_like(valid)
            colidx = np.zeros_like(colidx)
        Q = surfel_view_quantities(P, ids, cam, geom["flip"])
        if screen_shift is not None:
            Q["shift"] = screen_shift[torch.as_tensor(ids, dtype=torch.long)]
        fl_masks = None
        if flips:
            gm = ids[colidx]
            fl_masks = {k: np.zeros(colidx.shape, bool) for k in ("cut", "term", "branch")}
            for r in range(start, stop):
                for gid, kind in flips.get(r, ()):
                    fl_masks[kind][r - start] |= valid[r - start] & (gm[r - start] == gid)
        out = _composite(Q, cam, sub, colidx, valid, ghost, rp, flip=fl_masks, windows=windows)
        if loss_fn is not None:
            lval = loss_fn(out, np.arange(start, stop))
            if lval is not None and lval.requires_grad:
                lval.backward()
        for k in OUT_KEYS:
            res[k].append(out[k].detach().numpy())
        bl = out["blended"].numpy()
        ncon = out["n_contrib"].numpy()
        gid_mat = ids[colidx]
        last_gid = np.where(ncon > 0, gid_mat[np.arange(sub.shape[0]), np.maximum(ncon - 1, 0)], -1)
        midx = out["median_idx"].numpy()
        extra.setdefault("median_gid", []).append(
            np.where(midx > 0, gid_mat[np.arange(sub.shape[0]), np.maximum(midx - 1, 0)], -1))
        extra["n_contrib"].append(ncon)
        extra["last_gid"].append(last_gid)
        extra["nblend"].append(bl.sum(axis=1))
        for k in ("flag_cut", "flag_term", "flag_branch", "flag_clamp", "median_idx", "flag_median"):
            extra[k].append(out[k].numpy())
        tk = out["tie_kinds"].numpy()
        tr, tc, tkind = np.nonzero(tk)
        if tr.size:
            gid_t = (ids[colidx])[tr, tc]
            tie_list.append(np.stack([tr + start, gid_t, tkind], axis=1))
            tie_dist.append(out["tie_dist"].detach().numpy()[tr, tc, tkind])
        rr, cc = np.nonzero(bl)
        pairs.append(np.stack([rr + start, gid_mat[rr, cc]], axis=1) if rr.size else np.zeros((0, 2), np.int64))
        pairs_a = out["a"].detach().numpy()[rr, cc]
        pairs_w = out["w"].detach().numpy()[rr, cc]
        pairs[-1] = (pairs[-1], pairs_a, pairs_w)
        fl = out["flag_cut"].numpy() | out["flag_term"].numpy() | out["flag_branch"].numpy() | \
            out["flag_clamp"].numpy()
        if fl.any():
            rch = out["reached"].numpy()
            fr, fc = np.nonzero(rch & fl[:, None])
            flag_ids.append(np.unique(gid_mat[fr, fc]))
            te = out["tie_entry"].numpy()
            tie_ids.append(np.unique(gid_mat[te]))
        if keep_decisions:
            decisions.append({k: out[k].detach().numpy() for k in
                              ("blended", "skip", "surf", "first_stop", "clamp")} | {"gid": gid_mat})
        start = stop
    result = {k: np.concatenate(v, axis=0) if v else np.zeros((0,)) for k, v in res.items()}
    for k, v in extra.items():
        result[k] = np.concatenate(v, axis=0) if v else np.zeros((0,))
    if pairs:
        result["pairs"] = (np.concatenate([p[0] for p in pairs]), np.concatenate([p[1] for p in pairs]),
                           np.concatenate([p[2] for p in pairs]))
    else:
        result["pairs"] = (np.zeros((0, 2), np.int64), np.zeros(0), np.zeros(0))
    result["flag_ids"] = np.unique(np.concatenate(flag_ids)) if flag_ids else np.zeros(0, np.int64)
    result["tie_ids"] = np.unique(np.concatenate(tie_ids)) if tie_ids else np.zeros(0, np.int64)
    if tie_list:
        tl = np.concatenate(tie_list).astype(np.int64)
        td = np.concatenate(tie_dist)
        o = np.lexsort((tl[:, 2], tl[:, 1], tl[:, 0]))
        result["tie_list"], result["tie_dist"] = tl[o], td[o]
    else:
        result["tie_list"], result["tie_dist"] = np.zeros((0, 3), np.int64), np.zeros(0)
    if keep_decisions:
        result["decisions"] = decisions
    return result


def render_view(P: Params64, cam, geom, rp: RasterParams = RasterParams(), crop=None, **kw):
    """Render a whole view, or the crop (x0, y0, w, h), row-major pixels."""
    if crop is None:
        crop = (0, 0, int(cam.width), int(cam.height))
    x0, y0, w, h = crop
    jj, ii = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    pix = np.stack([ii.ravel(), jj.ravel()], axis=1)
    return render_pixels(P, cam, geom, pix, rp, **kw), pix


def render_alternatives(P: Params64, cam, geom, pix: np.ndarray, tie_list: np.ndarray,
                        rp: RasterParams = RasterParams(), max_ties: int = 4,
                        kinds=("cut", "term", "branch"), windows=None):
    """The other correct results of pixels whose list holds a tie entry.

    Where a value sits within float32 reach of a threshold (the alpha cutoff
    and the termination test of Section 4.3's front-to-back blending, and
    the surface/low-pass choice), an exact evaluation and a float32 one may
    decide it differently, and both results are correct.  For every pixel
    row of ``pix`` with at most ``max_ties`` tie entries of the given kinds
    (``tie_list`` of ``render_pixels``), the pixel is rendered once per
    non-empty subset of those entries taken the other way.

    Returns (alts, results, unresolved): ``alts`` a list of (row, flips)
    with flips a tuple of (surfel id, kind); ``results`` the render_pixels
    output whose i-th pixel is alts[i]; ``unresolved`` the rows with more
    tie entries than ``max_ties``.
    """
    codes = [TIE_KINDS.index(k) for k in kinds]
    tl = tie_list[np.isin(tie_list[:, 2], codes)] if len(tie_list) else np.zeros((0, 3), np.int64)
    alts, unresolved = [], []
    for row in np.unique(tl[:, 0]):
        ent = [(int(g), TIE_KINDS[int(k)]) for _, g, k in tl[tl[:, 0] == row]]
        if len(ent) > max_ties:
            unresolved.append(int(row))
            continue
        for m in range(1, 1 << len(ent)):
            alts.append((int(row), tuple(e for b, e in enumerate(ent) if m >> b & 1)))
    if not alts:
        return alts, None, unresolved
    alt_pix = np.asarray([pix[r] for r, _ in alts], np.int64).reshape(-1, 2)
    flips = {i: list(f) for i, (_, f) in enumerate(alts)}
    res = render_pixels(P, cam, geom, alt_pix, rp, flips=flips, windows=windows)
    return alts, res, unresolved
