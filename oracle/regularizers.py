"""The 2DGS regularisers of the total loss, Eq. 3 (oracle; test
infrastructure only).

Eq. 3 adds alpha L_d + beta L_n to the masked photometric and background
losses: the depth distortion and normal consistency losses of 2DGS, not
masked (Section 4.2), with 2DGS's coefficients (Section 5.1 leaves them
unchanged).  The paper names the two terms without defining them; the
readings taken here (listed with reasons in the design notes) are

  L_d,v   mean over the pixels of the rendered distortion
          dist(p) = sum_ij w_i w_j (z_i - z_j)^2 (a rasterizer output)
  s(p)    surface depth D(p) / A(p) where A(p) > 0, else 0 (the expected
          depth normalised by the accumulated opacity), or the median depth
          (the depth of the last blended entry starting with T > 1/2) when
          that variant is chosen
  P(p)    s(p) * ((i + 0.5 - c_x) / f_x, (j + 0.5 - c_y) / f_y, 1), the point
          seen by pixel p = (i, j) in camera space
  N_d(p)  n / max(|n|, 1e-12) with the central differences
          n = (P(i, j+1) - P(i, j-1)) x (P(i+1, j) - P(i-1, j)) at pixels
          with all four neighbours, 0 on the one-pixel border; for a surface
          in front of the camera it points towards the camera, like the
          rendered normals
  L_n,v   mean over the pixels of A(p) - N(p) . N_d(p), i.e.
          sum_i w_i (1 - n_i . N_d) with N = sum_i w_i n_i the rendered normal
  L_reg = (1/V) sum_v (w_dist L_d,v + w_normal L_n,v)

The gradients flow into A, D, N and dist; N_d is not detached, so D and A
also receive the gradient through the depth normals of their neighbours.
Everything is float64 torch; gradients come from autograd of these plain
definitions.
"""
from __future__ import annotations

import numpy as np
import torch

EPS_NORMAL = 1e-12


def _t(x):
    return x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, np.float64))


def surface_depth64(alpha, depth):
    """s = D / A where A > 0, else 0; (H,W)."""
    A, D = _t(alpha), _t(depth)
    pos = A > 0
    safe = torch.where(pos, A, torch.ones_like(A))
    return torch.where(pos, D / safe, torch.zeros_like(D))


def depth_points64(alpha, depth, cam, median=None):
    """Camera-space points P(p) = s(p) * ray(p); (H,W,3).  With ``median``
    the surface depth is the median depth instead of D / A."""
    s = surface_depth64(alpha, depth) if median is None else _t(median)
    H, W = s.shape
    ii = torch.arange(W, dtype=torch.float64)[None, :].expand(H, W)
    jj = torch.arange(H, dtype=torch.float64)[:, None].expand(H, W)
    rx = (ii + 0.5 - float(cam.cx)) / float(cam.fx)
    ry = (jj + 0.5 - float(cam.cy)) / float(cam.fy)
    return torch.stack([s * rx, s * ry, s], dim=-1)


def depth_normal64(alpha, depth, cam, median=None):
    """N_d of every pixel (zero on the border); (H,W,3)."""
    P = depth_points64(alpha, depth, cam, median)
    H, W, _ = P.shape
    out = torch.zeros_like(P)
    if H < 3 or W < 3:
        return out
    a = P[2:, 1:-1] - P[:-2, 1:-1]      # along +j (rows)
    b = P[1:-1, 2:] - P[1:-1, :-2]      # along +i (columns)
    n = torch.cross(a, b, dim=-1)
    nrm = torch.sqrt((n * n).sum(dim=-1, keepdim=True))
    nd = n / torch.clamp(nrm, min=EPS_NORMAL)
    out = torch.cat([torch.zeros(1, W - 2, 3, dtype=P.dtype), nd, torch.zeros(1, W - 2, 3, dtype=P.dtype)], dim=0)
    out = torch.cat([torch.zeros(H, 1, 3, dtype=P.dtype), out, torch.zeros(H, 1, 3, dtype=P.dtype)], dim=1)
    return out


def regularizer_view64(alpha, depth, normal, dist, cam, median=None):
    """(L_d, L_n) of one view; normal (3,H,W) planar like the rasterizer;
    ``median`` (H,W) selects the median-depth surface."""
    A, D, N, S = _t(alpha), _t(depth), _t(normal), _t(dist)
    Nd = depth_normal64(A, D, cam, median)
    L_d = S.mean()
    L_n = (A - (N.permute(1, 2, 0) * Nd).sum(dim=-1)).mean()
    return L_d, L_n


def regularizer_loss64(alphas, depths, normals, dists, cams, w_dist, w_normal, medians=None):
    """Per-view (L_d, L_n), the total (1/V) sum_v (w_dist L_d + w_normal L_n)
    and its gradients with respect to every input map (numpy float64).

    alphas, depths, dists: lists of (H,W); normals: list of (3,H,W);
    medians: optional list of (H,W) median depths (the surface depth of the
    normal consistency term; their gradients are returned as "median")."""
    V = len(alphas)
    ts = []
    for v in range(V):
        ts.append([torch.tensor(np.asarray(x, np.float64), requires_grad=True)
                   for x in (alphas[v], depths[v], normals[v], dists[v])])
    meds = None if medians is None else [torch.tensor(np.asarray(m, np.float64), requires_grad=True)
                                         for m in medians]
    per_view, total = [], 0.0
    for v in range(V):
        L_d, L_n = regularizer_view64(*ts[v], cams[v], None if meds is None else meds[v])
        per_view.append((float(L_d.detach()), float(L_n.detach())))
        total = total + w_dist * L_d + w_normal * L_n
    total = total / V
    total.backward()
    g = lambda x: x.grad.numpy() if x.grad is not None else np.zeros(tuple(x.shape))
    grads = [{"alpha": g(t[0]), "depth": g(t[1]), "normal": g(t[2]), "dist": g(t[3])} for t in ts]
    if meds is not None:
        for v in range(V):
            grads[v]["median"] = g(meds[v])
    return {"per_view": per_view, "total": float(total.detach()), "grads": grads}
