"""Torch-facing wrappers of the C ABI: device buffers, stream plumbing and
the autograd.Function.  PyTorch only provides memory and streams; every
step of the hot path runs in libsurfelrast.so.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import SrCamera, SrConfig, call

ALPHA_MIN = float(np.float32(1.0 / 255.0))
ALPHA_MAX = float(np.float32(0.99))
T_MIN = float(np.float32(1e-4))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stats(stats):
    """(hits, max_alpha, max_weight) of a forward: stats is None, the hits
    tensor alone (int32 [N], blended-pixel counts: the usage record of
    Section 4.3), or the three tensors (hits and the maxima)."""
    if stats is None:
        return None, None, None
    if isinstance(stats, torch.Tensor):
        return stats, None, None
    h, ma, mw = stats
    return h, ma, mw


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _device_index(device) -> int:
    d = torch.device(device)
    if d.type != "cuda":
        raise ValueError(f"the surfel rasterizer runs on a GPU, not on {d}")
    return d.index if d.index is not None else torch.cuda.current_device()


def _ctx(t: torch.Tensor):
    """The per-device default context for calls outside a Rasterizer."""
    return _lib.default_context(_device_index(t.device)).ptr


def make_config(sh_degree: int = 0, sh_stride: Optional[int] = None, tile=(16, 16), flags: int = 0,
                alpha_min=ALPHA_MIN, alpha_max=ALPHA_MAX, t_min=T_MIN, bwd_batch: int = 0) -> SrConfig:
    """Renderer configuration; bwd_batch: records per LDS batch of the
    backward compositing (32/64/128/256, 0: the library's default)."""
    K = (sh_degree + 1) ** 2
    return SrConfig(tile[0], tile[1], sh_degree, K if sh_stride is None else sh_stride,
                    alpha_min, alpha_max, t_min, flags, bwd_batch)


class ViewBatch:
    """V cameras laid out for one tile shape: a host array (launch geometry)
    and a byte-identical device copy (read by the kernels)."""

    def __init__(self, cams: Sequence, tile=(16, 16), device="cuda"):
        V = len(cams)
        arr = (SrCamera * max(V, 1))()
        for v, c in enumerate(cams):
            d = arr[v]
            vm = np.asarray(c.viewmat, np.float32).reshape(-1)
            for i in range(12):
                d.viewmat[i] = float(vm[i])
            d.fx, d.fy, d.cx, d.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
            for i in range(3):
                d.campos[i] = float(c.campos[i])
                d.bg[i] = float(np.asarray(c.bg)[i])
            d.znear = float(c.znear)
            d.width, d.height = int(c.width), int(c.height)
        P = ctypes.c_int64(0)
        T = ctypes.c_int32(0)
        call("sr_layout_views", ctypes.cast(arr, ctypes.c_void_p), V, tile[0], tile[1], ctypes.byref(P),
             ctypes.byref(T))
        self.host = arr
        self.V = V
        self.P = int(P.value)
        self.T = int(T.value)
        self.tile = tuple(tile)
        self.sizes = [(int(c.width), int(c.height)) for c in cams]
        self.pix_offsets = [int(arr[v].pix_offset) for v in range(V)]
        raw = bytes(memoryview(arr).cast("B"))[: 128 * V] if V else b""
        self.dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device) if V else \
            torch.zeros(128, dtype=torch.uint8, device=device)

    @property
    def host_ptr(self):
        return ctypes.cast(self.host, ctypes.c_void_p)

    def view_slice(self, v: int, channels: int = 1):
        W, H = self.sizes[v]
        o = self.pix_offsets[v]
        return slice(channels * o, channels * (o + W * H))


@dataclass
class Params:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opac: torch.Tensor
    sh: torch.Tensor

    @staticmethod
    def from_scene(scene, device="cuda"):
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)
        return Params(f(scene.means), f(scene.scales), f(scene.quats), f(scene.opac), f(scene.sh))


class Rasterizer:
    """Persistent device buffers for one (N, views, tile shape, capacity).

    preprocess -> bin -> forward -> (loss) -> backward, each one C-ABI call
    on the current torch stream; no host synchronisation except
    ``plan_capacity``, ``status`` and ``check_capacity``.  The rasterizer
    owns a context (sr_ctx): a binning that exceeds the capacity sets its
    status word, the later compositing calls flag their outputs (NaN) and
    ``check_capacity`` reports and clears it.
    """

    def __init__(self, N: int, views: ViewBatch, sh_degree: int, sh_stride: Optional[int] = None,
                 capacity: int = 0, device="cuda", shade: bool = True, bwd_batch: int = 0):
        self.N, self.views, self.device = int(N), views, device
        self.ctx = _lib.Context(_device_index(device))
        self.cfg = make_config(sh_degree, sh_stride, views.tile)
        self.set_bwd_batch(bwd_batch)
        self.shade = shade
        V, P, T = views.V, views.P, views.T
        VN = V * self.N
        i32, f32 = torch.int32, torch.float32
        z = lambda n, dt: torch.zeros(max(int(n), 1), dtype=dt, device=device)
        self.geom = z(VN * _lib.SR_GEOM_STRIDE, f32)
        self.app = z(VN * _lib.SR_APP_STRIDE, f32) if shade else None
        self.rect = z(VN * 4, torch.int16)
        self.tiles_touched = z(VN, i32)
        self.depth_key = z(VN, i32)
        self.in_frustum = z(self.N, torch.uint8)
        self.ranges = z(2 * T, i32)
        self.counters = z(_lib.SR_COUNTERS, i32)
        # forward outputs / saved state
        self.color = z(3 * P, f32)
        self.alpha = z(P, f32)
        self.depth = z(P, f32)
        self.normal = z(3 * P, f32)
        self.dist = z(P, f32)
        self.T_final = z(P, f32)
        self.n_contrib = z(P, i32)
        self.grad_rec = None
        self.loss_ws = z(_lib.workspace_bytes_loss(V, views.host), torch.uint8) if V else z(1, torch.uint8)
        self.loss_out = z(2 * max(V, 1) + 1, f32)
        self.capacity = 0
        self.set_capacity(capacity)

    # -- capacity ---------------------------------------------------------
    def set_capacity(self, cap: int):
        cap = int(cap)
        if cap == self.capacity and getattr(self, "ws", None) is not None:
            return
        self.capacity = cap
        self.vals = torch.zeros(max(cap, 1), dtype=torch.int32, device=self.device)
        ws = _lib.workspace_bytes_bin(self.N, self.views.V, cap)
        self.ws = torch.zeros(max(ws, 1), dtype=torch.uint8, device=self.device)
        self.ws_bytes = ws

    def count_instances(self, stream=None) -> int:
        """Instances the binning of the current projection needs: a
        count-only sr_bin_and_sort (one host sync)."""
        call("sr_bin_and_sort", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_key),
             _ptr(self.ws), self.ws_bytes, 0, None, None, _ptr(self.ranges), _ptr(self.counters), _stream(stream))
        return int(self.counters[1:2].cpu().numpy().view(np.uint32)[0])

    def plan_capacity(self, params: Params, slack: float = 1.05) -> int:
        """Projects once and sizes the instance buffers (one host sync)."""
        self.preprocess(params)
        need = self.count_instances()
        self.set_capacity(int(need * slack) + 1024)
        return need

    # -- steps ------------------------------------------------------------
    def set_bwd_batch(self, batch: int):
        """Records per LDS batch of the backward compositing (0: the
        library's default for the tile shape)."""
        tw, th = self.views.tile
        if not _lib.lib().sr_bwd_batch_supported(tw, th, int(batch)):
            raise ValueError(f"backward batch {batch} is not compiled for {tw}x{th} tiles")
        self.cfg.bwd_batch = int(batch)

    def preprocess(self, p: Params, stream=None):
        call("sr_preprocess", self.ctx.ptr, ctypes.byref(self.cfg), self.N, _ptr(p.means), _ptr(p.scales), _ptr(p.quats),
             _ptr(p.opac), _ptr(p.sh), self.views.V, self.views.host_ptr, _ptr(self.views.dev), _ptr(self.geom),
             _ptr(self.app) if self.shade else None, _ptr(self.rect), _ptr(self.tiles_touched),
             _ptr(self.depth_key), _ptr(self.in_frustum), _stream(stream))

    def bin(self, keys64: Optional[torch.Tensor] = None, stream=None):
        call("sr_bin_and_sort", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_key),
             _ptr(self.ws), self.ws_bytes, self.capacity, _ptr(self.vals), _ptr(keys64), _ptr(self.ranges),
             _ptr(self.counters), _stream(stream))

    def _cfg(self, accumulate: bool):
        if not accumulate:
            return self.cfg
        cfg = SrConfig.from_buffer_copy(self.cfg)
        cfg.flags |= _lib.SR_FLAG_ACCUMULATE
        return cfg

    def _schedule(self, stream=None):
        """(order, cost) of a scheduled launch: the tile order sorted from the
        last recorded tile costs, heaviest first (None before any), and the
        buffer the launch records this step's costs into."""
        T = self.views.T
        if T == 0:
            return None, None
        if getattr(self, "tile_cost", None) is None:
            self.tile_cost = torch.zeros(T, dtype=torch.int32, device=self.device)
            self.tile_order = torch.zeros(T, dtype=torch.int32, device=self.device)
            n = ctypes.c_size_t(0)
            call("sr_tile_order_workspace_size", T, ctypes.byref(n))
            self.order_ws = torch.zeros(max(n.value, 1), dtype=torch.uint8, device=self.device)
            self.costs_recorded = False
        order = None
        if self.costs_recorded:
            call("sr_tile_order", self.ctx.ptr, T, _ptr(self.tile_cost), _ptr(self.order_ws), self.order_ws.numel(),
                 _ptr(self.tile_order), _stream(stream))
            order = self.tile_order
        return order, self.tile_cost

    def forward(self, stats=None, accumulate: bool = False, stream=None, median: bool = False,
                schedule: bool = True):
        """Forward compositing; ``median`` also renders the median depth
        (self.median_depth) and its entry index (self.median_contrib);
        ``stats`` (hits alone, or hits with both maxima) accumulates the
        occlusion statistics in the same pass.  ``schedule`` as in
        train_step_raster: tiles launched heaviest first by the last recorded
        costs; backward_raster reuses the order."""
        h, ma, mw = _stats(stats)
        order, cost = self._schedule(stream) if schedule else (None, None)
        cfg = self._cfg(accumulate)
        md = mc = None
        if median:
            if getattr(self, "median_depth", None) is None:
                P = max(self.views.P, 1)
                self.median_depth = torch.zeros(P, dtype=torch.float32, device=self.device)
                self.median_contrib = torch.zeros(P, dtype=torch.int32, device=self.device)
            md, mc = self.median_depth, self.median_contrib
        call("sr_render_forward", self.ctx.ptr, ctypes.byref(cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.geom), _ptr(self.app), _ptr(self.vals), _ptr(self.ranges),
             _ptr(self.color), _ptr(self.alpha), _ptr(self.depth), _ptr(self.normal), _ptr(self.dist),
             _ptr(self.T_final), _ptr(self.n_contrib), _ptr(h), _ptr(ma), _ptr(mw), _ptr(md), _ptr(mc),
             _ptr(order), _ptr(cost), _stream(stream))
        self.last_order = order
        if cost is not None:
            self.costs_recorded = True

    def _grad_rec(self):
        if self.grad_rec is None:
            # zero on allocation; every projection backward leaves it zero
            self.grad_rec = torch.zeros(max(self.views.V * self.N * _lib.SR_GRAD_STRIDE, 1),
                                        dtype=torch.float32, device=self.device)
        return self.grad_rec

    def _median_contrib(self, dM):
        if dM is None:
            return None
        if getattr(self, "median_contrib", None) is None:
            raise ValueError("a median-depth gradient needs a forward with median=True")
        return self.median_contrib

    def backward_raster(self, dC=None, dA=None, dD=None, dN=None, dS=None, stream=None, dM=None,
                        schedule: bool = True):
        """Compositing backward; ``dM`` is the gradient of the median depth
        (after a forward with median=True); ``schedule``: launched in the
        order of the last forward (heaviest tiles first)."""
        order = getattr(self, "last_order", None) if schedule else None
        call("sr_backward_raster", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.geom), _ptr(self.app), _ptr(self.vals), _ptr(self.ranges),
             _ptr(self.alpha), _ptr(self.depth), _ptr(self.dist), _ptr(self.T_final), _ptr(self.n_contrib),
             _ptr(dC), _ptr(dA), _ptr(dD), _ptr(dN), _ptr(dS), _ptr(self._median_contrib(dM)), _ptr(dM),
             _ptr(self._grad_rec()), _ptr(self.tiles_touched), _ptr(order), _stream(stream))

    def backward_project(self, p: Params, grads: Params, stream=None, densify=None):
        """Projection backward; ``densify`` = (grad_sum float32 [N], count
        int32 [N]) accumulates the density-control statistic."""
        dg, dc = (None, None) if densify is None else densify
        # every compositing backward of this object marks the records it
        # gives gradients (bit 31 of tiles_touched): read only those
        cfg = SrConfig.from_buffer_copy(self.cfg)
        cfg.flags |= _lib.SR_FLAG_MARKED_GRADIENTS
        call("sr_backward_project", self.ctx.ptr, ctypes.byref(cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(p.means), _ptr(p.scales), _ptr(p.quats), _ptr(p.sh), _ptr(self.geom),
             _ptr(self.app), _ptr(self.tiles_touched), _ptr(self._grad_rec()), _ptr(grads.means),
             _ptr(grads.scales), _ptr(grads.quats), _ptr(grads.opac), _ptr(grads.sh), _ptr(dg), _ptr(dc),
             _stream(stream))

    def backward(self, p: Params, grads: Params, dC=None, dA=None, dD=None, dN=None, dS=None, stream=None,
                 dM=None):
        """Both halves of the backward; the parameter gradients are added to."""
        self.backward_raster(dC, dA, dD, dN, dS, stream, dM)
        self.backward_project(p, grads, stream)

    def backward_combined(self, p: Params, grads: Params, dC=None, dA=None, dD=None, dN=None, dS=None,
                          stream=None, dM=None):
        """The single-call form (sr_render_backward)."""
        call("sr_render_backward", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(p.means), _ptr(p.scales), _ptr(p.quats), _ptr(p.opac), _ptr(p.sh),
             _ptr(self.geom), _ptr(self.app), _ptr(self.vals), _ptr(self.ranges), _ptr(self.alpha),
             _ptr(self.depth), _ptr(self.dist), _ptr(self.T_final), _ptr(self.n_contrib), _ptr(dC), _ptr(dA),
             _ptr(dD), _ptr(dN), _ptr(dS), _ptr(self._median_contrib(dM)), _ptr(dM), _ptr(self._grad_rec()),
             _ptr(grads.means), _ptr(grads.scales),
             _ptr(grads.quats), _ptr(grads.opac), _ptr(grads.sh), _stream(stream))

    def loss(self, mask: torch.Tensor, target: Optional[torch.Tensor], gamma: float = 0.5, w_c: float = 1.0,
             dL_dalpha: Optional[torch.Tensor] = None, dL_dcolor: Optional[torch.Tensor] = None, stream=None):
        call("sr_background_loss", self.ctx.ptr, self.views.V, self.views.host_ptr, _ptr(self.views.dev), _ptr(self.alpha),
             _ptr(mask), _ptr(self.color) if target is not None else None, _ptr(target), float(gamma), float(w_c),
             _ptr(self.loss_ws), self.loss_ws.numel(), _ptr(self.loss_out), _ptr(dL_dalpha), _ptr(dL_dcolor),
             _stream(stream))
        return self.loss_out

    def regularizer_loss(self, w_dist: float, w_normal: float, dL_dalpha: torch.Tensor, dL_ddepth: torch.Tensor,
                         dL_dnormal: torch.Tensor, dL_ddist: torch.Tensor, stream=None,
                         dL_dmedian: Optional[torch.Tensor] = None):
        """The 2DGS terms of Eq. 3 on the current forward outputs (sr_regularizer_loss):
        returns loss [2V+1] (L_d per view, L_n per view, weighted total);
        dL_dalpha is added to, the other gradients are overwritten.  With
        ``dL_dmedian`` the normal term uses the median depth of the last
        forward (median=True) and its gradient is written there."""
        if getattr(self, "reg_out", None) is None:
            self.reg_out = torch.zeros(2 * self.views.V + 1, dtype=torch.float32, device=self.device)
        med = None if dL_dmedian is None else self.median_depth
        call("sr_regularizer_loss", self.ctx.ptr, self.views.V, self.views.host_ptr, _ptr(self.views.dev), _ptr(self.alpha),
             _ptr(self.depth), _ptr(self.normal), _ptr(self.dist), _ptr(med), float(w_dist), float(w_normal),
             _ptr(self.loss_ws), self.loss_ws.numel(), _ptr(self.reg_out), _ptr(dL_dalpha), _ptr(dL_ddepth),
             _ptr(dL_dnormal), _ptr(dL_ddist), _ptr(dL_dmedian), _stream(stream))
        return self.reg_out

    def ssim_loss(self, mask: torch.Tensor, target: torch.Tensor, w_s: float = 0.2,
                  dL_dcolor: Optional[torch.Tensor] = None, stream=None):
        """Masked D-SSIM / SSIM / PSNR of the current colour outputs
        (sr_ssim_loss): returns [SSIM per view, PSNR per view, weighted
        D-SSIM]; the gradient is added to dL_dcolor when given."""
        with_grad = dL_dcolor is not None
        need = _lib.workspace_bytes_ssim(self.views.V, self.views.host, with_grad)
        if getattr(self, "ssim_ws", None) is None or self.ssim_ws.numel() < need:
            self.ssim_ws = torch.zeros(max(need, 1), dtype=torch.uint8, device=self.device)
        if getattr(self, "ssim_out", None) is None:
            self.ssim_out = torch.zeros(2 * self.views.V + 1, dtype=torch.float32, device=self.device)
        call("sr_ssim_loss", self.ctx.ptr, self.views.V, self.views.host_ptr, _ptr(self.views.dev), _ptr(self.color),
             _ptr(target), _ptr(mask), float(w_s), _ptr(self.ssim_ws), self.ssim_ws.numel(), _ptr(self.ssim_out),
             _ptr(dL_dcolor), _stream(stream))
        return self.ssim_out

    def train_step_raster(self, mask: torch.Tensor, target: torch.Tensor, gamma: float = 0.5, w_c: float = 1.0,
                          stats=None, accumulate: bool = False, stream=None, schedule: bool = True,
                          noalloc: bool = False):
        """Fused forward + loss gradients + backward compositing (one launch;
        ``stats`` as in forward); follow with backward_project.  With
        ``schedule`` every call records the per-tile costs and launches in the
        order of the previous call's costs, heaviest tiles first (the first
        call uses the default order; results do not depend on the order).
        ``noalloc``: sr_train_step_raster_noalloc, the per-tile loss partials
        in the library's scratch array instead of a buffer of this object."""
        h, ma, mw = _stats(stats)
        cfg = self._cfg(accumulate)
        order, cost = self._schedule(stream) if schedule else (None, None)
        common = (self.ctx.ptr, ctypes.byref(cfg), self.N, self.views.V, self.views.host_ptr, _ptr(self.views.dev),
                  _ptr(self.geom), _ptr(self.app), _ptr(self.vals), _ptr(self.ranges), _ptr(mask), _ptr(target),
                  float(gamma), float(w_c), _ptr(self.color), _ptr(self.alpha), _ptr(self.depth), _ptr(self.normal),
                  _ptr(self.dist), _ptr(self.T_final), _ptr(self.n_contrib), _ptr(h), _ptr(ma), _ptr(mw))
        tail = (_ptr(self.loss_out), _ptr(self._grad_rec()), _ptr(self.tiles_touched), _ptr(order), _ptr(cost),
                _stream(stream))
        if noalloc:
            call("sr_train_step_raster_noalloc", *common, *tail)
        else:
            if getattr(self, "tile_loss", None) is None:
                self.tile_loss = torch.zeros(2 * max(self.views.T, 1), dtype=torch.float32, device=self.device)
            call("sr_train_step_raster", *common, _ptr(self.tile_loss), *tail)
        if cost is not None:
            self.costs_recorded = True
        return self.loss_out

    def prune_stats(self, hits, max_alpha, max_weight, accumulate=False, stream=None, cull: bool = True):
        """Occlusion statistics of the current binning (sr_prune_stats);
        ``cull`` lets each wave skip entries by their pixel rectangles."""
        cfg = self._cfg(accumulate)
        call("sr_prune_stats", self.ctx.ptr, ctypes.byref(cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.geom), _ptr(self.rect) if cull else None, _ptr(self.vals),
             _ptr(self.ranges), _ptr(hits), _ptr(max_alpha), _ptr(max_weight), _stream(stream))

    def count_pairs(self, stream=None, waves=False):
        """(reached pairs, blended pairs) of the current binning, and with
        ``waves`` also (wave steps, wave steps with a blend, pairs up to
        each pixel's last blend) - syncs."""
        out = torch.zeros(5, dtype=torch.int64, device=self.device)
        call("sr_render_count", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.geom), _ptr(self.app), _ptr(self.vals), _ptr(self.ranges), _ptr(out),
             _stream(stream))
        c = out.cpu().numpy()
        if waves:
            return int(c[0]), int(c[1]), int(c[2]), int(c[3]), int(c[4])
        return int(c[0]), int(c[1])

    def status(self):
        """(visible pairs, instances needed, instances stored, status) - syncs."""
        c = self.counters.cpu().numpy().view(np.uint32)
        return int(c[0]), int(c[1]), int(c[2]), int(c[3])

    def check_capacity(self, stream=None):
        """Reads and clears the context's status word (syncs); raises when a
        binning since the last check exceeded the capacity (the compositing
        calls after it flagged their outputs).  Returns the instance count
        of the last binning."""
        bits, need_max = self.ctx.read_status(_stream(stream), clear=True)
        vis, need, stored, st = self.status()
        if bits & _lib.SR_STATUS_CAPACITY:
            raise _lib.SurfelRasterError(_lib.SR_ERR_CAPACITY,
                                         f"instance capacity {self.capacity} exceeded: {need_max} needed")
        return need


@dataclass
class PruneStats:
    hits: torch.Tensor          # int32 [N] blended (pixel, surfel) pairs
    max_alpha: torch.Tensor     # float32 [N] largest blended alpha
    max_weight: torch.Tensor    # float32 [N] largest blending weight a T
    in_frustum: torch.Tensor    # uint8 [N] not culled in some view
    mask: torch.Tensor          # uint8 [N] 1 = prune (max_alpha < tau)


def _new_prune_stats(n: int, dev) -> PruneStats:
    return PruneStats(torch.zeros(n, dtype=torch.int32, device=dev), torch.zeros(n, device=dev),
                      torch.zeros(n, device=dev), torch.zeros(n, dtype=torch.uint8, device=dev),
                      torch.zeros(n, dtype=torch.uint8, device=dev))


def _prune_pass(prim: int, means, scales, quats, opac, cams: Sequence, views_per_chunk: int, tau: float, tile,
                slack: float, stats: Optional[PruneStats], check: bool, stream=None) -> PruneStats:
    """sr_prune_plan (capacity, one host sync) then sr_prune_contrib (the
    whole pass on the device) over every view, in chunks of views."""
    n = int(means.shape[0])
    dev = means.device
    accumulate = stats is not None
    if stats is None:
        stats = _new_prune_stats(n, dev)
    views = ViewBatch(cams, tile=tile, device=dev)
    ctx = _lib.Context(_device_index(dev))
    cfg = make_config(0, None, views.tile, flags=_lib.SR_FLAG_ACCUMULATE if accumulate else 0)
    V = views.V
    vpc = max(1, min(int(views_per_chunk), max(V, 1)))
    args = (n, _ptr(means), _ptr(scales), _ptr(quats), _ptr(opac), V, views.host_ptr, _ptr(views.dev), vpc)

    def ws_bytes(cap):
        b = ctypes.c_size_t(0)
        call("sr_prune_workspace_size", ctypes.byref(cfg), prim, n, V, views.host_ptr if V else None, vpc, cap,
             ctypes.byref(b))
        return b.value

    b0 = ws_bytes(0)
    ws = torch.zeros(max(b0, 1), dtype=torch.uint8, device=dev)
    cap = ctypes.c_uint32(0)
    call("sr_prune_plan", ctx.ptr, ctypes.byref(cfg), prim, *args, _ptr(ws), b0, ctypes.byref(cap), _stream(stream))
    capacity = int(cap.value * slack) + 1024
    b1 = ws_bytes(capacity)
    del ws
    ws = torch.empty(max(b1, 1), dtype=torch.uint8, device=dev)
    call("sr_prune_contrib", ctx.ptr, ctypes.byref(cfg), prim, *args, float(tau), capacity, _ptr(ws), b1,
         _ptr(stats.hits), _ptr(stats.max_alpha), _ptr(stats.max_weight), _ptr(stats.in_frustum), _ptr(stats.mask),
         _stream(stream))
    if check:
        bits, need = ctx.read_status(_stream(stream), clear=True)
        if bits & _lib.SR_STATUS_CAPACITY:
            raise _lib.SurfelRasterError(_lib.SR_ERR_CAPACITY, f"pruning pass: {need} instances needed, "
                                                               f"capacity {capacity}")
    return stats


def prune_contrib(params: Params, cams: Sequence, views_per_chunk: int = 32, tau: float = ALPHA_MIN,
                  tile=(16, 16), slack: float = 1.02, stats: Optional[PruneStats] = None,
                  check: bool = True) -> PruneStats:
    """Occlusion-aware pruning pass (Section 4.3) over every view
    (sr_prune_contrib): projection without shading, binning and the
    compositing decisions, accumulating the statistics over views (and over
    calls when ``stats`` is given), then the mask.  Views are processed in
    chunks to bound the per-view records; the capacity is planned by
    sr_prune_plan.  ``check`` reads the status word at the end (syncs)."""
    return _prune_pass(_lib.SR_PRIM_SURFEL, params.means, params.scales, params.quats, params.opac, cams,
                       views_per_chunk, tau, tile, slack, stats, check)


def prune_mask(max_alpha: torch.Tensor, tau: float = ALPHA_MIN, stream=None) -> torch.Tensor:
    out = torch.empty(max_alpha.numel(), dtype=torch.uint8, device=max_alpha.device)
    call("sr_prune_mask", _ctx(max_alpha), max_alpha.numel(), _ptr(max_alpha), float(tau), _ptr(out),
         _stream(stream))
    return out


# ----------------------------------------------------------------------------
# autograd
# ----------------------------------------------------------------------------

class SurfelRasterize(torch.autograd.Function):
    """(means, scales, quats, opac, sh) -> packed (color [3P], alpha [P],
    depth [P], normal [3P], dist [P]) for the views of ``rast``, and with
    ``median`` also the median depth [P].  The rasterizer's buffers hold the
    saved state: call backward before the next forward through the same
    Rasterizer."""

    @staticmethod
    def forward(ctx, means, scales, quats, opac, sh, rast: Rasterizer, check: bool = False, median: bool = False):
        p = Params(means.detach().contiguous(), scales.detach().contiguous(), quats.detach().contiguous(),
                   opac.detach().contiguous(), sh.detach().contiguous())
        rast.preprocess(p)
        rast.bin()
        if check:
            rast.check_capacity()
        rast.forward(median=median)
        ctx.rast = rast
        ctx.p = p
        ctx.median = median
        out = (rast.color.clone(), rast.alpha.clone(), rast.depth.clone(), rast.normal.clone(), rast.dist.clone())
        if median:
            out = out + (rast.median_depth[: rast.views.P].clone(),)
        return out

    @staticmethod
    def backward(ctx, gC, gA, gD, gN, gS, gM=None):
        p, rast = ctx.p, ctx.rast
        g = Params(torch.zeros_like(p.means), torch.zeros_like(p.scales), torch.zeros_like(p.quats),
                   torch.zeros_like(p.opac), torch.zeros_like(p.sh))
        c = lambda t: None if t is None else t.contiguous()
        rast.backward(p, g, c(gC), c(gA), c(gD), c(gN), c(gS), dM=c(gM) if ctx.median else None)
        return g.means, g.scales, g.quats, g.opac, g.sh, None, None, None


def rasterize(means, scales, quats, opac, sh, rast: Rasterizer, check: bool = False, median: bool = False):
    """Differentiable rasterization; ``median`` adds the median depth as a
    sixth output.  ``check`` reads the capacity status after the binning
    (a host sync, so not inside a captured graph); without it a binning
    over capacity shows as NaN outputs and in ``rast.check_capacity()``."""
    return SurfelRasterize.apply(means, scales, quats, opac, sh, rast, check, median)


class BackgroundLoss(torch.autograd.Function):
    """Masked losses (Eq. 1 and the L1 part of Eq. 2) of all views:
    returns (1/V) sum_v (w_c L1_v + gamma L_b,v) and the per-view terms
    (non-differentiable: a loss built from them raises in backward)."""

    @staticmethod
    def forward(ctx, alpha, color, target, mask, views: ViewBatch, gamma: float, w_c: float, ws):
        V = views.V
        loss = torch.zeros(2 * V + 1, dtype=torch.float32, device=alpha.device)
        dA = torch.empty_like(alpha)
        dC = torch.empty_like(color) if target is not None else None
        call("sr_background_loss", _ctx(alpha), V, views.host_ptr, _ptr(views.dev), _ptr(alpha.contiguous()),
             _ptr(mask),
             _ptr(color.contiguous()) if target is not None else None, _ptr(target), float(gamma), float(w_c),
             _ptr(ws), ws.numel(), _ptr(loss), _ptr(dA), _ptr(dC), _stream())
        ctx.save_for_backward(dA, dC if dC is not None else torch.zeros(0, device=alpha.device))
        ctx.has_c = dC is not None
        per_view = loss[: 2 * V]
        # the per-view terms are reported, not differentiated: only the total carries a gradient
        ctx.mark_non_differentiable(per_view)
        return loss[2 * V], per_view

    @staticmethod
    def backward(ctx, g_total, g_loss):
        dA, dC = ctx.saved_tensors
        return (dA * g_total, (dC * g_total) if ctx.has_c else None, None, None, None, None, None, None)


class RegularizerLoss(torch.autograd.Function):
    """The 2DGS terms of Eq. 3 (sr_regularizer_loss) of all views: returns
    (1/V) sum_v (w_dist L_d,v + w_normal L_n,v) and the per-view terms
    [L_d,0..V-1, L_n,0..V-1].  With ``median`` (the median depth [P]) the
    normal term takes its surface depth from that map instead of D / A."""

    @staticmethod
    def forward(ctx, alpha, depth, normal, dist, views: ViewBatch, w_dist: float, w_normal: float, ws,
                median=None):
        V = views.V
        loss = torch.zeros(2 * V + 1, dtype=torch.float32, device=alpha.device)
        dA = torch.zeros_like(alpha)
        dD, dN, dS = torch.empty_like(depth), torch.empty_like(normal), torch.empty_like(dist)
        med = None if median is None else median.contiguous()
        dM = None if median is None else torch.empty_like(med)
        call("sr_regularizer_loss", _ctx(alpha), V, views.host_ptr, _ptr(views.dev), _ptr(alpha.contiguous()),
             _ptr(depth.contiguous()), _ptr(normal.contiguous()), _ptr(dist.contiguous()), _ptr(med),
             float(w_dist), float(w_normal), _ptr(ws), ws.numel(), _ptr(loss), _ptr(dA), _ptr(dD), _ptr(dN),
             _ptr(dS), _ptr(dM), _stream())
        ctx.save_for_backward(dA, dD, dN, dS, dM if dM is not None else torch.zeros(0, device=alpha.device))
        ctx.has_m = dM is not None
        per_view = loss[: 2 * V]
        ctx.mark_non_differentiable(per_view)
        return loss[2 * V], per_view

    @staticmethod
    def backward(ctx, g_total, g_loss):
        dA, dD, dN, dS, dM = ctx.saved_tensors
        return (dA * g_total, dD * g_total, dN * g_total, dS * g_total, None, None, None, None,
                (dM * g_total) if ctx.has_m else None)


class SsimLoss(torch.autograd.Function):
    """Masked D-SSIM of all views (sr_ssim_loss): returns
    (1/V) sum_v w_s (1 - SSIM_v) and [SSIM_0..V-1, PSNR_0..V-1]."""

    @staticmethod
    def forward(ctx, color, target, mask, views: ViewBatch, w_s: float, ws):
        V = views.V
        out = torch.zeros(2 * V + 1, dtype=torch.float32, device=color.device)
        dC = torch.zeros_like(color)
        call("sr_ssim_loss", _ctx(color), V, views.host_ptr, _ptr(views.dev), _ptr(color.contiguous()),
             _ptr(target),
             _ptr(mask), float(w_s), _ptr(ws), ws.numel(), _ptr(out), _ptr(dC), _stream())
        ctx.save_for_backward(dC)
        per_view = out[: 2 * V]
        ctx.mark_non_differentiable(per_view)
        return out[2 * V], per_view

    @staticmethod
    def backward(ctx, g_total, g_out):
        (dC,) = ctx.saved_tensors
        return dC * g_total, None, None, None, None, None


def compact_surfels(prune: torch.Tensor, arrays: Sequence[torch.Tensor], opac: Optional[torch.Tensor] = None,
                    min_opacity: float = 0.0, stream=None):
    """Drop the pruned surfels (prune uint8 [N], 1 = drop; and, with opac,
    those below min_opacity) from every per-surfel array (float32, first
    dimension N), keeping the order (sr_compact_surfels).  Returns the
    compacted arrays (new tensors) - syncs to read the kept count."""
    N = int(prune.shape[0])
    if len(arrays) > _lib.SR_COMPACT_MAX_ARRAYS:
        raise ValueError(f"at most {_lib.SR_COMPACT_MAX_ARRAYS} arrays per call")
    dev = prune.device
    srcs = [a.contiguous().reshape(N, int(np.prod(a.shape[1:])) if a.dim() > 1 else 1) for a in arrays]
    dsts = [torch.empty_like(a) for a in srcs]
    widths = (ctypes.c_int32 * max(len(srcs), 1))(*[int(a.shape[1]) for a in srcs])
    sp = (ctypes.c_void_p * max(len(srcs), 1))(*[a.data_ptr() for a in srcs])
    dp = (ctypes.c_void_p * max(len(srcs), 1))(*[a.data_ptr() for a in dsts])
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().sr_compact_workspace_size(N, ctypes.byref(n)))
    ws = torch.zeros(max(n.value, 4), dtype=torch.uint8, device=dev)
    kept = torch.zeros(1, dtype=torch.int32, device=dev)
    pr = prune.contiguous()                      # held across the call
    op = None if opac is None else opac.contiguous()
    call("sr_compact_surfels", _ctx(prune), N, _ptr(pr), _ptr(op), float(min_opacity), len(srcs),
         ctypes.cast(sp, ctypes.c_void_p), ctypes.cast(dp, ctypes.c_void_p), ctypes.cast(widths, ctypes.c_void_p),
         _ptr(ws), ws.numel(), _ptr(kept), _stream(stream))
    k = int(kept.item())
    return [d[:k].reshape((k,) + tuple(a.shape[1:])) for d, a in zip(dsts, arrays)]


class Pruner3D:
    """The occlusion-pruning pass for 3D Gaussians (Appendix B):
    sr_preprocess_3d -> sr_bin_and_sort -> sr_prune_contrib_3d over a batch
    of views.  Parameters: means [N,3], scales [N,3], quats [N,4], opac [N]."""

    def __init__(self, N: int, views: ViewBatch, capacity: int = 0, device="cuda"):
        self.N, self.views, self.device = int(N), views, device
        self.ctx = _lib.Context(_device_index(device))
        self.cfg = make_config(0, None, views.tile)
        VN = views.V * self.N
        z = lambda n, dt: torch.zeros(max(int(n), 1), dtype=dt, device=device)
        self.geom3 = z(VN * 8, torch.float32)
        self.rect = z(VN * 4, torch.int16)
        self.tiles_touched = z(VN, torch.int32)
        self.depth_key = z(VN, torch.int32)
        self.in_frustum = z(self.N, torch.uint8)
        self.ranges = z(2 * views.T, torch.int32)
        self.counters = z(_lib.SR_COUNTERS, torch.int32)
        self.capacity = -1
        self.set_capacity(capacity)

    def set_capacity(self, cap: int):
        cap = int(cap)
        if cap == self.capacity:
            return
        self.capacity = cap
        self.vals = torch.zeros(max(cap, 1), dtype=torch.int32, device=self.device)
        self.ws_bytes = _lib.workspace_bytes_bin(self.N, self.views.V, cap)
        self.ws = torch.zeros(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.device)

    def preprocess(self, means, scales, quats, opac, stream=None):
        call("sr_preprocess_3d", self.ctx.ptr, ctypes.byref(self.cfg), self.N, _ptr(means), _ptr(scales), _ptr(quats),
             _ptr(opac), self.views.V, self.views.host_ptr, _ptr(self.views.dev), _ptr(self.geom3),
             _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_key), _ptr(self.in_frustum),
             _stream(stream))

    def plan_capacity(self, means, scales, quats, opac, slack: float = 1.05) -> int:
        """Projects and counts the instances (count-only binning, one host
        sync), then sizes the instance buffers."""
        self.preprocess(means, scales, quats, opac)
        call("sr_bin_and_sort", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_key),
             _ptr(self.ws), self.ws_bytes, 0, None, None, _ptr(self.ranges), _ptr(self.counters), _stream())
        need = int(self.counters[1:2].cpu().numpy().view(np.uint32)[0])
        self.set_capacity(int(need * slack) + 1024)
        return need

    def bin(self, keys64: Optional[torch.Tensor] = None, stream=None):
        call("sr_bin_and_sort", self.ctx.ptr, ctypes.byref(self.cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.rect), _ptr(self.tiles_touched), _ptr(self.depth_key),
             _ptr(self.ws), self.ws_bytes, self.capacity, _ptr(self.vals), _ptr(keys64), _ptr(self.ranges),
             _ptr(self.counters), _stream(stream))

    def prune_stats(self, hits, max_alpha, max_weight, accumulate: bool = False, stream=None):
        cfg = self.cfg
        if accumulate:
            cfg = SrConfig.from_buffer_copy(self.cfg)
            cfg.flags |= _lib.SR_FLAG_ACCUMULATE
        call("sr_prune_stats_3d", self.ctx.ptr, ctypes.byref(cfg), self.N, self.views.V, self.views.host_ptr,
             _ptr(self.views.dev), _ptr(self.geom3), _ptr(self.vals), _ptr(self.ranges), _ptr(hits),
             _ptr(max_alpha), _ptr(max_weight), _stream(stream))

    def run(self, means, scales, quats, opac, hits, max_alpha, max_weight, accumulate: bool = False,
            stream=None):
        self.preprocess(means, scales, quats, opac, stream)
        self.bin(stream=stream)
        self.prune_stats(hits, max_alpha, max_weight, accumulate, stream)

    def status(self):
        c = self.counters.cpu().numpy().view(np.uint32)
        return int(c[0]), int(c[1]), int(c[2]), int(c[3])


def prune_contrib_3d(means, scales, quats, opac, cams: Sequence, views_per_chunk: int = 32, tau: float = ALPHA_MIN,
                     tile=(16, 16), slack: float = 1.02, stats: Optional[PruneStats] = None,
                     check: bool = True) -> PruneStats:
    """The occlusion-pruning pass for 3D Gaussians over every view
    (sr_prune_contrib with SR_PRIM_GAUSS3D; chunks of views bound the
    per-view records), statistics accumulated, then the mask."""
    return _prune_pass(_lib.SR_PRIM_GAUSS3D, means, scales, quats, opac, cams, views_per_chunk, tau, tile, slack,
                       stats, check)
