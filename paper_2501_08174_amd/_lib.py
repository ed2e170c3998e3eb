"""ctypes binding of libsurfelrast.so (the C ABI in include/surfelrast.h).

Argument marshalling only: every step runs in the HIP library.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import sys
from ctypes import POINTER, byref, c_float, c_int32, c_int64, c_size_t, c_uint32, c_void_p, c_char_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsurfelrast.so")

SR_OK = 0
SR_ERR_ARG = -1
SR_ERR_CAPACITY = -2
SR_ERR_HIP = -3
SR_ERR_UNSUPPORTED = -4
SR_ERR_STATE = -5
SR_STATUS_CAPACITY = 1
SR_PRIM_SURFEL = 0
SR_PRIM_GAUSS3D = 1
ABI_VERSION = 4           # sr_version() of the library these signatures describe
SR_FLAG_ACCUMULATE = 1
SR_FLAG_MARKED_GRADIENTS = 2
SR_GEOM_STRIDE = 16
SR_APP_STRIDE = 8
SR_GRAD_STRIDE = 24
SR_COUNTERS = 4
SR_COMPACT_MAX_ARRAYS = 8
SR_TILE_GROUP = 4
SR_INST_ID_BITS = 24
SR_NOALLOC_MAX_TILES = 262144

EXPORTED = (
    "sr_last_error", "sr_version", "sr_create", "sr_destroy", "sr_read_status", "sr_clear_status",
    "sr_tile_supported", "sr_bwd_batch_supported", "sr_layout_views", "sr_preprocess", "sr_bin_workspace_size", "sr_workspace_size",
    "sr_bin_and_sort", "sr_render_forward", "sr_render_backward", "sr_backward_raster", "sr_backward_project",
    "sr_loss_workspace_size", "sr_background_loss", "sr_regularizer_loss", "sr_ssim_workspace_size",
    "sr_ssim_loss", "sr_compact_workspace_size", "sr_compact_surfels", "sr_preprocess_3d", "sr_prune_stats_3d",
    "sr_train_step_raster", "sr_train_step_raster_noalloc", "sr_prune_stats", "sr_prune_workspace_size",
    "sr_prune_plan", "sr_prune_contrib", "sr_render_count", "sr_prune_mask", "sr_tile_order_workspace_size", "sr_tile_order",
)


class SurfelRasterError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"surfelrast error {code}: {msg}")
        self.code = code


class SrCamera(ctypes.Structure):
    _fields_ = [
        ("viewmat", c_float * 12), ("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
        ("campos", c_float * 3), ("znear", c_float), ("bg", c_float * 3),
        ("width", c_int32), ("height", c_int32), ("tiles_x", c_int32), ("tiles_y", c_int32),
        ("tile_offset", c_int32), ("pix_offset", c_int64), ("group_offset", c_int32), ("groups_x", c_int32),
    ]


class SrConfig(ctypes.Structure):
    _fields_ = [
        ("tile_w", c_int32), ("tile_h", c_int32), ("sh_degree", c_int32), ("sh_stride", c_int32),
        ("alpha_min", c_float), ("alpha_max", c_float), ("t_min", c_float), ("flags", c_uint32),
        ("bwd_batch", c_int32),
    ]


assert ctypes.sizeof(SrCamera) == 128
assert ctypes.sizeof(SrConfig) == 36

_lib = None
P = c_void_p   # device or host pointer passed as an integer address


def _declare(lib):
    V = c_void_p
    sig = {
        "sr_last_error": (c_char_p, []),
        "sr_version": (c_int32, []),
        "sr_create": (c_int32, [V, c_int32]),
        "sr_destroy": (c_int32, [V]),
        "sr_read_status": (c_int32, [V, V, c_int32, V, V]),
        "sr_clear_status": (c_int32, [V, V]),
        "sr_tile_supported": (c_int32, [c_int32, c_int32]),
        "sr_bwd_batch_supported": (c_int32, [c_int32, c_int32, c_int32]),
        "sr_layout_views": (c_int32, [V, c_int32, c_int32, c_int32, POINTER(c_int64), POINTER(c_int32)]),
        "sr_preprocess": (c_int32, [V, V, c_int32, V, V, V, V, V, c_int32, V, V, V, V, V, V, V, V, V]),
        "sr_bin_workspace_size": (c_int32, [c_int32, c_int32, c_uint32, POINTER(c_size_t)]),
        "sr_workspace_size": (c_int32, [V, c_int32, c_int32, V, c_uint32, POINTER(c_size_t)]),
        "sr_bin_and_sort": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, c_size_t, c_uint32, V, V, V, V,
                                      V]),
        "sr_render_forward": (c_int32, [V, V, c_int32, c_int32] + [V] * 21),
        "sr_render_backward": (c_int32, [V, V, c_int32, c_int32, V, V] + [V] * 28),
        "sr_backward_raster": (c_int32, [V, V, c_int32, c_int32] + [V] * 22),
        "sr_backward_project": (c_int32, [V, V, c_int32, c_int32] + [V] * 18),
        "sr_loss_workspace_size": (c_int32, [c_int32, V, POINTER(c_size_t)]),
        "sr_background_loss": (c_int32, [V, c_int32, V, V, V, V, V, V, c_float, c_float, V, c_size_t, V, V, V,
                                         V]),
        "sr_regularizer_loss": (c_int32, [V, c_int32, V, V, V, V, V, V, V, c_float, c_float, V, c_size_t, V, V,
                                          V, V, V, V, V]),
        "sr_ssim_workspace_size": (c_int32, [c_int32, V, c_int32, POINTER(c_size_t)]),
        "sr_ssim_loss": (c_int32, [V, c_int32, V, V, V, V, V, c_float, V, c_size_t, V, V, V]),
        "sr_compact_workspace_size": (c_int32, [c_int32, POINTER(c_size_t)]),
        "sr_preprocess_3d": (c_int32, [V, V, c_int32, V, V, V, V, c_int32, V, V, V, V, V, V, V, V]),
        "sr_prune_stats_3d": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, V, V, V]),
        "sr_compact_surfels": (c_int32, [V, c_int32, V, V, c_float, c_int32, V, V, V, V, c_size_t, V, V]),
        "sr_train_step_raster": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, V, V, c_float, c_float]
                                 + [V] * 17),
        "sr_train_step_raster_noalloc": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, V, V, c_float,
                                                   c_float] + [V] * 16),
        "sr_tile_order_workspace_size": (c_int32, [c_int32, POINTER(c_size_t)]),
        "sr_tile_order": (c_int32, [V, c_int32, V, V, c_size_t, V, V]),
        "sr_prune_stats": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, V, V, V, V]),
        "sr_prune_workspace_size": (c_int32, [V, c_int32, c_int32, c_int32, V, c_int32, c_uint32,
                                              POINTER(c_size_t)]),
        "sr_prune_plan": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, c_int32, V, V, c_int32, V, c_size_t,
                                    POINTER(c_uint32), V]),
        "sr_prune_contrib": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, c_int32, V, V, c_int32, c_float,
                                       c_uint32, V, c_size_t, V, V, V, V, V, V]),
        "sr_render_count": (c_int32, [V, V, c_int32, c_int32, V, V, V, V, V, V, V, V]),
        "sr_prune_mask": (c_int32, [V, c_int32, V, c_float, V, V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               f"'python -m paper_2501_08174_amd.build' (no CPU fallback exists)")
        l = ctypes.CDLL(LIB_PATH)
        _declare(l)
        if l.sr_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {l.sr_version()}, this binding is written for "
                               f"{ABI_VERSION}: rebuild it with 'python -m paper_2501_08174_amd.build'")
        _lib = l
    return _lib


def check(status: int):
    if status != SR_OK:
        raise SurfelRasterError(status, lib().sr_last_error().decode())


def call(name: str, *args):
    check(getattr(lib(), name)(*args))


def workspace_bytes_bin(N: int, V: int, cap: int) -> int:
    out = c_size_t(0)
    check(lib().sr_bin_workspace_size(N, V, cap, byref(out)))
    return out.value


def workspace_bytes_ssim(V: int, cams_host, with_grad: bool = True) -> int:
    out = c_size_t(0)
    check(lib().sr_ssim_workspace_size(V, ctypes.cast(cams_host, c_void_p) if V else None, int(with_grad),
                                       byref(out)))
    return out.value


def workspace_bytes_loss(V: int, cams_host) -> int:
    out = c_size_t(0)
    check(lib().sr_loss_workspace_size(V, ctypes.cast(cams_host, c_void_p) if V else None, byref(out)))
    return out.value


class Context:
    """An sr_ctx: the HIP device its calls run on and that device's status
    word (instance-capacity failures of the binning, read with
    ``read_status``)."""

    def __init__(self, device: int):
        h = c_void_p()
        check(lib().sr_create(byref(h), int(device)))
        self.handle = h
        self.device = int(device)

    @property
    def ptr(self):
        return self.handle

    def read_status(self, stream=None, clear: bool = True):
        """(status bits, largest instance count a failed binning needed);
        synchronises the stream."""
        bits, need = c_uint32(0), ctypes.c_uint64(0)
        st = lib().sr_read_status(self.handle, stream, int(clear), byref(bits), byref(need))
        if st not in (SR_OK, SR_ERR_CAPACITY):
            check(st)
        return int(bits.value), int(need.value)

    def clear_status(self, stream=None):
        check(lib().sr_clear_status(self.handle, stream))

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the
        # process end releases the context instead
        try:
            h = getattr(self, "handle", None)
            if h is not None and h.value and not sys.is_finalizing() and _lib is not None:
                _lib.sr_destroy(h)
                self.handle = None
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int) -> Context:
    """One context per device for the calls that do not belong to a
    rasterizer (losses, masks, compaction)."""
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]
