"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only entry points validate arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "surfelrast.h")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2501_08174_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsurfelrast.so is not built (run python -m paper_2501_08174_amd.build)")
    return _lib


def test_header_symbols_exported(lib):
    names = _header_functions()
    assert len(names) >= 13
    l = lib.lib()
    for n in names:
        assert hasattr(l, n), n
    assert set(names) == set(lib.EXPORTED)


def test_layout_views_and_validation(lib):
    from paper_2501_08174_amd._lib import SrCamera
    cams = (SrCamera * 3)()
    for c, (w, h) in zip(cams, [(40, 21), (33, 48), (1, 1)]):
        c.width, c.height, c.fx, c.fy = w, h, 10.0, 10.0
    P = ctypes.c_int64()
    T = ctypes.c_int32()
    lib.call("sr_layout_views", ctypes.cast(cams, ctypes.c_void_p), 3, 16, 16, ctypes.byref(P), ctypes.byref(T))
    assert P.value == 40 * 21 + 33 * 48 + 1
    assert T.value == 3 * 2 + 3 * 3 + 1
    assert [c.tile_offset for c in cams] == [0, 6, 15]
    assert [c.pix_offset for c in cams] == [0, 840, 840 + 1584]
    # 4x4-tile binning groups: ceil(tiles / 4) per side, numbered view after view
    assert [c.groups_x for c in cams] == [1, 1, 1] and [c.group_offset for c in cams] == [0, 1, 2]
    big = (SrCamera * 2)()
    for c, (w, h) in zip(big, [(200, 130), (64, 65)]):
        c.width, c.height, c.fx, c.fy = w, h, 10.0, 10.0
    lib.call("sr_layout_views", ctypes.cast(big, ctypes.c_void_p), 2, 16, 16, None, None)
    assert (big[0].tiles_x, big[0].tiles_y, big[0].groups_x) == (13, 9, 4)
    assert (big[1].group_offset, big[1].groups_x) == (4 * 3, 1)
    bad = (SrCamera * 1)()
    bad[0].width, bad[0].height = 0, 5
    with pytest.raises(lib.SurfelRasterError) as e:
        lib.call("sr_layout_views", ctypes.cast(bad, ctypes.c_void_p), 1, 16, 16, None, None)
    assert e.value.code == lib.SR_ERR_ARG
    assert "size" in str(e.value)


def test_argument_errors_before_launch(lib):
    """Invalid configurations are rejected on the host (no device touched)."""
    from paper_2501_08174_amd._lib import SrConfig
    l = lib.lib()
    cfg = SrConfig(12, 12, 0, 1, 1 / 255, 0.99, 1e-4, 0)
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_UNSUPPORTED
    assert l.sr_tile_supported(16, 16) == 1 and l.sr_tile_supported(8, 8) == 1 and l.sr_tile_supported(7, 3) == 0
    # backward LDS batches: 32..256, at most the tile's pixels (0: the default)
    for b in (0, 32, 64, 128, 256):
        assert l.sr_bwd_batch_supported(16, 16, b) == 1 and l.sr_bwd_batch_supported(32, 8, b) == 1
    assert l.sr_bwd_batch_supported(16, 8, 128) == 1 and l.sr_bwd_batch_supported(16, 8, 256) == 0
    assert l.sr_bwd_batch_supported(8, 8, 0) == 1 and l.sr_bwd_batch_supported(8, 8, 64) == 1
    assert l.sr_bwd_batch_supported(8, 8, 128) == 0 and l.sr_bwd_batch_supported(16, 16, 48) == 0
    assert l.sr_bwd_batch_supported(7, 3, 0) == 0
    cfg = SrConfig(8, 8, 0, 1, 1 / 255, 0.99, 1e-4, 0, 128)
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_UNSUPPORTED
    assert b"batch" in l.sr_last_error()
    cfg = SrConfig(16, 16, 4, 25, 1 / 255, 0.99, 1e-4, 0)
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_UNSUPPORTED
    cfg = SrConfig(16, 16, 3, 9, 1 / 255, 0.99, 1e-4, 0)
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_ARG
    cfg = SrConfig(16, 16, 0, 1, 0.5, 0.4, 1e-4, 0)
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_ARG
    cfg = SrConfig(16, 16, 0, 1, 1 / 255, 0.99, 1e-4, 0)
    assert l.sr_preprocess(None, ctypes.byref(cfg), -1, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_ERR_ARG
    # N = 0 and V = 0 are valid no-ops
    assert l.sr_preprocess(None, ctypes.byref(cfg), 0, None, None, None, None, None, 0, None, None, None, None, None,
                           None, None, None, None) == lib.SR_OK
    n = ctypes.c_size_t()
    assert l.sr_bin_workspace_size(1000, 4, 12345, ctypes.byref(n)) == lib.SR_OK and n.value > 0
    assert l.sr_bin_workspace_size(-5, 4, 12345, ctypes.byref(n)) == lib.SR_ERR_ARG
    # workspace too small is an argument error
    counters = ctypes.c_void_p(8)
    assert l.sr_bin_and_sort(None, ctypes.byref(cfg), 10, 0, None, None, None, None, None, None, 0, 100, None, None,
                             None, counters, None) == lib.SR_ERR_ARG
    # binned surfel ids hold 24 bits: larger N is rejected before anything runs
    assert l.sr_bin_and_sort(None, ctypes.byref(cfg), 1 << 24, 0, None, None, None, None, None, None, 0, 100, None, None,
                             None, counters, None) == lib.SR_ERR_UNSUPPORTED
    assert lib.SR_TILE_GROUP == 4 and lib.SR_INST_ID_BITS == 24
    # the median depth and its entry index go together, and its gradient needs the index
    md = ctypes.c_void_p(256)
    assert l.sr_render_forward(None, ctypes.byref(cfg), 0, 0, None, None, *([None] * 14), md, None, None, None,
                               None) == lib.SR_ERR_ARG
    assert l.sr_render_forward(None, ctypes.byref(cfg), 0, 0, None, None, *([None] * 14), md, md, None, None,
                               None) == lib.SR_OK
    assert l.sr_backward_raster(None, ctypes.byref(cfg), 0, 0, None, None, *([None] * 14), None, md, None, None,
                                None, None) == lib.SR_ERR_ARG
    assert l.sr_render_backward(None, ctypes.byref(cfg), 0, 0, None, None, *([None] * 19), None, md, None,
                                *([None] * 6)) == lib.SR_ERR_ARG
    # statistics: none, hits alone, or hits with both maxima
    h = ctypes.c_void_p(512)
    fwd = lambda hits, ma, mw: l.sr_render_forward(None, ctypes.byref(cfg), 0, 0, None, None, *([None] * 11), hits, ma,
                                                   mw, None, None, None, None, None)
    step = lambda hits, ma, mw: l.sr_train_step_raster(None, ctypes.byref(cfg), 0, 0, None, None, None, None, None, None,
                                                       None, None, 0.5, 1.0, *([None] * 7), hits, ma, mw, None,
                                                       None, None, None, None, None, None)
    for f in (fwd, step):
        assert f(None, None, None) == lib.SR_OK
        assert f(h, None, None) == lib.SR_OK
        assert f(h, h, h) == lib.SR_OK
        assert f(h, h, None) == lib.SR_ERR_ARG
        assert f(h, None, h) == lib.SR_ERR_ARG
        assert f(None, h, h) == lib.SR_ERR_ARG


def test_regularizer_loss_arguments(lib):
    """sr_regularizer_loss: V = 0 is a no-op; missing buffers, unlaid-out or
    empty views, a small workspace and a median map without its gradient
    buffer are argument errors (host checks only)."""
    l = lib.lib()
    assert l.sr_regularizer_loss(None, 0, None, None, None, None, None, None, None, 0.0, 0.0, None, 0, None, None, None,
                                 None, None, None, None) == lib.SR_OK
    assert l.sr_regularizer_loss(None, -1, None, None, None, None, None, None, None, 0.0, 0.0, None, 0, None, None, None,
                                 None, None, None, None) == lib.SR_ERR_ARG
    cams = (lib.SrCamera * 2)()
    for c, (w, h) in zip(cams, [(5, 4), (3, 3)]):
        c.width, c.height, c.fx, c.fy = w, h, 10.0, 10.0
    cams[1].pix_offset = 20
    p = ctypes.c_void_p(256)    # never dereferenced: the checks fail first
    args = lambda ws, med=None, dmed=None: (2, ctypes.cast(cams, ctypes.c_void_p), p, p, p, p, p, med, 1.0, 1.0, p,
                                            ws, p, p, p, p, p, dmed, None)
    n = ctypes.c_size_t()
    assert l.sr_loss_workspace_size(2, ctypes.cast(cams, ctypes.c_void_p), ctypes.byref(n)) == lib.SR_OK
    assert l.sr_regularizer_loss(None, *args(n.value - 1)) == lib.SR_ERR_ARG
    assert l.sr_regularizer_loss(None, 2, ctypes.cast(cams, ctypes.c_void_p), p, None, p, p, p, None, 1.0, 1.0, p, n.value,
                                 p, p, p, p, p, None, None) == lib.SR_ERR_ARG
    assert l.sr_regularizer_loss(None, *args(n.value, med=p)) == lib.SR_ERR_ARG
    assert l.sr_regularizer_loss(None, *args(n.value, dmed=p)) == lib.SR_ERR_ARG
    cams[1].pix_offset = 19
    assert l.sr_regularizer_loss(None, *args(n.value)) == lib.SR_ERR_ARG
    cams[1].pix_offset = 20
    cams[0].fx = 0.0
    assert l.sr_regularizer_loss(None, *args(n.value)) == lib.SR_ERR_ARG


def test_ssim_arguments(lib):
    """sr_ssim_loss / sr_ssim_workspace_size host checks (nothing launched)."""
    l = lib.lib()
    n = ctypes.c_size_t()
    assert l.sr_ssim_workspace_size(0, None, 1, ctypes.byref(n)) == lib.SR_OK and n.value == 0
    cams = (lib.SrCamera * 2)()
    for c, (w, h) in zip(cams, [(40, 9), (3, 2)]):
        c.width, c.height, c.fx, c.fy = w, h, 10.0, 10.0
    cams[1].pix_offset = 360
    cp = ctypes.cast(cams, ctypes.c_void_p)
    assert l.sr_ssim_workspace_size(2, cp, 0, ctypes.byref(n)) == lib.SR_OK
    m = n.value
    assert l.sr_ssim_workspace_size(2, cp, 1, ctypes.byref(n)) == lib.SR_OK
    assert n.value >= m + 9 * 366 * 4
    p = ctypes.c_void_p(256)
    assert l.sr_ssim_loss(None, 2, cp, p, p, p, p, 0.2, p, n.value - 1, p, p, None) == lib.SR_ERR_ARG
    assert l.sr_ssim_loss(None, 2, cp, p, None, p, p, 0.2, p, n.value, p, p, None) == lib.SR_ERR_ARG
    cams[1].pix_offset = 361
    assert l.sr_ssim_loss(None, 2, cp, p, p, p, p, 0.2, p, n.value, p, p, None) == lib.SR_ERR_ARG
    assert l.sr_ssim_loss(None, -1, None, None, None, None, None, 0.2, None, 0, None, None, None) == lib.SR_ERR_ARG


def test_compact_arguments(lib):
    """sr_compact_surfels host checks (nothing launched)."""
    l = lib.lib()
    n = ctypes.c_size_t()
    assert l.sr_compact_workspace_size(100000, ctypes.byref(n)) == lib.SR_OK and n.value >= 4 * 13
    assert l.sr_compact_workspace_size(-1, ctypes.byref(n)) == lib.SR_ERR_ARG
    p = ctypes.c_void_p(256)
    src = (ctypes.c_void_p * 2)(256, 512)
    dst = (ctypes.c_void_p * 2)(1024, 512)
    w = (ctypes.c_int32 * 2)(3, 2)
    cast = lambda a: ctypes.cast(a, ctypes.c_void_p)
    # dst aliases src for the second array
    assert l.sr_compact_surfels(None, 10, p, None, 0.0, 2, cast(src), cast(dst), cast(w), p, n.value, p, None) == \
        lib.SR_ERR_ARG
    assert l.sr_compact_surfels(None, 10, p, None, 0.0, 9, cast(src), cast(dst), cast(w), p, n.value, p, None) == \
        lib.SR_ERR_ARG
    w[0] = 0
    dst[1] = 2048
    assert l.sr_compact_surfels(None, 10, p, None, 0.0, 2, cast(src), cast(dst), cast(w), p, n.value, p, None) == \
        lib.SR_ERR_ARG
    w[0] = 3
    assert l.sr_compact_surfels(None, 10, p, None, 0.0, 2, cast(src), cast(dst), cast(w), p, 0, p, None) == \
        lib.SR_ERR_ARG


def test_tile_order_arguments(lib):
    """sr_tile_order / sr_tile_order_workspace_size host checks (nothing launched)."""
    l = lib.lib()
    n = ctypes.c_size_t()
    assert l.sr_tile_order_workspace_size(0, ctypes.byref(n)) == lib.SR_OK and n.value == 0
    assert l.sr_tile_order_workspace_size(-1, ctypes.byref(n)) == lib.SR_ERR_ARG
    assert l.sr_tile_order_workspace_size(65788, ctypes.byref(n)) == lib.SR_OK and n.value >= 4 * 4 * 65788
    p = ctypes.c_void_p(256)
    assert l.sr_tile_order(None, 0, None, None, 0, None, None) == lib.SR_OK
    assert l.sr_tile_order(None, -3, p, p, n.value, p, None) == lib.SR_ERR_ARG
    assert l.sr_tile_order(None, 65788, p, p, n.value - 1, p, None) == lib.SR_ERR_ARG
    assert l.sr_tile_order(None, 65788, None, p, n.value, p, None) == lib.SR_ERR_ARG
    assert l.sr_tile_order(None, 65788, p, p, n.value, None, None) == lib.SR_ERR_ARG


def test_context_status_and_workspace_arguments(lib):
    """The context calls, the step workspace and the whole pruning pass:
    host checks only (no device is touched; without a GPU sr_create finds
    no device)."""
    l = lib.lib()
    assert lib.SR_ERR_STATE == -5 and lib.SR_STATUS_CAPACITY == 1
    assert l.sr_destroy(None) == lib.SR_OK
    assert l.sr_create(None, 0) == lib.SR_ERR_ARG
    h = ctypes.c_void_p()
    assert l.sr_create(ctypes.byref(h), -1) == lib.SR_ERR_ARG
    assert l.sr_read_status(None, None, 1, None, None) == lib.SR_ERR_ARG
    assert l.sr_clear_status(None, None) == lib.SR_ERR_ARG
    cams = (lib.SrCamera * 3)()
    for c, (w, hh) in zip(cams, [(40, 21), (33, 48), (64, 64)]):
        c.width, c.height, c.fx, c.fy = w, hh, 10.0, 10.0
    cp = ctypes.cast(cams, ctypes.c_void_p)
    lib.call("sr_layout_views", cp, 3, 16, 16, None, None)
    cfg = lib.SrConfig(16, 16, 0, 1, 1 / 255, 0.99, 1e-4, 0)
    n, part = ctypes.c_size_t(), ctypes.c_size_t()
    # one step workspace covers each call's own
    assert l.sr_workspace_size(ctypes.byref(cfg), 500, 3, cp, 7000, ctypes.byref(n)) == lib.SR_OK
    assert l.sr_bin_workspace_size(500, 3, 7000, ctypes.byref(part)) == lib.SR_OK and n.value >= part.value
    assert l.sr_loss_workspace_size(3, cp, ctypes.byref(part)) == lib.SR_OK and n.value >= part.value
    assert l.sr_ssim_workspace_size(3, cp, 1, ctypes.byref(part)) == lib.SR_OK and n.value >= part.value
    assert l.sr_tile_order_workspace_size(3 * 2 + 3 * 3 + 16, ctypes.byref(part)) == lib.SR_OK
    assert n.value >= part.value
    assert l.sr_workspace_size(ctypes.byref(cfg), -1, 3, cp, 7000, ctypes.byref(n)) == lib.SR_ERR_ARG
    # the pruning pass: primitive kind, chunking, sizes
    ws = lambda prim, vpc, cap: (l.sr_prune_workspace_size(ctypes.byref(cfg), prim, 1000, 3, cp, vpc, cap,
                                                           ctypes.byref(n)), n.value)
    assert ws(2, 2, 0)[0] == lib.SR_ERR_ARG
    assert ws(lib.SR_PRIM_SURFEL, 0, 0)[0] == lib.SR_ERR_ARG
    st, one = ws(lib.SR_PRIM_SURFEL, 1, 0)
    st2, two = ws(lib.SR_PRIM_SURFEL, 2, 0)
    st3, big = ws(lib.SR_PRIM_SURFEL, 2, 100000)
    assert st == st2 == st3 == lib.SR_OK and one < two < big
    assert ws(lib.SR_PRIM_GAUSS3D, 2, 0)[1] < two       # 8 floats of geometry per record instead of 16
    p = ctypes.c_void_p(256)
    prune = lambda ctx, ws_bytes, vpc=2: l.sr_prune_contrib(ctx, ctypes.byref(cfg), lib.SR_PRIM_SURFEL, 1000, p, p, p,
                                                            p, 3, cp, p, vpc, 1 / 255, 0, p, ws_bytes, p, p, p, None,
                                                            p, None)
    assert prune(None, two - 1) == lib.SR_ERR_ARG                      # workspace too small
    assert prune(None, two, vpc=0) == lib.SR_ERR_ARG
    assert prune(None, two) == lib.SR_ERR_ARG                          # valid but for the context
    assert b"ctx" in l.sr_last_error()
    cap = ctypes.c_uint32()
    assert l.sr_prune_plan(None, ctypes.byref(cfg), lib.SR_PRIM_SURFEL, 1000, p, p, p, p, 3, cp, p, 2, p, two,
                           ctypes.byref(cap), None) == lib.SR_ERR_ARG
    # a call with work to enqueue needs a context; one without returns at once
    assert l.sr_prune_mask(None, 10, p, 0.5, p, None) == lib.SR_ERR_ARG and b"ctx" in l.sr_last_error()
    assert l.sr_prune_mask(None, 0, None, 0.5, None, None) == lib.SR_OK
    assert l.sr_tile_order(None, 0, None, None, 0, None, None) == lib.SR_OK
