"""sr_train_step_raster_noalloc, the training step for callers that cannot
allocate device memory (its per-tile loss partials in the library's static
scratch array), against sr_train_step_raster through the C ABI: two calls in
a row, the second on a smaller view batch, give the allocating call's
outputs, losses and statistics bit for bit and its gradients up to the
rounding order of float atomics; a batch beyond the array's capacity is
rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2501_08174_amd import _lib, scenes
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch, make_config

pytestmark = pytest.mark.gpu
OUTS = ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _step(sc, noalloc):
    views = ViewBatch(sc.cams)
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    p = Params.from_scene(sc)
    rast.plan_capacity(p)
    rast.preprocess(p)
    rast.bin()
    mask = torch.tensor(np.concatenate([m.reshape(-1) for m in sc.masks]).astype(np.uint8), device="cuda")
    target = torch.tensor(np.concatenate([t.reshape(-1) for t in sc.targets]), device="cuda")
    hits = torch.zeros(sc.n, dtype=torch.int32, device="cuda")
    loss = rast.train_step_raster(mask, target, 0.5, 1.0, stats=hits, schedule=False, noalloc=noalloc)
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    rast.backward_project(p, g)
    rast.check_capacity()
    torch.cuda.synchronize()
    return ({k: getattr(rast, k).clone() for k in OUTS}, loss.clone(), hits,
            [t.clone() for t in (g.means, g.scales, g.quats, g.opac, g.sh)], views.T)


def test_noalloc_step_equals_allocating_step():
    big = scenes.make_random_scene(81, 3000, n_views=3, width=[150, 97, 120], height=[90, 121, 64], sh_degree=3,
                                   scale_range=(0.01, 0.4))
    small = scenes.make_random_scene(82, 800, n_views=2, width=[61, 40], height=[37, 64], sh_degree=3,
                                     scale_range=(0.02, 0.3))
    refs = [_step(sc, False) for sc in (big, small)]
    got = [_step(sc, True) for sc in (big, small)]          # two calls in a row, the second smaller
    assert refs[1][4] < refs[0][4]
    for (fa, la, ha, ga, _), (fb, lb, hb, gb, _) in zip(refs, got):
        for k in OUTS:
            assert torch.equal(fa[k], fb[k]), k
        assert torch.equal(la, lb) and torch.isfinite(la).all()
        assert torch.equal(ha, hb)
        for x, y in zip(ga, gb):
            assert float((x - y).abs().max().item()) <= 1e-5 * float(y.abs().max().item()) + 1e-12


def test_noalloc_rejects_more_tiles_than_the_array_holds():
    cams = (_lib.SrCamera * 2)()
    for c in cams:
        c.width, c.height, c.fx, c.fy = 8192, 8192, 100.0, 100.0
    P, T = ctypes.c_int64(0), ctypes.c_int32(0)
    _lib.call("sr_layout_views", ctypes.cast(cams, ctypes.c_void_p), 2, 16, 16, ctypes.byref(P), ctypes.byref(T))
    assert T.value > _lib.SR_NOALLOC_MAX_TILES
    ctx = _lib.Context(torch.cuda.current_device())
    cfg = make_config(0)
    dummy = ctypes.c_void_p(256)        # never dereferenced: the size check fails first
    st = _lib.lib().sr_train_step_raster_noalloc(ctx.ptr, ctypes.byref(cfg), 10, 2, ctypes.cast(cams, ctypes.c_void_p),
                                                  dummy, *([None] * 6), 0.5, 1.0, *([None] * 16))
    assert st == _lib.SR_ERR_ARG and b"SR_NOALLOC_MAX_TILES" in _lib.lib().sr_last_error()
