"""HIP-graph capture of the training step (projection, binning, fused
compositing with the usage counts, projection backward): every replay of the
captured step equals the eager step, with eager work of the same library and
of torch, and synchronisations, between the replays."""
import numpy as np
import pytest
import torch

from paper_2501_08174_amd import scenes
from paper_2501_08174_amd.raster import Params, Rasterizer, ViewBatch

pytestmark = pytest.mark.gpu

OUTS = ("color", "alpha", "depth", "normal", "dist", "T_final", "n_contrib")


def test_graph_replays_match_eager_step():
    sc = scenes.make_random_scene(41, 3000, n_views=3, width=[96, 130, 64], height=[80, 57, 120], sh_degree=3,
                                  scale_range=(0.01, 0.3))
    rng = np.random.default_rng(5)
    views = ViewBatch(sc.cams)
    mask = torch.tensor(rng.integers(0, 2, views.P).astype(np.uint8), device="cuda")
    target = torch.tensor(rng.uniform(size=3 * views.P).astype(np.float32), device="cuda")
    p = Params.from_scene(sc)
    g = Params(*[torch.zeros_like(t) for t in (p.means, p.scales, p.quats, p.opac, p.sh)])
    grads = (g.means, g.scales, g.quats, g.opac, g.sh)
    hits = torch.zeros(sc.n, dtype=torch.int32, device="cuda")
    rast = Rasterizer(sc.n, views, sc.sh_degree, sh_stride=sc.sh.shape[1])
    rast.plan_capacity(p)

    def step():
        rast.preprocess(p)
        rast.bin()
        loss = rast.train_step_raster(mask, target, 0.5, 1.0, stats=hits)   # hits cleared by the call
        rast.backward_project(p, g)
        return loss

    def snapshot(loss):
        torch.cuda.synchronize()
        return ({k: getattr(rast, k).clone() for k in OUTS}, hits.clone(), loss.clone(),
                [t.clone() for t in grads])

    for t in grads:
        t.zero_()
    ref = snapshot(step())
    assert int((ref[1] > 0).sum().item()) > 0

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        loss_g = step()

    for rep in range(3):
        # eager work between the replays: a forward of the same rasterizer
        # (overwrites the outputs the replay must restore) and a torch reduction
        rast.forward()
        noise = torch.rand(4096, device="cuda").sum()
        for t in grads:
            t.zero_()
        torch.cuda.synchronize()
        assert float(noise.item()) > 0.0
        graph.replay()
        outs, h, loss, gr = snapshot(loss_g)
        for k in OUTS:
            assert torch.equal(outs[k], ref[0][k]), (rep, k)
        assert torch.equal(h, ref[1]), rep
        assert torch.equal(loss, ref[2]), rep
        for x, y in zip(gr, ref[3]):
            # the gradient accumulators take float atomics: order-dependent rounding only
            tol = 1e-5 * float(y.abs().max().item()) + 1e-12
            assert float((x - y).abs().max().item()) <= tol, rep
        print(f"replay {rep}: outputs, counts and loss identical; gradients within atomic-order rounding",
              flush=True)
