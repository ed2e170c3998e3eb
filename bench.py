"""Throughput of the object-centric 2DGS hot path on one MI355X.

One step = projection -> binning/sort -> forward compositing (recording the
blended-pixel count of every surfel, the usage the occlusion pruning of
Section 4.3 acts on) -> masked L1 + background loss -> backward compositing
-> projection backward, over all views of the batch (every stage is one
launch for all views; the compositing forward, loss and backward share one
fused launch).  The default workload is the 1M-surfel batch of 16 views
with uneven sides (400..1600 px) and degree-3 colour; per-view mode runs
the same kernels one view at a time.  Besides the headline step the line
carries the same step with the full occlusion statistics (also the maximum
alpha and weight) and with no usage record, the separate-launch step, the
hipGraph replay, the step with the whole Eq. 3 loss (D-SSIM and the 2DGS
regularisers, with the expected and with the median depth), the density
statistic and compaction, and with --prune-legs the occlusion-pruning pass
for surfels and 3D Gaussians.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ragged16-1m]

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Lane-op and byte costs per unit of work (see the design notes): forward
# compositing ~45 lane-ops per blended pair and ~26 per skipped pair,
# backward ~110 per blended pair (recompute, gradients, wave reduction) and
# ~26 per skipped pair.
FWD_OPS_BLEND, FWD_OPS_SKIP = 45.0, 26.0
BWD_OPS_BLEND, BWD_OPS_SKIP = 110.0, 26.0
VALU_PEAK = 256 * 64 * 2.4e9          # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
HBM_PEAK = 8.0e12                      # bytes/s
# masked D-SSIM with its gradient, per pixel: colour and target read (24 B),
# mask (1 B), the colour gradient read and written (24 B); per channel 5
# moments x 11 taps x 2 passes (110 FMA) + 3 products + ~22 for S and its
# three derivatives, backward 3 maps x 22 taps + ~6 to combine: ~207, x 3
SSIM_BYTES_PX, SSIM_OPS_PX = 49, 620


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_train_raster_ragged16_1m_traffic.md")


def measured_traffic(workload, tile):
    """HBM bytes per launch of the fused compositing kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the copy-kernel
    calibration written there), or None when the summary is missing, was
    taken on another workload or tile shape, or when the kernel sources have
    changed since (their SHA-256 differs)."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines() if ": " in line and
                      line.split(": ", 1)[0] in ("workload", "kernel_sources", "kernel_source_sha256",
                                                 "traffic_bytes_per_launch"))
        if kv["workload"].strip() != f"{workload} {tile[0]}x{tile[1]}":
            return None
        h = hashlib.sha256()
        for rel in kv["kernel_sources"].split():
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != kv["kernel_source_sha256"].strip():
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ragged16-1m", choices=["frame800-100k", "ragged16-1m", "wide8-3m"])
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--tile", default="auto",
                    help="WxH tile shape, or 'auto' to pick the tile shape and backward batch by timing")
    ap.add_argument("--bwd-batch", type=int, default=0,
                    help="backward LDS batch with an explicit --tile (0: the library's default)")
    ap.add_argument("--no-unfused", action="store_true", help="skip timing the separate-launch step")
    ap.add_argument("--no-eq3", action="store_true", help="skip timing the step with the whole Eq. 3 loss")
    ap.add_argument("--prune-legs", action="store_true",
                    help="also time the occlusion-pruning pass (surfels and 3D Gaussians) on the shell scene")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for the HBM traffic counters)")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    return ap.parse_args()


def make_scene(name):
    from paper_2501_08174_amd import scenes
    return {"frame800-100k": scenes.make_frame800_100k, "ragged16-1m": scenes.make_ragged16_1m,
            "wide8-3m": scenes.make_wide8_3m}[name]()


class Pipeline:
    """Persistent buffers and one training step over a set of views."""

    def __init__(self, scene, cams, masks, targets, params, grads, stats, tile=(16, 16), bwd_batch=0):
        import torch
        from paper_2501_08174_amd.raster import Rasterizer, ViewBatch
        self.views = ViewBatch(cams, tile=tile)
        self.rast = Rasterizer(scene.n, self.views, scene.sh_degree, sh_stride=scene.sh.shape[1],
                               bwd_batch=bwd_batch)
        self.p, self.g, self.stats = params, grads, stats
        self.used = torch.zeros(scene.n, dtype=torch.int32, device="cuda")
        self.mask = torch.tensor(np.concatenate([m.reshape(-1) for m in masks]), device="cuda")
        self.target = torch.tensor(np.concatenate([t.reshape(-1) for t in targets]), device="cuda")
        self.dA = torch.zeros_like(self.rast.alpha)
        self.dC = torch.zeros_like(self.rast.color)
        self.dD = torch.zeros_like(self.rast.depth)
        self.dN = torch.zeros_like(self.rast.normal)
        self.dS = torch.zeros_like(self.rast.dist)
        self.dM = torch.zeros_like(self.rast.depth)
        self.need = self.rast.plan_capacity(params, slack=1.02)

    STAGES = ("preprocess", "bin_sort", "train_raster", "backward_project")
    STAGES_UNFUSED = ("preprocess", "bin_sort", "forward", "loss", "backward_raster", "backward_project")
    STAGES_EQ3 = ("preprocess", "bin_sort", "forward", "loss", "ssim", "regularizers", "backward_raster",
                  "backward_project")

    def step(self, ev=None, fused=True, eq3=None, stats="hits"):
        """One training step; the compositing is the fused forward + loss +
        backward launch (fused=True) or the three separate launches; with
        eq3 = (w_dist, w_normal[, median]) the loss is the whole Eq. 3 (the
        2DGS regularisers need neighbouring pixels, so the launches are
        separate); with median the normal term takes the median depth as its
        surface.  stats: "hits" (default) has the forward count the blended
        pixels of every surfel into self.used, the record of used Gaussians
        the renderer keeps during training for the occlusion pruning applied
        every 100 or 600 iterations (Section 4.3, Section 5.1); "full" also
        takes the maximum alpha and weight (self.stats); None records
        nothing."""
        r = self.rast
        st = {"hits": self.used, "full": self.stats, None: None}[stats]
        rec = (lambda i: ev[i].record()) if ev is not None else (lambda i: None)
        rec(0)
        r.preprocess(self.p)
        rec(1)
        r.bin()
        rec(2)
        if eq3 is not None:
            # L_c^M = (1 - lambda) L1 + lambda D-SSIM on the masked images (lambda = 0.2)
            med = len(eq3) > 2 and eq3[2]
            r.forward(stats=st, accumulate=True, median=med)
            rec(3)
            r.loss(self.mask, self.target, 0.5, 0.8, self.dA, self.dC)
            rec(4)
            r.ssim_loss(self.mask, self.target, 0.2, dL_dcolor=self.dC)
            rec(5)
            dM = self.dM if med else None
            r.regularizer_loss(eq3[0], eq3[1], self.dA, self.dD, self.dN, self.dS, dL_dmedian=dM)
            rec(6)
            r.backward_raster(dC=self.dC, dA=self.dA, dD=self.dD, dN=self.dN, dS=self.dS, dM=dM)
            rec(7)
        elif fused:
            r.train_step_raster(self.mask, self.target, 0.5, 1.0, stats=st, accumulate=True)
            rec(3)
        else:
            r.forward(stats=st, accumulate=True)
            rec(3)
            r.loss(self.mask, self.target, 0.5, 1.0, self.dA, self.dC)
            rec(4)
            r.backward_raster(dC=self.dC, dA=self.dA)
            rec(5)
        r.backward_project(self.p, self.g)
        rec(8 if eq3 is not None else (4 if fused else 6))


def _oracle_crops(scene, seconds_budget, threads):
    """Oracle forward + backward (FP64 autograd) over 64x64 crops of view 0:
    (pixels per second, crops, seconds)."""
    import torch
    import oracle
    from oracle.render import Params64, render_pixels
    torch.set_num_threads(threads)
    rp = oracle.RasterParams()
    cam = scene.cams[0]
    g = oracle.view_geometry64(scene.means, scene.scales, scene.quats, scene.opac, cam, rp)
    P = Params64.from_arrays(scene.means, scene.scales, scene.quats, scene.opac, scene.sh, scene.sh_degree,
                             requires_grad=True)
    x0, y0 = cam.width // 2 - 32, cam.height // 2 - 32
    done_px, t0, crops = 0, time.perf_counter(), 0
    while True:
        jj, ii = np.meshgrid(np.arange(y0, y0 + 64), np.arange(x0, x0 + 64), indexing="ij")
        pix = np.stack([ii.ravel(), jj.ravel()], axis=1)
        render_pixels(P, cam, g, pix, rp, loss_fn=lambda out, rows: out["color"].sum() + out["alpha"].sum())
        done_px += pix.shape[0]
        crops += 1
        if time.perf_counter() - t0 > seconds_budget or crops >= 8:
            break
        x0 = (x0 + 64) % max(cam.width - 64, 1)
    dt = time.perf_counter() - t0
    return done_px / dt, crops, dt


def cpu_baseline_child(workload):
    """The crop leg on one core (run as a child process with
    OMP_NUM_THREADS=1, started before the parent touches the GPU)."""
    scene = make_scene(workload)
    px_s, crops, dt = _oracle_crops(scene, 20.0, 1)
    print(json.dumps({"value": px_s / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
                      "sample": f"{crops} crop(s) of 64x64 px of view 0, fwd+bwd FP64, {scene.n} surfels, "
                                f"{dt:.1f} s"}), flush=True)


def start_one_core_baseline(workload):
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", MKL_NUM_THREADS="1", HIP_VISIBLE_DEVICES="",
               CUDA_VISIBLE_DEVICES="")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                             "--workload", workload], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env,
                            text=True)


def cpu_baseline(scene, one_core_proc=None, seconds_budget=20.0):
    """The oracle timed on the host: the headline leg (fwd+bwd on 64x64 crops
    of view 0 of the benchmark workload, all cores), the same on one core
    (child process), the 64x64 single-view workload's full frame (forward),
    and a sample of the shell-scene pruning statistics (the plain-C oracle
    loop over four of its 100 views)."""
    import oracle
    from oracle.prune_native import prune_stats_views64
    from oracle.render import Params64, render_view
    from paper_2501_08174_amd import scenes
    threads = len(os.sched_getaffinity(0))
    one = None
    if one_core_proc is not None:
        # the one-core leg finishes first: a busy core would stall every
        # parallel region of the all-core leg
        try:
            txt, _ = one_core_proc.communicate(timeout=180)
            one = json.loads(txt.strip().splitlines()[-1])
        except Exception as e:  # the headline leg stands without it
            one = {"error": repr(e)[:200]}
    px_s, crops, dt = _oracle_crops(scene, seconds_budget, threads)
    out = {"value": px_s / 1e6, "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
           "sample": f"{crops} crops of 64x64 px of view 0 ({scene.cams[0].width}x{scene.cams[0].height}), "
                     f"fwd+bwd FP64, {scene.n} surfels, {dt:.1f} s"}
    legs = {}
    rp = oracle.RasterParams()
    f1 = scenes.make_frame64_1k()
    cam = f1.cams[0]
    g = oracle.view_geometry64(f1.means, f1.scales, f1.quats, f1.opac, cam, rp)
    P = Params64.from_arrays(f1.means, f1.scales, f1.quats, f1.opac, f1.sh, f1.sh_degree)
    t0 = time.perf_counter()
    render_view(P, cam, g, rp)
    t1 = time.perf_counter() - t0
    legs["frame64_1k_forward"] = {"value": cam.width * cam.height / t1 / 1e6, "unit": "Mpixel/s",
                                  "cores": threads, "sample": f"the full 64x64 frame, 1k surfels, forward FP64, "
                                                              f"{t1:.2f} s"}
    sh = scenes.make_shell100()
    t0 = time.perf_counter()
    prune_stats_views64(sh.means, sh.scales, sh.quats, sh.opac, sh.cams[:4], rp, workers=min(threads, 16))
    t4 = time.perf_counter() - t0
    px4 = sum(c.width * c.height for c in sh.cams[:4])
    legs["shell100_pruning_sample"] = {"value": px4 / t4 / 1e6, "unit": "Mpixel/s", "cores": min(threads, 16),
                                       "sample": f"occlusion statistics of 4 of the 100 views (800x800, 1.1M "
                                                 f"surfels), plain-C FP64 loop, {t4:.1f} s"}
    if one is not None:
        legs["one_core"] = one
    out["legs"] = legs
    return out


def main():
    args = parse()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is a "
              f"design (view sharding + one all-reduce of the surfel gradients), not built.", file=sys.stderr)
        sys.exit(2)
    # the one-core oracle leg runs beside the GPU work, in a child started
    # before this process touches the GPU
    one_core = None if args.no_cpu_baseline else start_one_core_baseline(args.workload)
    import torch
    from paper_2501_08174_amd.raster import Params

    t_gen = time.perf_counter()
    scene = make_scene(args.workload)
    t_gen = time.perf_counter() - t_gen
    N, V = scene.n, scene.v
    params = Params.from_scene(scene)
    grads = Params(*[torch.zeros_like(t) for t in (params.means, params.scales, params.quats, params.opac,
                                                   params.sh)])
    stats = (torch.zeros(N, dtype=torch.int32, device="cuda"), torch.zeros(N, device="cuda"),
             torch.zeros(N, device="cuda"))
    tune = {}
    if args.tile == "auto":
        from paper_2501_08174_amd.autotune import autotune
        mask = torch.tensor(np.concatenate([m.reshape(-1) for m in scene.masks]), device="cuda")
        target = torch.tensor(np.concatenate([t.reshape(-1) for t in scene.targets]), device="cuda")
        tile, bwd_batch = autotune(scene.cams, params, scene.sh_degree, scene.sh.shape[1], mask, target,
                                   use_cache=False, report=tune)
        del mask, target
        torch.cuda.empty_cache()
    else:
        tile = tuple(int(x) for x in args.tile.split("x"))
        bwd_batch = args.bwd_batch
    pipe = Pipeline(scene, scene.cams, scene.masks, scene.targets, params, grads, stats, tile, bwd_batch)
    P = pipe.views.P

    for _ in range(args.warmup):
        pipe.step()
    torch.cuda.synchronize()
    vis, need, stored, status = pipe.rast.status()
    assert status == 0, "instance capacity exceeded"

    # timed region: K eager steps with per-stage events
    ns = len(Pipeline.STAGES)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        pipe.step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(ns)] for k in range(args.steps)])
    step_ms = stage_ms.sum(axis=1)
    ms_per_step = wall / args.steps * 1e3

    result = {
        "metric": f"fwd+bwd Mpixel/s (batched, {N / 1e6:g}M surfels)",
        "value": P / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {V} views, {P} px, {N} surfels, SH degree {scene.sh_degree}",
                   "views": V, "pixels": P, "surfels": N, "mode": "batched", "tile": f"{tile[0]}x{tile[1]}",
                   "bwd_batch": pipe.rast.cfg.bwd_batch},
        "autotune_ms": tune.get("ms"),
        "views_per_s": V / (ms_per_step * 1e-3),
        "median_step_ms_events": float(np.median(step_ms)),
        "stage_ms_mean": dict(zip(Pipeline.STAGES, [float(x) for x in stage_ms.mean(axis=0)])),
        "counts": {"visible_pairs": vis, "instances": need},
        "scene_gen_s": t_gen,
    }

    # work accounting for the roofline (outside the timed region)
    R, B, WS, WB, R_bwd = pipe.rast.count_pairs(waves=True)
    upto_last = int(pipe.rast.n_contrib[:P].to(torch.int64).sum().item())
    mean_ms = dict(zip(Pipeline.STAGES, stage_ms.mean(axis=0)))
    fwd_ops = FWD_OPS_BLEND * B + FWD_OPS_SKIP * (R - B)
    bwd_ops = BWD_OPS_BLEND * B + BWD_OPS_SKIP * max(R_bwd - B, 0)
    ops = fwd_ops + bwd_ops
    achieved = ops / (mean_ms["train_raster"] * 1e-3) / 1e12
    result["roofline"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK / 1e12, "unit": "Tlane-op/s",
                          "frac": achieved / (VALU_PEAK / 1e12),
                          "traffic": measured_traffic(args.workload, tile),
                          "kernel": "k_train_raster with the usage counts (fused forward + loss + backward "
                                    "compositing)",
                          "ops_per_launch": ops}
    result["counts"].update({"reached_pairs": R, "blended_pairs": B, "backward_pairs": R_bwd,
                             "list_entries_up_to_last": upto_last,
                             "forward_wave_steps": WS, "forward_wave_steps_blending": WB})

    # the same step with the full occlusion statistics in the fused launch
    # (hits, maximum alpha and maximum weight; they feed the density/pruning
    # leg below), and with no usage record at all
    def stats_leg(mode):
        ev_s = [[torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)] for _ in range(args.steps)]
        pipe.step(stats=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            pipe.step(ev_s[k], stats=mode)
        torch.cuda.synchronize()
        s_ms = (time.perf_counter() - t0) / args.steps * 1e3
        st_s = np.array([[ev_s[k][i].elapsed_time(ev_s[k][i + 1]) for i in range(ns)] for k in range(args.steps)])
        return {"ms_per_step": s_ms, "Mpixel_per_s": P / (s_ms * 1e-3) / 1e6,
                "stage_ms_mean": dict(zip(Pipeline.STAGES, [float(x) for x in st_s.mean(axis=0)]))}
    result["full_prune_stats"] = stats_leg("full")
    result["no_usage_record"] = stats_leg(None)

    if not args.no_unfused:
        # the same step with separate forward / loss / backward launches
        ns_u = len(Pipeline.STAGES_UNFUSED)
        ev_u = [[torch.cuda.Event(enable_timing=True) for _ in range(ns_u + 1)] for _ in range(args.steps)]
        for k in range(args.steps):
            pipe.step(ev_u[k], fused=False)
        torch.cuda.synchronize()
        st_u = np.array([[ev_u[k][i].elapsed_time(ev_u[k][i + 1]) for i in range(ns_u)] for k in range(args.steps)])
        result["unfused"] = {"ms_per_step": float(st_u.sum(axis=1).mean()),
                             "stage_ms_mean": dict(zip(Pipeline.STAGES_UNFUSED,
                                                       [float(x) for x in st_u.mean(axis=0)]))}

    if not args.no_eq3:
        # the whole Eq. 3: masked photometric loss (0.8 L1 + 0.2 D-SSIM) +
        # background + 2DGS distortion and normal consistency (2DGS's weights
        # for bounded scenes)
        w_dist, w_normal = 1000.0, 0.05
        ns_e = len(Pipeline.STAGES_EQ3)

        def eq3_leg(median):
            ev_e = [[torch.cuda.Event(enable_timing=True) for _ in range(ns_e + 1)] for _ in range(args.steps)]
            pipe.step(eq3=(w_dist, w_normal, median))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(args.steps):
                pipe.step(ev_e[k], eq3=(w_dist, w_normal, median))
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            return ms, np.array([[ev_e[k][i].elapsed_time(ev_e[k][i + 1]) for i in range(ns_e)]
                                 for k in range(args.steps)])
        e_ms, st_e = eq3_leg(False)
        reg_ms = float(st_e[:, Pipeline.STAGES_EQ3.index("regularizers")].mean())
        reg_bytes = 52 * P
        ssim_ms = float(st_e[:, Pipeline.STAGES_EQ3.index("ssim")].mean())
        ssim_bytes = SSIM_BYTES_PX * P
        result["eq3"] = {"ms_per_step": e_ms, "Mpixel_per_s": P / (e_ms * 1e-3) / 1e6, "w_dist": w_dist,
                         "w_normal": w_normal,
                         "stage_ms_mean": dict(zip(Pipeline.STAGES_EQ3, [float(x) for x in st_e.mean(axis=0)])),
                         "regularizer_roofline": {"bound": "hbm", "achieved": reg_bytes / (reg_ms * 1e-3) / 1e9,
                                                  "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                                  "frac": reg_bytes / (reg_ms * 1e-3) / HBM_PEAK,
                                                  "bytes_per_launch": reg_bytes},
                         "ssim_roofline": {"bound": "hbm", "achieved": ssim_bytes / (ssim_ms * 1e-3) / 1e9,
                                           "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                           "frac": ssim_bytes / (ssim_ms * 1e-3) / HBM_PEAK,
                                           "bytes_per_call": ssim_bytes,
                                           "valu_frac": SSIM_OPS_PX * P / (ssim_ms * 1e-3) / VALU_PEAK,
                                           "lane_ops_per_call": SSIM_OPS_PX * P}}
        # the same step with the median depth as the surface of the normal term
        m_ms, st_m = eq3_leg(True)
        result["eq3_median"] = {"ms_per_step": m_ms, "Mpixel_per_s": P / (m_ms * 1e-3) / 1e6,
                                "stage_ms_mean": dict(zip(Pipeline.STAGES_EQ3, [float(x) for x in st_m.mean(axis=0)]))}

    if not args.no_eq3:
        # density control and pruning of a training step: the screen-gradient
        # statistic fused into the projection backward (its cost), and the
        # compaction of the parameters by the occlusion-pruning mask
        from paper_2501_08174_amd.raster import compact_surfels, prune_mask
        dsum = torch.zeros(N, device="cuda")
        dcnt = torch.zeros(N, dtype=torch.int32, device="cuda")
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        t_plain, t_dens = [], []
        for k in range(args.steps):
            pipe.rast.preprocess(pipe.p)
            pipe.rast.bin()
            pipe.rast.train_step_raster(pipe.mask, pipe.target, 0.5, 1.0)
            e[0].record()
            pipe.rast.backward_project(pipe.p, pipe.g)
            e[1].record()
            pipe.rast.train_step_raster(pipe.mask, pipe.target, 0.5, 1.0)
            e[2].record()
            pipe.rast.backward_project(pipe.p, pipe.g, densify=(dsum, dcnt))
            e[3].record()
            torch.cuda.synchronize()
            t_plain.append(e[0].elapsed_time(e[1]))
            t_dens.append(e[2].elapsed_time(e[3]))
        pm = prune_mask(stats[1], 1.0 / 255.0)
        arrays = [params.means, params.scales, params.quats, params.opac, params.sh]
        compact_surfels(pm, arrays)
        torch.cuda.synchronize()
        e[4].record()
        out = compact_surfels(pm, arrays)
        e[5].record()
        torch.cuda.synchronize()
        kept = int(out[0].shape[0])
        row = sum(int(np.prod(a.shape[1:])) if a.dim() > 1 else 1 for a in arrays) * 4
        c_ms = e[4].elapsed_time(e[5])
        c_bytes = 2 * N + kept * row * 2                   # mask read by both passes; kept rows read and written
        result["density_and_pruning"] = {
            "projection_backward_ms": float(np.median(t_plain)),
            "projection_backward_with_statistic_ms": float(np.median(t_dens)),
            "pruned": N - kept, "kept": kept,
            "compaction_ms_incl_host_sync": c_ms,
            "compaction_GBps": c_bytes / (c_ms * 1e-3) / 1e9}

    if args.prune_legs:
        # the occlusion-pruning pass (Section 4.3) on the shell scene of 100
        # views of 800x800 (1.1M primitives), for surfels and for 3D Gaussians
        from paper_2501_08174_amd import scenes as _sc
        from paper_2501_08174_amd.raster import prune_contrib, prune_contrib_3d
        sc4, s3 = _sc.make_shell100_3d()
        p4 = Params.from_scene(sc4)
        s3t = torch.tensor(s3, device="cuda")
        P4 = sum(c.width * c.height for c in sc4.cams)
        legs = {}
        for name, fn in (("surfels", lambda: prune_contrib(p4, sc4.cams, views_per_chunk=32)),
                         ("gaussians_3d", lambda: prune_contrib_3d(p4.means, s3t, p4.quats, p4.opac, sc4.cams,
                                                                   views_per_chunk=32))):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            legs[name] = {"s": dt, "Mpixel_per_s": P4 / dt / 1e6,
                          "pruned": int(st.mask.sum().item()), "of": sc4.n}
        result["pruning_pass"] = {"workload": "shell100: shell scene, 100 views 800x800, 1.1M primitives, "
                                              "views in chunks of 32 (capacity planning included)", **legs}
        del p4, s3t

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = src.numel() * 4
        del src, dst

    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            pipe.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            pipe.step()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        result["ms_per_step_graph"] = (time.perf_counter() - t0) / args.steps * 1e3

    if not args.no_per_view:
        pipes = []
        for v in range(V):
            pv = Pipeline(scene, [scene.cams[v]], [scene.masks[v]], [scene.targets[v]], params, grads, stats, tile,
                          bwd_batch)
            pipes.append(pv)
        for _ in range(args.warmup):
            for pv in pipes:
                pv.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for pv in pipes:
                pv.step()
        torch.cuda.synchronize()
        pv_ms = (time.perf_counter() - t0) / args.steps * 1e3
        result["per_view"] = {"ms_per_step": pv_ms, "Mpixel_per_s": P / (pv_ms * 1e-3) / 1e6,
                              "views_per_s": V / (pv_ms * 1e-3)}
        # equal accuracy: the batched forward is bit-identical to the per-view one
        pipe.step()
        for pv in pipes:
            pv.step()
        torch.cuda.synchronize()
        same = all(torch.equal(pipe.rast.alpha[pipe.views.view_slice(v)], pv.rast.alpha[: pv.views.P]) and
                   torch.equal(pipe.rast.color[pipe.views.view_slice(v, 3)], pv.rast.color[: 3 * pv.views.P])
                   for v, pv in enumerate(pipes))
        result["per_view"]["forward_bit_identical"] = bool(same)
        del pipes

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene, one_core)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
