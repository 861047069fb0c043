"""Benchmark: forward frames/s and forward+backward steps/s of the 4D-rotor
Gaussian render path on one MI355X.

Workload (default): 500,000 4D Gaussians, SH degree 3, one 1352x1014 render
at t = 0.5 from (0, 0, -4); a step = forward render + L1 loss gradient against
a seeded U[0,1] target + backward to all Gaussian parameters.  Inputs are
seeded synthetic arrays resident in HBM before timing starts.

Prints one JSON line.  `value` is fwd+bwd steps/s; per-stage kernel times come
from HIP events the library records on the stream it launches on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (256 CU x 2.4 GHz x 256 flop/clk/CU)

# Arithmetic of one evaluated (pixel, Gaussian) pair in the forward compositing
# loop: offset (2), quadratic form (7), exponent (2: scale + exp), opacity
# product, clamp, two threshold tests (4), transmittance update (2),
# weight (1) and colour accumulation (3 fma = 6).  Skipped pairs do less; the
# count is an upper bound on useful work per evaluated pair.
FLOPS_PER_PAIR_FWD = 24


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile-size", type=int, default=16)
    ap.add_argument("--fwd-ppt", type=int, default=0,
                    help="forward rasteriser pixels per lane (0 = library default)")
    ap.add_argument("--bwd-ppt", type=int, default=0,
                    help="backward rasteriser pixels per lane (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of "
                         "known traffic, to scale hardware byte counters)")
    ap.add_argument("--cpu-pixels", type=int, nargs=2, default=(16, 64),
                    help="two oracle pixel-sample sizes used to fit fixed + per-pixel cost")
    return ap.parse_args()


def cpu_baseline(g, view, st, pix_counts):
    """The FP64 oracle (forward + autograd backward) on the same scene, timed
    on a bounded pixel sample; the full-frame step time is extrapolated
    linearly in the number of pixels from two sample sizes."""
    import torch

    import workloads as W
    from oracle import render as O

    H, Wd = int(view["height"]), int(view["width"])
    times = []
    for P in pix_counts:
        pix = W.pixel_sample(H, Wd, P, seed=7)
        t0 = time.perf_counter()
        out = O.render(g, view, st, pixels=pix, requires_grad=True)
        out["image"].sum().backward()
        times.append(time.perf_counter() - t0)
    (p1, p2), (t1, t2) = pix_counts, times
    per_pixel = max((t2 - t1) / (p2 - p1), 1e-12)
    fixed = max(t1 - per_pixel * p1, 0.0)
    step_s = fixed + per_pixel * H * Wd
    return {
        "value": 1.0 / step_s, "unit": "steps/s", "cores": torch.get_num_threads(), "kind": "oracle",
        "sample": (f"FP64 oracle forward+autograd backward, all {g['opacity'].shape[0]} Gaussians "
                   f"preprocessed, {p1} and {p2} sampled pixels composited "
                   f"({t1:.1f} s, {t2:.1f} s); full {Wd}x{H} frame extrapolated linearly "
                   f"(fixed {fixed:.2f} s + {per_pixel * 1e3:.1f} ms/pixel)"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the render path is "
              "single-GPU in this build", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2402_03307_amd as r4d
    import workloads as W

    dev = torch.device("cuda:0")
    g, views, st = W.scene_500k_step()
    st = dict(st, tile_size=args.tile_size, fwd_pixels_per_thread=args.fwd_ppt,
              bwd_pixels_per_thread=args.bwd_ppt)
    view = views[0]
    H, Wd = int(view["height"]), int(view["width"])
    n = int(g["opacity"].shape[0])
    params = {k: torch.as_tensor(g[k]).to(dev).contiguous()
              for k in ("means", "log_scales", "rotors", "opacity", "sh")}
    params["sh_degree"] = g["sh_degree"]
    target = torch.as_tensor(W.target_image(H, Wd)).to(dev)
    rend = r4d.Renderer(dev)
    if args.calibration_copy_mib:
        nbytes = args.calibration_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        imgs, saved = rend.forward(params, views, st, save=True)
        _, dl = rend.l1_loss_grad(imgs[0], target)
        rend.backward(params, views, st, saved, [dl])
        saved.release()

    def fwd():
        rend.forward(params, views, st, save=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"timed {args.steps} fwd+bwd steps: {step_ms:.3f} ms/step", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        fwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd()
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(f"timed {args.steps} forward renders: {fwd_ms:.3f} ms/frame", file=sys.stderr,
          flush=True)

    # per-stage kernel times (separate pass: events are recorded around each stage)
    rend.set_timing(True)
    rend.timings(reset=True)
    k_stage = max(3, min(args.steps, 10))
    last_saved = None
    for _ in range(k_stage):
        imgs, saved = rend.forward(params, views, st, save=True)
        _, dl = rend.l1_loss_grad(imgs[0], target)
        rend.backward(params, views, st, saved, [dl])
        if last_saved is not None:
            last_saved.release()
        last_saved = saved
    torch.cuda.synchronize()
    tim = rend.timings(reset=True)
    rend.set_timing(False)
    stats = last_saved.stats(0)
    n_eval = last_saved.copy(0, r4d.BUF_NEVAL, n).to(torch.int64).sum().item()
    n_contrib = last_saved.copy(0, r4d.BUF_NCONTRIB, n).to(torch.int64).sum().item()
    last_saved.release()
    stages = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim.items()}
    print("stage ms: " + ", ".join(f"{k}={v:.3f}" for k, v in stages.items()), file=sys.stderr,
          flush=True)

    n_vis, D = stats["n_visible"], stats["n_dup"]
    k = (g["sh_degree"] + 1) ** 2
    # algorithmic bytes per launch of the HBM-bound stages
    alg_bytes = {
        # params 68 B/Gaussian + per-Gaussian outputs (rect 8, count 4, key 4, index 4)
        # + SH (12k B) and record (48 B) of each visible Gaussian
        "preprocess_fwd": n * (68 + 20) + n_vis * (12 * k + 48),
        # 4 passes x (read + write of 8 B pairs) over all Gaussians
        "depth_sort": 4 * n * 16,
        # 2 passes over D (u32 key, u32 value) pairs, read + write
        "tile_sort": 2 * D * 16,
        "emit": D * 8 + n * 16,
        # params + 9 screen-space gradients read, 17 + 3k gradients written
        "preprocess_bwd": n * (68 + 12 * k) + n * 36 + n * 4 * (17 + 3 * k),
    }
    dominant = max(stages, key=stages.get)
    dom_ms = stages[dominant]
    if dominant in alg_bytes:
        achieved = alg_bytes[dominant] / (dom_ms * 1e-3) / 1e9
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": None}
    else:
        pairs = n_eval if dominant == "raster_fwd" else n_contrib
        achieved = pairs * FLOPS_PER_PAIR_FWD / (dom_ms * 1e-3) / 1e12
        roofline = {"kernel": dominant, "bound": "alu", "achieved": achieved,
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                    "pairs": pairs}
    hbm_stages = {}
    for name, b in alg_bytes.items():
        if stages.get(name):
            gbs = b / (stages[name] * 1e-3) / 1e9
            hbm_stages[name] = {"alg_bytes": b, "ms": stages[name], "GB/s": gbs,
                                "frac": gbs / HBM_PEAK_GBS}

    out = {
        "metric": "frames/s and fwd+bwd steps/s at 500k 4D Gaussians, 1352x1014; batched vs plain",
        "value": 1e3 / step_ms,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "500k 4D Gaussians, SH degree 3, one 1352x1014 render at t=0.5; "
                               "step = forward + L1 grad + backward",
                   "n_gaussians": n, "width": Wd, "height": H, "tile_size": args.tile_size,
                   "fwd_pixels_per_thread": args.fwd_ppt or "auto",
                   "bwd_pixels_per_thread": args.bwd_ppt or "auto",
                   "plain_or_batched": "plain"},
        "fwd_frames_per_s": 1e3 / fwd_ms,
        "fwd_ms": fwd_ms,
        "n_visible": n_vis,
        "n_dup": D,
        "pairs_evaluated_fwd": n_eval,
        "pairs_blended": n_contrib,
        "stage_ms": stages,
        "hbm_stages": hbm_stages,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, view, st, tuple(args.cpu_pixels))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
