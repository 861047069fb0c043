"""Benchmark: forward frames/s and forward+backward steps/s of the 4D-rotor
Gaussian render path on one MI355X, plain and batched.

Headline workload: 500,000 4D Gaussians, SH degree 3, one 1352x1014 render at
t = 0.5 from (0, 0, -4); a step = forward render + L1 loss gradient against a
seeded U[0,1] target + backward to all Gaussian parameters.  The headline value
is the step rate of the graph mode (the launch sequence captured once in a HIP
graph and replayed, no host synchronisation); the plain mode (one entry-count
readback per render) is reported beside it.

Batched vs plain: 200,000 Gaussians, 16 renders of mixed resolution, each
step forward + L1 + backward of all 16 renders, once as 16 plain per-render
call sequences and once as one graph-mode call over the 16 renders (tile 16,
and with the autotuned tile size / sort chunking).

Speed field: the headline workload rendered with its 2D flow images (the
projected speed of each Gaussian's sliced mean, composited with the colour
weights) in the same pass, forward + colour and flow L1 + backward.

4D consistency loss (Sec. 3.3) of the headline Gaussian set: the exact 4D KNN
(K = 8) and the loss with its gradient.  A whole optimisation step of the
headline workload: render step, entropy and consistency terms, fused Adam.
A static scene: 500k static 3D Gaussians (no time dimension) through the
static path at the headline camera and resolution.

Further lines (per_config): 2,000 Gaussians at 128x128 (forward), 300,000
Gaussians over 30 orbit renders (forward), 3,000,000 Gaussians over 16
renders (graph-mode forward + backward).

Inputs are seeded synthetic arrays resident in HBM before timing starts.
Prints one JSON line.  Per-stage kernel times come from HIP events the
library records on the stream it launches on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# FP32 FMA issue rate without packed dual-FP32 instructions (this build disables
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.  The published 157.3
# TFLOP/s counts the packed form.
FP32_VECTOR_PEAK_TFLOPS = 78.6

# Arithmetic of the compositing loops, counted per (pixel, Gaussian) pair as
# the algorithm needs it (fma = 2, exp2 / rcp / min / compare = 1; the lane
# reductions, ballots and masks of the kernels are not counted).
# Forward, every evaluated pair: offset (2), whitened offset (6), exponent (3),
# exp2, opacity product, clamp, the extent/alpha test, transmittance product
# (2) and the T_min test = 18; every blended pair adds its weight (1) and the
# colour accumulation (3 fma = 6) = 7.
FLOPS_PER_EVAL_FWD = 18
FLOPS_PER_BLEND_FWD = 7
# Backward, every pair up to the pixel's last contributor: the forward
# evaluation = 15; every blended pair: 1 / (1 - a) (2), transmittance in front
# (1), weight (1), g . colour (5), dL/da (3), colour-behind update (2), the
# alpha-weighted gradient (1), the two offset products (2) and the nine moment
# sums (2 adds + 7 fma = 16) = 33.
FLOPS_PER_WALK_BWD = 15
FLOPS_PER_BLEND_BWD = 33


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
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched and per-config measurements")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched-vs-plain measurement (for profiling it)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a kernel of "
                         "known traffic, to scale hardware byte counters)")
    ap.add_argument("--cpu-pixels", type=int, nargs=2, default=(512, 2048),
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
    try:
        host_cores = len(os.sched_getaffinity(0))
    except AttributeError:
        host_cores = os.cpu_count()
    return {
        "value": 1.0 / step_s, "unit": "steps/s", "cores": torch.get_num_threads(),
        "host_cores": host_cores, "kind": "oracle",
        "sample": (f"FP64 oracle forward+autograd backward, all {g['opacity'].shape[0]} Gaussians "
                   f"preprocessed, {p1} and {p2} sampled pixels composited "
                   f"({t1:.1f} s, {t2:.1f} s); full {Wd}x{H} frame extrapolated linearly "
                   f"(fixed {fixed:.2f} s + {per_pixel * 1e3:.2f} ms/pixel)"),
    }


def device_params(g, dev):
    import torch
    p = {k: torch.as_tensor(g[k]).to(dev).contiguous()
         for k in ("means", "log_scales", "rotors", "opacity", "sh")}
    p["sh_degree"] = g["sh_degree"]
    return p


def timed(fn, steps, warmup):
    """Mean wall time per call of fn over `steps` calls after `warmup`, with the
    device synchronised on both sides."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


class Stepper:
    """forward + L1 + backward of a list of renders in one mode."""

    def __init__(self, r4d, rend, params, views, st, targets_flat):
        import torch
        self.r4d, self.rend, self.p, self.views, self.st = r4d, rend, params, views, st
        self.targets = targets_flat
        self.graph = st.get("mode") == "graph"
        self.grad = torch.empty_like(targets_flat)
        self.last = None

    def step(self):
        imgs, saved = self.rend.forward(self.p, self.views, self.st, save=True, flat=True)
        _, dl = self.rend.l1_loss_grad_views(imgs, self.targets, self.views, self.grad)
        self.rend.backward(self.p, self.views, self.st, saved, dl)
        if self.last is not None and not self.graph:
            self.last.release()
        self.last = saved

    def forward(self):
        self.rend.forward(self.p, self.views, self.st, save=False, flat=True)

    def check(self):
        if self.last is not None:
            self.last.check()


class FlowStepper:
    """forward + losses + backward of the speed-field render: colour L1 against
    the targets and L1 of the flow images against zero flow."""

    def __init__(self, r4d, rend, params, views, st, targets_flat):
        import torch
        self.rend, self.p, self.views, self.st = rend, params, views, st
        self.targets = targets_flat
        self.graph = st.get("mode") == "graph"
        self.grad = torch.empty_like(targets_flat)
        nflow = targets_flat.numel() // 3 * 2
        self.zero_flow = torch.zeros(nflow, dtype=targets_flat.dtype, device=targets_flat.device)
        self.grad_flow = torch.empty_like(self.zero_flow)
        self.last = None

    def step(self):
        imgs, flows, saved = self.rend.forward(self.p, self.views, self.st, save=True, flat=True,
                                               flow=True)
        _, dl = self.rend.l1_loss_grad_views(imgs, self.targets, self.views, self.grad)
        _, dlf = self.rend.l1_loss_grad(flows, self.zero_flow, self.grad_flow)
        self.rend.backward(self.p, self.views, self.st, saved, dl, dlf)
        if self.last is not None and not self.graph:
            self.last.release()
        self.last = saved

    def forward(self):
        self.rend.forward(self.p, self.views, self.st, save=False, flat=True, flow=True)

    def check(self):
        if self.last is not None:
            self.last.check()


def flow_render(r4d, rend, params, views, st, args):
    """The speed-field (optical flow) render of the headline workload: colour and
    flow images in one pass, step = forward + colour L1 + flow L1 + backward;
    graph mode, plus per-stage times of the plain mode."""
    import torch
    targets = flat_targets(views, params["means"].device)
    s = FlowStepper(r4d, rend, params, views, dict(st, mode="graph"), targets)
    step_ms = timed(s.step, args.steps, args.warmup)
    s.check()
    fwd_ms = timed(s.forward, args.steps, args.warmup)
    del s
    plain = FlowStepper(r4d, rend, params, views, dict(st, mode="per_view"), targets)
    rend.set_timing(True)
    rend.timings(reset=True)
    for _ in range(max(3, min(args.steps, 10))):
        plain.step()
    torch.cuda.synchronize()
    tim = rend.timings(reset=True)
    rend.set_timing(False)
    plain.last.release()
    res = {"workload": "the headline workload rendered with its speed field: colour + 2-channel "
                       "flow images; step = forward + colour L1 + flow L1 + backward; graph mode",
           "ms_per_step": step_ms, "steps_per_s": 1e3 / step_ms, "fwd_ms": fwd_ms,
           "fwd_frames_per_s": 1e3 / fwd_ms,
           "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim.items()}}
    print(f"flow render: {res}", file=sys.stderr, flush=True)
    return res


def consistency4d(r4d, rend, params, args):
    """4D consistency loss of the headline Gaussian set (Sec. 3.3): the 4D KNN
    (K = 8, unit scene scales) and the loss with its gradient."""
    import torch
    n = int(params["means"].shape[1])
    k = 8
    nb = rend.knn4d(params["means"], k)
    grads = {key: torch.zeros_like(params[key]) for key in ("rotors", "log_scales")}
    knn_ms = timed(lambda: rend.knn4d(params["means"], k), args.steps, args.warmup)
    loss_ms = timed(lambda: rend.consistency4d(params, nb, 0.05, grads), args.steps, args.warmup)
    # algorithmic bytes of the loss + gradient: speeds (48 B parameters in, 16 B
    # out), the pass over the neighbour lists (4k B indices, 16(k + 1) B speeds,
    # 4 B signs, 12 B atomics per neighbour), the gradient (48 B parameters and
    # 16 B signs/sums in, 48 B gradients read and written twice)
    alg = n * (64 + 4 * k + 16 * (k + 1) + 4 + 12 * k + 64 + 96)
    res = {"workload": "500k 4D Gaussians (the headline set): KNN with K = 8 in 4D (unit "
                       "scales), then the 4D consistency loss and its gradient",
           "n": n, "k": k, "knn_ms": knn_ms, "knn_points_per_s": n / (knn_ms * 1e-3),
           "loss_grad_ms": loss_ms,
           "loss_grad_hbm": {"alg_bytes": alg, "GB/s": alg / (loss_ms * 1e-3) / 1e9,
                             "frac": alg / (loss_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    print(f"consistency4d: {res}", file=sys.stderr, flush=True)
    return res


def training_step(r4d, rend, params, views, st, args):
    """One whole optimisation step of the headline workload on a copy of the
    parameters: graph-mode render forward + L1 + backward, the entropy and 4D
    consistency terms added to the gradients (lambda_2 = 0.01, lambda_3 = 0.05,
    neighbours from one 4D KNN), and the fused Adam update."""
    import torch
    p = {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in params.items()}
    targets = flat_targets(views, p["means"].device)
    state = r4d.TrainState(p)
    nb = rend.knn4d(p["means"], 8)
    sg = dict(st, mode="graph")
    grad_img = torch.empty_like(targets)
    box = {}

    def step():
        imgs, saved = rend.forward(p, views, sg, save=True, flat=True)
        _, dl = rend.l1_loss_grad_views(imgs, targets, views, grad_img)
        grads = rend.backward(p, views, sg, saved, dl)
        rend.entropy_loss_grad(p["opacity"], 0.01, grads["opacity"])
        rend.consistency4d(p, nb, 0.05, grads)
        rend.adam_step(state, grads, None)
        box["grads"] = grads

    ms = timed(step, args.steps, args.warmup)
    grads = box["grads"]
    adam_ms = timed(lambda: rend.adam_step(state, grads, None), args.steps, args.warmup)
    total = sum(p[k].numel() for k in ("means", "log_scales", "rotors", "opacity", "sh"))
    alg = total * 28  # parameter, gradient, two moments read; parameter, two moments written
    res = {"workload": "the headline workload: one optimisation step (graph render fwd + L1 + "
                       "bwd, entropy 0.01, 4D consistency 0.05 with fixed K = 8 lists, fused "
                       "Adam of all 65 floats per Gaussian)",
           "ms_per_step": ms, "steps_per_s": 1e3 / ms, "adam_ms": adam_ms,
           "adam_hbm": {"alg_bytes": alg, "GB/s": alg / (adam_ms * 1e-3) / 1e9,
                        "frac": alg / (adam_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    print(f"training step: {res}", file=sys.stderr, flush=True)
    del state, p
    return res


def static_scene(r4d, rend, dev, st, args):
    """Static 3D Gaussians (the 3D/4D unification): 500k static Gaussians, SH 3,
    the headline camera and resolution; graph-mode forward + L1 + backward, and
    the preprocess stage times of the plain mode."""
    import torch

    import workloads as W
    g, views, _ = W.scene_static_500k()
    p = {k: torch.as_tensor(g[k]).to(dev).contiguous()
         for k in ("means", "log_scales", "quats", "opacity", "sh")}
    p["sh_degree"] = g["sh_degree"]
    targets = flat_targets(views, dev)
    grad = torch.empty_like(targets)
    sg = dict(st, mode="graph")

    def step(s_):
        imgs, saved = rend.forward_static(p, views, s_, save=True, flat=True)
        _, dl = rend.l1_loss_grad_views(imgs, targets, views, grad)
        rend.backward_static(p, views, s_, saved, dl)
        if s_.get("mode") != "graph":
            saved.release()

    ms = timed(lambda: step(sg), args.steps, args.warmup)
    fwd_ms = timed(lambda: rend.forward_static(p, views, sg, save=False, flat=True), args.steps,
                   args.warmup)
    rend.set_timing(True)
    rend.timings(reset=True)
    for _ in range(max(3, min(args.steps, 10))):
        step(dict(st, mode="per_view"))
    torch.cuda.synchronize()
    tim = rend.timings(reset=True)
    rend.set_timing(False)
    # the same Gaussians through the 4D path (rotors (w, -z, y, -x, 0, 0, 0, 0),
    # time log-scale 40): what the fast path saves
    q = p["quats"]
    n = q.shape[1]
    zero = torch.zeros(n, device=dev)
    p4 = {"means": torch.cat([p["means"], torch.full((1, n), 0.5, device=dev)]).contiguous(),
          "log_scales": torch.cat([p["log_scales"], torch.full((1, n), 40.0, device=dev)]).contiguous(),
          "rotors": torch.stack([q[0], -q[3], q[2], -q[1], zero, zero, zero, zero]).contiguous(),
          "opacity": p["opacity"], "sh": p["sh"], "sh_degree": p["sh_degree"]}
    s4 = Stepper(r4d, rend, p4, views, sg, targets)
    ms4 = timed(s4.step, args.steps, args.warmup)
    del s4
    rend.set_timing(True)
    rend.timings(reset=True)
    plain4 = Stepper(r4d, rend, p4, views, dict(st, mode="per_view"), targets)
    for _ in range(max(3, min(args.steps, 10))):
        plain4.step()
    torch.cuda.synchronize()
    tim4 = rend.timings(reset=True)
    rend.set_timing(False)
    plain4.last.release()
    del plain4, p4
    res = {"workload": "500k static 3D Gaussians, SH degree 3, one 1352x1014 render; step = "
                       "forward + L1 + backward; graph mode",
           "ms_per_step": ms, "steps_per_s": 1e3 / ms, "fwd_ms": fwd_ms,
           "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim.items()},
           "same_set_via_4d_path": {
               "ms_per_step": ms4,
               "stage_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim4.items()}}}
    print(f"static scene: {res}", file=sys.stderr, flush=True)
    del p
    return res


def per_view_step(r4d, rend, params, views, st, targets):
    """The plain baseline: one call sequence per render."""
    saved_all = []
    grads = []

    def step():
        for v, tgt in zip(views, targets):
            imgs, saved = rend.forward(params, [v], st, save=True, flat=True)
            _, dl = rend.l1_loss_grad(imgs, tgt)
            grads.append(rend.backward(params, [v], st, saved, dl))
            saved.release()
        grads.clear()

    return step


def flat_targets(views, dev):
    import torch

    import workloads as W
    return torch.cat([torch.as_tensor(W.target_image(int(v["height"]), int(v["width"]))).reshape(-1)
                      for v in views]).to(dev)


def kernel_source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2402_03307_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stage_alg_bytes(n, k, renders, packed=True):
    """Algorithmic HBM bytes per launch of the memory-bound stages of one run.
    n Gaussians, k SH coefficients per channel; renders: (visible Gaussians,
    tile entries emitted and sorted (the front lists), tiles) of each render in
    the run.  Every render reads the
    parameters once; the preprocess backward reads them once for the run."""
    V = len(renders)
    vis = sum(r[0] for r in renders)
    D = sum(r[1] for r in renders)
    tiles = sum(r[2] for r in renders)
    return {
        # params 68 B/Gaussian + per-Gaussian outputs (box 8, count 4, key 4)
        # + SH (12k B), record (48 B) and compacted key/index (8 B) of each visible one
        "preprocess_fwd": V * n * (68 + 16) + vis * (12 * k + 48 + 8),
        # visible keys only: 4 passes x (read + write of 8 B key/index pairs) + histogram
        "depth_sort": vis * (4 * 16 + 4),
        # order + gathered count read, 8 B offset written per Gaussian
        "count_scan": V * (n * 4 * 2 + n * 8),
        # per visible Gaussian order 4 + offset 8 + box 8 + record 32 B read; per
        # entry the packed word + low tile byte (5 B) or the (tile, index) pair (8 B)
        "emit": vis * 52 + D * (5 if packed else 8),
        # low pass (5 in, 5 out) + high byte count (1) + high pass (5 in; index 4
        # + 16-bit tile 2 out) per entry, the emission's low byte counts aside
        "tile_sort": D * 22,
        # sorted 16-bit tile ids read; ranges written, and cleared by the preprocess
        "tile_ranges": D * 2 + tiles * 16,
        # params + screen-space gradients (9 doubles per render) read, 17 + 3k
        # gradients written
        "preprocess_bwd": n * (68 + 12 * k) + V * n * 72 + n * 4 * (17 + 3 * k),
    }


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    it was taken from the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"kernel sources sha256\[:16\]: (\w+)", text)
    m_b = re.search(r"hbm bytes per launch: (\d+)", text)
    if not m_src or not m_b or m_src.group(1) != kernel_source_digest():
        return None
    return int(m_b.group(1))


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
    if args.only_batched:
        rend = r4d.Renderer(dev)
        print(json.dumps({"batched_vs_plain": batched_vs_plain(r4d, rend, dev, args)}), flush=True)
        return
    g, views, st = W.scene_500k_step()
    st = dict(st, tile_size=args.tile_size, fwd_pixels_per_thread=args.fwd_ppt,
              bwd_pixels_per_thread=args.bwd_ppt)
    view = views[0]
    H, Wd = int(view["height"]), int(view["width"])
    n = int(g["opacity"].shape[0])
    params = device_params(g, dev)
    targets = flat_targets(views, dev)
    rend = r4d.Renderer(dev)
    if args.calibration_copy_mib:
        nbytes = args.calibration_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- headline: graph mode; plain beside it
    graph = Stepper(r4d, rend, params, views, dict(st, mode="graph"), targets)
    plain = Stepper(r4d, rend, params, views, dict(st, mode="per_view"), targets)
    step_ms = timed(graph.step, args.steps, args.warmup)
    graph.check()
    print(f"graph mode: {args.steps} fwd+bwd steps: {step_ms:.3f} ms/step", file=sys.stderr,
          flush=True)
    fwd_ms = timed(graph.forward, args.steps, args.warmup)
    plain_step_ms = timed(plain.step, args.steps, args.warmup)
    plain_fwd_ms = timed(plain.forward, args.steps, args.warmup)
    print(f"graph fwd {fwd_ms:.3f} ms; plain step {plain_step_ms:.3f} ms, plain fwd "
          f"{plain_fwd_ms:.3f} ms", file=sys.stderr, flush=True)

    # ---- per-stage kernel times (plain mode, events around each stage)
    rend.set_timing(True)
    rend.timings(reset=True)
    k_stage = max(3, min(args.steps, 10))
    last_saved = None
    for _ in range(k_stage):
        imgs, saved = rend.forward(params, views, st, save=True)
        _, dl = rend.l1_loss_grad(imgs[0], targets.view(3, H, Wd))
        rend.backward(params, views, st, saved, [dl])
        if last_saved is not None:
            last_saved.release()
        last_saved = saved
    torch.cuda.synchronize()
    tim = rend.timings(reset=True)
    rend.set_timing(False)
    stats = last_saved.stats(0)
    n_eval = last_saved.copy(0, r4d.BUF_NEVAL, n).to(torch.int64).sum().item()
    n_blend = last_saved.copy(0, r4d.BUF_NBLEND, n).to(torch.int64).sum().item()
    n_contrib = last_saved.copy(0, r4d.BUF_NCONTRIB, n).to(torch.int64).sum().item()
    last_saved.release()
    stages = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tim.items()}
    print("stage ms: " + ", ".join(f"{k}={v:.3f}" for k, v in stages.items()), file=sys.stderr,
          flush=True)

    n_vis, D, D_front = stats["n_visible"], stats["n_dup"], stats["n_front"]
    k = (g["sh_degree"] + 1) ** 2
    tiles = stats["tiles_x"] * stats["tiles_y"]
    # the binning stages emit and sort the front lists (D_front entries)
    alg_bytes = stage_alg_bytes(n, k, [(n_vis, D_front, tiles)])
    dominant = max(stages, key=stages.get)
    dom_ms = stages[dominant]
    workload = "500k_1352x1014_tile16"
    traffic = measured_traffic(dominant, workload)
    if dominant in alg_bytes:
        achieved = alg_bytes[dominant] / (dom_ms * 1e-3) / 1e9
        roofline = {"kernel": dominant, "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": traffic}
    else:
        fwd = dominant == "raster_fwd"
        flops = (n_eval * FLOPS_PER_EVAL_FWD + n_blend * FLOPS_PER_BLEND_FWD if fwd else
                 n_contrib * FLOPS_PER_WALK_BWD + n_blend * FLOPS_PER_BLEND_BWD)
        achieved = flops / (dom_ms * 1e-3) / 1e12
        roofline = {"kernel": dominant, "bound": "alu", "achieved": achieved,
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                    "flops": flops}
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
                               "step = forward + L1 grad + backward; graph mode",
                   "n_gaussians": n, "width": Wd, "height": H, "tile_size": args.tile_size,
                   "fwd_pixels_per_thread": args.fwd_ppt or "auto",
                   "bwd_pixels_per_thread": args.bwd_ppt or "auto"},
        "fwd_frames_per_s": 1e3 / fwd_ms,
        "fwd_ms": fwd_ms,
        "plain": {"steps_per_s": 1e3 / plain_step_ms, "ms_per_step": plain_step_ms,
                  "fwd_frames_per_s": 1e3 / plain_fwd_ms, "fwd_ms": plain_fwd_ms},
        "n_visible": n_vis,
        "n_dup": D,
        "front_lists": {"entries": D_front, "rest_tiles": stats["rest_tiles"],
                        "rest_entries": stats["rest_entries"]},
        "pairs_evaluated_fwd": n_eval,
        "pairs_walked_bwd": n_contrib,
        "pairs_blended": n_blend,
        "raster_tflops": {
            "raster_fwd": (n_eval * FLOPS_PER_EVAL_FWD + n_blend * FLOPS_PER_BLEND_FWD)
            / (stages["raster_fwd"] * 1e-3) / 1e12,
            "raster_bwd": (n_contrib * FLOPS_PER_WALK_BWD + n_blend * FLOPS_PER_BLEND_BWD)
            / (stages["raster_bwd"] * 1e-3) / 1e12},
        "stage_ms": stages,
        "hbm_stages": hbm_stages,
        "roofline": roofline,
    }
    del graph, plain

    if not args.no_extra:
        out["flow_render"] = flow_render(r4d, rend, params, views, st, args)
        out["consistency4d"] = consistency4d(r4d, rend, params, args)
        out["training_step"] = training_step(r4d, rend, params, views, st, args)
        out["static_scene"] = static_scene(r4d, rend, dev, st, args)
        out["batched_vs_plain"] = batched_vs_plain(r4d, rend, dev, args)
        out["per_config"] = per_config(r4d, rend, dev, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, view, st, tuple(args.cpu_pixels))
    print(json.dumps(out), flush=True)


def batched_vs_plain(r4d, rend, dev, args):
    import torch

    import workloads as W
    g, views, st = W.scene_200k_batch()
    params = device_params(g, dev)
    targets = flat_targets(views, dev)
    sizes = [3 * int(v["height"]) * int(v["width"]) for v in views]
    tlist = list(torch.split(targets, sizes))
    steps = max(3, args.steps // 2)
    plain_ms = timed(per_view_step(r4d, rend, params, views, dict(st, mode="per_view"), tlist),
                     steps, 2)
    res = {"workload": "200k 4D Gaussians, SH 3, 16 renders (random cameras on the radius-4 "
                       "sphere, t ~ U[0,1], resolutions from {800x800, 1014x1352, 1352x1014, "
                       "960x540}); step = forward + L1 + backward of all 16",
           "plain_ms_per_step": plain_ms, "renders": len(views)}
    for label, ts in (("batched", 16), ("batched_autotuned", 0)):
        s = Stepper(r4d, rend, params, views, dict(st, mode="graph", tile_size=ts), targets)
        ms = timed(s.step, steps, 2)
        s.check()
        cfg = s.last.config()
        res[f"{label}_ms_per_step"] = ms
        res[f"{label}_speedup"] = plain_ms / ms
        res[f"{label}_tile_size"] = cfg["tile_size"]
        res[f"{label}_sort_items"] = cfg["sort_items"]
        res[f"{label}_renders_per_s"] = len(views) * 1e3 / ms
        del s
    print(f"batched vs plain: {res}", file=sys.stderr, flush=True)
    return res


def per_config(r4d, rend, dev, args):
    import torch

    import workloads as W
    res = {}
    # 2k Gaussians, 128x128, forward only
    g, views, st = W.scene_2k()
    p = device_params(g, dev)
    ms = timed(lambda: rend.forward(p, views, dict(st, mode="graph"), save=False), args.steps,
               args.warmup)
    res["2k_128x128_fwd"] = {"fwd_ms": ms, "frames_per_s": 1e3 / ms, "mode": "graph"}
    # 300k Gaussians, 30 orbit renders, forward
    g, views, st = W.scene_300k_orbit()
    p = device_params(g, dev)
    steps = max(2, args.steps // 4)
    ms_plain = timed(lambda: rend.forward(p, views, dict(st, mode="per_view"), save=False,
                                          flat=True), steps, 1)
    ms_graph = timed(lambda: rend.forward(p, views, dict(st, mode="graph"), save=False, flat=True),
                     steps, 1)
    _, saved = rend.forward(p, views, dict(st, mode="graph"), save=True)
    so = [saved.stats(v) for v in range(len(views))]
    saved.release()
    res["300k_30_orbit_fwd"] = {"plain_ms_per_30": ms_plain, "graph_ms_per_30": ms_graph,
                                "plain_frames_per_s": 30e3 / ms_plain,
                                "graph_frames_per_s": 30e3 / ms_graph,
                                "tile_entries_total": sum(x["n_dup"] for x in so),
                                "front_entries_total": sum(x["n_front"] for x in so),
                                "rest_tiles_total": sum(x["rest_tiles"] for x in so)}
    del p
    torch.cuda.empty_cache()
    print(f"per config (so far): {res}", file=sys.stderr, flush=True)
    # 3M Gaussians, 16 renders, graph-mode forward + backward
    g, views, st = W.scene_3m_large()
    p = device_params(g, dev)
    targets = flat_targets(views, dev)
    s = Stepper(r4d, rend, p, views, dict(st, mode="graph"), targets)
    ms = timed(s.step, 3, 1)
    s.check()
    st3 = [s.last.stats(v) for v in range(len(views))]
    res["3m_16_renders_fwd_bwd"] = {"graph_ms_per_step": ms, "renders_per_s": 16e3 / ms,
                                    "tile_entries_total": sum(x["n_dup"] for x in st3),
                                    "front_entries_total": sum(x["n_front"] for x in st3),
                                    "rest_tiles_total": sum(x["rest_tiles"] for x in st3)}
    # per-stage times of the same step in fused mode (one launch per stage over
    # all 16 renders), and the memory-bound stages' share of HBM peak
    fused = Stepper(r4d, rend, p, views, dict(st, mode="fused"), targets)
    fused.step()
    rend.set_timing(True)
    rend.timings(reset=True)
    for _ in range(3):
        fused.step()
    torch.cuda.synchronize()
    tim = rend.timings(reset=True)
    rend.set_timing(False)
    stages = {k_: (v[0] / v[1] if v[1] else 0.0) for k_, v in tim.items()}
    renders = []
    for v in range(len(views)):
        sv = fused.last.stats(v)
        renders.append((sv["n_visible"], sv["n_front"], sv["tiles_x"] * sv["tiles_y"]))
    fused.last.release()
    alg = stage_alg_bytes(int(g["opacity"].shape[0]), (g["sh_degree"] + 1) ** 2, renders)
    hbm = {}
    for name, b in alg.items():
        if stages.get(name):
            gbs = b / (stages[name] * 1e-3) / 1e9
            hbm[name] = {"alg_bytes": b, "ms": stages[name], "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    res["3m_16_renders_fwd_bwd"].update({"fused_stage_ms": stages, "hbm_stages": hbm,
                                         "visible_total": sum(r[0] for r in renders)})
    del s, p
    torch.cuda.empty_cache()
    print(f"per config: {res}", file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
