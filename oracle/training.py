"""CPU oracle for the optimisation step around the render (Sec. 3.3 "Entropy
Loss"; Sec. 4 "Implementation Details", which defers learning rates, opacity
reset and densification to 3D Gaussian Splatting).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

What is computed (float64 numpy / torch):
  * entropy loss L = (1/N) sum_i -o_i ln o_i over the opacities (Sec. 3.3);
  * Adam (Kingma and Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
  * learning rates per parameter group, the position rate decayed
    exponentially from lr0 to lr1 over `steps` steps:
    lr(t) = exp((1 - u) ln lr0 + u ln lr1), u = min(t / steps, 1);
  * the optimiser keeps opacity as a logit l (o = sigmoid(l)); the render's
    opacity gradient becomes dL/dl = dL/do * o (1 - o);
  * opacity reset: o <- min(o, cap), with the opacity moments cleared.

Readings (listed in the design notes): the parameters the render takes are the
activated opacity and the log-scales, raw rotors, SH and 4D means; the 4D mean
(x, y, z, t) is one position group; SH degree-0 coefficients (rows 0..2 of the
[3k][n] array) and the higher bands have separate rates.
"""
from __future__ import annotations

import math

import numpy as np
import torch

GROUPS = ("means", "log_scales", "rotors", "opacity", "sh")


def entropy_loss(opacity: torch.Tensor) -> torch.Tensor:
    """(1/N) sum -o ln o (FP64, differentiable)."""
    o = opacity.to(torch.float64)
    return (-o * torch.log(o)).mean()


def position_lr(step: int, lr0: float, lr1: float, steps: int) -> float:
    """Exponential interpolation from lr0 (step 0) to lr1 (step >= steps)."""
    u = min(max(step / steps, 0.0), 1.0) if steps > 0 else 1.0
    return math.exp((1.0 - u) * math.log(lr0) + u * math.log(lr1))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def logit(o):
    return np.log(o) - np.log1p(-o)


def group_lr(cfg: dict, group: str, sh_rows: int, step: int) -> np.ndarray | float:
    """Learning rate of a group at `step` (the 1-based step being taken is
    step + 1; the decay is evaluated at the 0-based step), as a scalar or, for
    SH, a per-row column."""
    if group == "means":
        return position_lr(step, cfg["lr_means_init"], cfg["lr_means_final"], cfg["lr_means_steps"])
    if group == "sh":
        col = np.full((sh_rows, 1), cfg["lr_sh_rest"])
        col[:3] = cfg["lr_sh_dc"]
        return col
    return cfg["lr_" + group]


def adam_step(params: dict, opacity_logit: np.ndarray, grads: dict, m: dict, v: dict, step: int,
              cfg: dict):
    """One Adam step in float64 on copies; returns (params, opacity_logit, m, v).

    params: the render's arrays (opacity activated); grads: the render-side
    gradients (w.r.t. the activated opacity); m, v: moments per group (the
    opacity ones in logit space); step: steps already taken (0 before the
    first)."""
    t = step + 1
    b1, b2, eps = cfg["beta1"], cfg["beta2"], cfg["eps"]
    p_out = {k: np.array(params[k], dtype=np.float64, copy=True) for k in GROUPS}
    l_out = np.array(opacity_logit, dtype=np.float64, copy=True)
    m_out = {k: np.array(m[k], dtype=np.float64, copy=True) for k in GROUPS}
    v_out = {k: np.array(v[k], dtype=np.float64, copy=True) for k in GROUPS}
    for k in GROUPS:
        g = np.asarray(grads[k], dtype=np.float64)
        if k == "opacity":
            o = sigmoid(l_out)
            g = g * o * (1.0 - o)
        m_out[k] = b1 * m_out[k] + (1 - b1) * g
        v_out[k] = b2 * v_out[k] + (1 - b2) * g * g
        mh = m_out[k] / (1 - b1 ** t)
        vh = v_out[k] / (1 - b2 ** t)
        lr = group_lr(cfg, k, p_out["sh"].shape[0], step)
        upd = lr * mh / (np.sqrt(vh) + eps)
        if k == "opacity":
            l_out = l_out - upd
            p_out[k] = sigmoid(l_out)
        else:
            p_out[k] = p_out[k] - upd
    return p_out, l_out, m_out, v_out


def opacity_reset(opacity_logit: np.ndarray, m_opacity: np.ndarray, v_opacity: np.ndarray,
                  cap: float):
    """o <- min(o, cap) (as a logit), opacity moments cleared."""
    o = np.minimum(sigmoid(np.asarray(opacity_logit, dtype=np.float64)), cap)
    return logit(o), o, np.zeros_like(m_opacity, dtype=np.float64), np.zeros_like(
        v_opacity, dtype=np.float64)


# ---------------------------------------------------------------------------
# Densification and pruning (the paper applies 3D Gaussian Splatting's
# adaptive density control to its 4D Gaussians, Sec. 4 "Implementation
# Details"): statistics from the screen-space mean gradients, then clone,
# split and prune.


def densify_stat_increment(grad_mean2: np.ndarray, width: int, height: int) -> np.ndarray:
    """Per visible Gaussian: the norm of the gradient w.r.t. its projected mean
    in normalised device coordinates (pixel gradient times (W/2, H/2)).
    grad_mean2: [n, 2] pixel-space gradients."""
    g = np.asarray(grad_mean2, dtype=np.float64)
    return np.sqrt((g[:, 0] * (0.5 * width)) ** 2 + (g[:, 1] * (0.5 * height)) ** 2)


def densify(params: dict, opacity_logit: np.ndarray, m: dict, v: dict, accum: np.ndarray,
            count: np.ndarray, normals: np.ndarray, cfg: dict):
    """Clone, split and prune.  Decisions are taken in float32 (the stored
    precision) exactly as stated here; new positions in float64.

    params: float32 arrays ([C][n] layouts); accum (float32 [n]) / count
    (int [n]): summed NDC gradient norms and visible-render counts; normals:
    [4][2n] standard normal draws (column 2i + c for child c of Gaussian i);
    cfg: grad_threshold, size_threshold (world units), min_opacity,
    max_size (world units, 0 = no size pruning).

    A Gaussian is selected when count > 0 and fl32(accum / count) >=
    grad_threshold.  Selected with max(log s_x, log s_y, log s_z) <=
    fl32(ln size_threshold): cloned (an identical copy with zero moments).
    Selected above it: split into 2 children at mu + R diag(s) z_c (the 4D
    mean, rotation and scales of the Gaussian, z_c its two normal draws), log
    scales minus fl32(ln 1.6), everything else copied, zero moments; the
    parent is removed.  Every resulting Gaussian is then dropped if its
    opacity < min_opacity or (max_size > 0 and its largest spatial log scale >
    fl32(ln max_size)).  Output order: surviving originals, then clones, then
    children (two per split parent), each in index order.  Returns the new
    (params, opacity_logit, m, v)."""
    f32 = np.float32
    n = params["opacity"].shape[0]
    acc = np.asarray(accum, dtype=f32)
    cnt = np.asarray(count)
    with np.errstate(divide="ignore", invalid="ignore"):
        avg = np.where(cnt > 0, acc / np.maximum(cnt, 1).astype(f32), f32(0)).astype(f32)
    selected = (cnt > 0) & (avg >= f32(cfg["grad_threshold"]))
    ls = np.asarray(params["log_scales"], dtype=f32)
    max_ls = ls[:3].max(axis=0)
    small = max_ls <= f32(math.log(cfg["size_threshold"]))
    clone = selected & small
    split = selected & ~small
    op = np.asarray(params["opacity"], dtype=f32)
    min_op = f32(cfg["min_opacity"])
    big_log = f32(math.log(cfg["max_size"])) if cfg["max_size"] > 0 else None
    shrink = f32(math.log(1.6))

    def survives(o, max_log_scale):
        ok = ~(o < min_op)
        if big_log is not None:
            ok &= ~(max_log_scale > big_log)
        return ok

    keep = ~split & survives(op, max_ls)
    clone_ok = clone & survives(op, max_ls)
    child_ls = (ls - shrink).astype(f32)
    child_ok = split & survives(op, child_ls[:3].max(axis=0))
    ids_keep = np.nonzero(keep)[0]
    ids_clone = np.nonzero(clone_ok)[0]
    ids_split = np.nonzero(child_ok)[0]
    # children positions: mu + R diag(s) z, in float64 from the stored values
    r = torch.as_tensor(np.asarray(params["rotors"], dtype=np.float64)[:, ids_split].T)
    from . import render as Rn
    R = Rn.rotor_to_matrix(Rn.rotor_normalize(r)).numpy() if ids_split.size else np.zeros((0, 4, 4))
    s = np.exp(ls[:, ids_split].astype(np.float64))
    mu = np.asarray(params["means"], dtype=np.float64)[:, ids_split]
    children_mu = []
    for c in range(2):
        z = np.asarray(normals, dtype=np.float64)[:, 2 * ids_split + c]
        children_mu.append(mu + np.einsum("nij,jn->in", R, s * z))
    out, out_m, out_v = {}, {}, {}
    for k in GROUPS:
        a = np.asarray(params[k])
        cols = [a[..., ids_keep], a[..., ids_clone]]
        if k == "means":
            ch = np.stack(children_mu, axis=-1).reshape(4, -1)   # child 0, 1 of each parent
            cols.append(ch.astype(f32))
        elif k == "log_scales":
            cols.append(np.repeat(child_ls[:, ids_split], 2, axis=1))
        else:
            cols.append(np.repeat(a[..., ids_split], 2, axis=-1))
        out[k] = np.concatenate(cols, axis=-1).astype(f32)
        zeros = np.zeros(a.shape[:-1] + (ids_clone.size + 2 * ids_split.size,))
        out_m[k] = np.concatenate([np.asarray(m[k])[..., ids_keep], zeros], axis=-1)
        out_v[k] = np.concatenate([np.asarray(v[k])[..., ids_keep], zeros], axis=-1)
    lg = np.asarray(opacity_logit)
    out_l = np.concatenate([lg[ids_keep], lg[ids_clone], np.repeat(lg[ids_split], 2)])
    return out, out_l, out_m, out_v
