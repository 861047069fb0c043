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
