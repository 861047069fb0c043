"""CPU oracle for static 3D Gaussians (the 3D/4D unification of Sec. 3.2.1: a
rotor whose temporal components vanish acts on space as a quaternion, and a
Gaussian that does not move is its own slice at every time).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

A static Gaussian (mu [3], log-scales [3], quaternion q = (w, x, y, z),
opacity, SH) is rendered as the 4D Gaussian with rotor (w, -z, y, -x, 0, 0, 0,
0) -- whose spatial block is the quaternion's rotation (pinned in the rotor
tests) -- mean (mu, t0) and time log-scale 40, so that the opacity decay
exp(-(t - t0)^2 / (2 W)) rounds to 1 for every t of interest: no decay and no
time cull.  Gradients flow to the 3D parameters through this map.
"""
from __future__ import annotations

import numpy as np
import torch

from . import render as R

STATIC_KEYS = ("means", "log_scales", "quats", "opacity", "sh")
LOG_TIME_SCALE = 40.0


def params3_to_torch(g3: dict, requires_grad: bool = False) -> dict:
    out = {}
    for k in STATIC_KEYS:
        t = torch.as_tensor(np.asarray(g3[k]), dtype=torch.float64).clone()
        if requires_grad:
            t.requires_grad_(True)
        out[k] = t
    out["sh_degree"] = int(g3["sh_degree"])
    return out


def to_4d(P3: dict, t0: float = 0.0) -> dict:
    """The 4D parameters (float64 torch, differentiable) of a static set."""
    n = P3["opacity"].shape[0]
    one = torch.ones(1, n, dtype=torch.float64)
    w, x, y, z = P3["quats"].unbind(0)
    zero = torch.zeros(n, dtype=torch.float64)
    return {"means": torch.cat([P3["means"], t0 * one]),
            "log_scales": torch.cat([P3["log_scales"], LOG_TIME_SCALE * one]),
            "rotors": torch.stack([w, -z, y, -x, zero, zero, zero, zero]),
            "opacity": P3["opacity"], "sh": P3["sh"], "sh_degree": P3["sh_degree"]}


def render_static(g3: dict, view: dict, st: dict | None = None, requires_grad: bool = False,
                  pixels=None):
    """Render of a static set; 'params' holds the float64 3D leaves."""
    P3 = params3_to_torch(g3, requires_grad=requires_grad)
    out = R.render(None, view, st, pixels=pixels, P=to_4d(P3))
    out["params"] = P3
    return out
