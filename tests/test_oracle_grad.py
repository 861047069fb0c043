"""Pin for the oracle's reference gradient: torch autograd through the FP64
oracle versus central finite differences of the oracle's forward, on the
64-Gaussian 32x32 scene (the first 64 Gaussians of the 500k workload).
Parameters whose +-h perturbation flips a discrete decision (a cull, a skip,
the stop rule) are skipped, since the rendered image is only piecewise smooth.
"""
import numpy as np
import torch

import workloads as W
from oracle import render as O

GROUPS = ("means", "log_scales", "rotors", "opacity", "sh")


def _loss_and_sig(g, view, weight):
    out = O.render(g, view, {})
    sig = (out["n_contrib"].numpy().copy(), out["pre"]["valid"].numpy().copy())
    return float((out["image"] * weight).sum()), sig


def test_autograd_matches_central_differences():
    g, views, st = W.scene_fd_subset()
    view = views[0]
    g64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    weight = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, (3, 32, 32)))
    out = O.render(g64, view, st, requires_grad=True)
    (out["image"] * weight).sum().backward()
    grads = {k: out["params"][k].grad.numpy() for k in GROUPS}
    rng = np.random.default_rng(5)
    live = np.nonzero(grads["opacity"])[0]          # Gaussians that reach some pixel
    assert live.size >= 10
    checked = 0
    for key in GROUPS:
        arr = g64[key]
        for gi in rng.choice(live, size=10, replace=False):
            comp = rng.integers(0, arr.shape[0]) if arr.ndim == 2 else None
            idx = (comp, gi) if comp is not None else (gi,)
            theta = arr[idx]
            h = 1e-6 * max(1.0, abs(theta))
            gp = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g64.items()}
            gm = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g64.items()}
            gp[key][idx] = theta + h
            gm[key][idx] = theta - h
            lp, sp = _loss_and_sig(gp, view, weight)
            lm, sm = _loss_and_sig(gm, view, weight)
            if not (np.array_equal(sp[0], sm[0]) and np.array_equal(sp[1], sm[1])):
                continue
            fd = (lp - lm) / (2 * h)
            ad = grads[key][idx]
            scale = max(abs(fd), abs(ad), 1e-6)
            assert abs(fd - ad) <= 1e-5 * scale + 1e-8, (key, idx, fd, ad)
            checked += 1
    assert checked >= 35
