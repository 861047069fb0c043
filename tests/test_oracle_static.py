"""Pins for the oracle's static 3D Gaussians (Sec. 3.2.1, 3D/4D unification).

* the sliced covariance equals R(q) diag(s^2) R(q)^T with the textbook
  quaternion matrix of the normalised quaternion, the sliced mean is mu and the
  sliced opacity is the opacity (no decay);
* the image does not depend on the view's time;
* gradients w.r.t. the 3D parameters match central differences.
"""
import numpy as np
import torch

import workloads as W
from oracle import static3d as S


def static_set(n, deg=0, seed=3):
    rng = np.random.default_rng(seed)
    k = (deg + 1) ** 2
    f = np.float32
    return {"means": rng.uniform(-0.6, 0.6, (3, n)).astype(f),
            "log_scales": rng.normal(-2.8, 0.4, (3, n)).astype(f),
            "quats": rng.normal(size=(4, n)).astype(f),
            "opacity": rng.uniform(0.2, 0.95, n).astype(f),
            "sh": np.concatenate([rng.uniform(0.2, 1.5, (3, n)),
                                  rng.normal(0, 0.1, (3 * k - 3, n))]).astype(f),
            "sh_degree": deg}


def _quat_matrix(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_static_slice_is_the_3d_gaussian():
    g = static_set(40)
    v = W.view((0.0, 0.0, -3.0), 48, 40, 60.0, 0.7)
    out = S.render_static(g, v, {})
    pre = out["pre"]
    for i in range(40):
        R3 = _quat_matrix(g["quats"][:, i].astype(np.float64))
        s2 = np.exp(2 * g["log_scales"][:, i].astype(np.float64))
        cov = R3 @ np.diag(s2) @ R3.T
        assert np.abs(pre["cov3"][i].detach().numpy() - cov).max() < 1e-14 * s2.max() + 1e-18
        assert np.abs(pre["mu3"][i].detach().numpy() - g["means"][:, i]).max() == 0.0
    assert torch.equal(pre["opacity"].detach(), torch.as_tensor(g["opacity"], dtype=torch.float64))


def test_static_render_is_time_independent():
    g = static_set(300, 1)
    a = S.render_static(g, W.view((0.5, -0.3, -3.0), 40, 36, 50.0, 0.0), {})["image"]
    b = S.render_static(g, W.view((0.5, -0.3, -3.0), 40, 36, 50.0, 123.0), {})["image"]
    assert torch.equal(a, b)
    assert float(a.max()) > 0.1


def test_static_gradients_match_central_differences():
    g = static_set(24, 1, seed=4)
    v = W.view((0.0, 0.0, -3.0), 20, 20, 30.0, 0.5)
    wts = torch.as_tensor(np.random.default_rng(5).uniform(-1, 1, (3, 20, 20)))
    out = S.render_static(g, v, {}, requires_grad=True)
    (out["image"] * wts).sum().backward()
    P = out["params"]
    rng = np.random.default_rng(6)
    checked = 0
    for key, rows in (("means", 3), ("log_scales", 3), ("quats", 4), ("opacity", None), ("sh", 12)):
        for _ in range(3):
            i = int(rng.integers(0, 24))
            idx = (int(rng.integers(0, rows)), i) if rows else (i,)
            h = 1e-6

            def val(dv):
                g2 = {k: (np.asarray(vv, dtype=np.float64).copy() if isinstance(vv, np.ndarray) else vv)
                      for k, vv in g.items()}
                g2[key][idx] += dv
                return float((S.render_static(g2, v, {})["image"] * wts).sum())
            fd = (val(h) - val(-h)) / (2 * h)
            ad = float(P[key].grad[idx])
            if abs(fd) > 1e-8:
                checked += 1
            assert abs(ad - fd) <= 1e-5 * max(1.0, abs(fd)), (key, idx, ad, fd)
    assert checked >= 6
