"""Static 3D Gaussians (the 3D/4D unification, Sec. 3.2.1) on the GPU against
the CPU oracle, and against the GPU's own 4D path on the equivalent rotors.

Tolerances as for the 4D render: images 1e-4 on unambiguous pixels; gradients
per group relative 1e-3 (elementwise like the render); the float64
instantiation against central differences of its own forward; the static path
against the 4D path of the same Gaussians (rotor (w, -z, y, -x, 0, 0, 0, 0),
time log-scale 40): images within 2e-5 (two float32 routes to one covariance).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import static3d as S

from helpers import image_errors

pytestmark = pytest.mark.gpu

KEYS = ("means", "log_scales", "quats", "opacity", "sh")


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


@pytest.fixture(scope="module")
def rend(r4d, device):
    return r4d.Renderer(device)


def to_dev(g, device, dtype=torch.float32):
    out = {k: torch.as_tensor(np.asarray(g[k])).to(device=device, dtype=dtype).contiguous()
           for k in KEYS}
    out["sh_degree"] = g["sh_degree"]
    return out


def test_static_image_matches_oracle(rend, device):
    g = W.static_gaussians(2000, 0)
    v = W.view((0.0, 0.0, -4.0), 128, 112, 150.0, 0.5)
    print("case: static 2k 128x112", flush=True)
    ref = S.render_static(g, v, W.settings())
    imgs, _ = rend.forward_static(to_dev(g, device), [v], W.settings())
    err, n_amb = image_errors(imgs[0].cpu().numpy().astype(np.float64), ref["image"].numpy(),
                              ref["ambiguous"].numpy())
    print(f"max err {err:.3g}, ambiguous {n_amb}")
    assert n_amb <= 0.01 * 128 * 112
    assert err <= 1e-4


def test_static_gradients_match_oracle(rend, device):
    g = W.subset(W.static_gaussians(5000, 3), 64)
    v = W.view((0.0, 0.0, -4.0), 32, 32, 40.0, 0.5)
    w = np.random.default_rng(2).uniform(-1, 1, (3, 32, 32))
    ref = S.render_static(g, v, W.settings(), requires_grad=True)
    (ref["image"] * torch.as_tensor(w)).sum().backward()
    p = to_dev(g, device)
    imgs, saved = rend.forward_static(p, [v], W.settings())
    err, _ = image_errors(imgs[0].cpu().numpy().astype(np.float64), ref["image"].detach().numpy(),
                          ref["ambiguous"].numpy())
    assert err <= 1e-4
    grads = rend.backward_static(p, [v], W.settings(), saved,
                                 [torch.as_tensor(w, dtype=torch.float32, device=device)])
    for k in KEYS:
        gg = grads[k].cpu().numpy().astype(np.float64)
        gr = ref["params"][k].grad.numpy()
        rel = float(np.linalg.norm(gg - gr) / max(np.linalg.norm(gr), 1e-30))
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-3, k
        assert np.all(np.abs(gg - gr) <= 1e-3 * (np.abs(gr) + 1e-2 * np.abs(gr).max()) + 1e-7), k


def test_static_fp64_gradients_match_central_differences(rend, device):
    g = W.subset(W.static_gaussians(5000, 3), 64)
    g64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    v = W.view((0.0, 0.0, -4.0), 32, 32, 40.0, 0.5)
    w = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, (3, 32, 32)), dtype=torch.float64,
                        device=device)
    p = to_dev(g64, device, torch.float64)
    _, saved = rend.forward_static(p, [v], W.settings())
    grads = {k: t.cpu().numpy() for k, t in rend.backward_static(p, [v], W.settings(), saved, [w]).items()}
    live = np.nonzero(grads["opacity"])[0]
    assert live.size >= 10
    rng = np.random.default_rng(5)
    checked = 0

    def loss_and_sig(pp):
        im, sv = rend.forward_static(pp, [v], W.settings())
        return float((im[0] * w).sum()), sv.copy(0, 6, 0).cpu().numpy()

    for key in KEYS:
        arr = g64[key]
        for gi in rng.choice(live, size=6, replace=False):
            idx = (int(rng.integers(0, arr.shape[0])), gi) if arr.ndim == 2 else (gi,)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            vals, sigs = [], []
            for sgn in (1, -1):
                q = {k: (t.copy() if isinstance(t, np.ndarray) else t) for k, t in g64.items()}
                q[key][idx] += sgn * h
                lv, sg = loss_and_sig(to_dev(q, device, torch.float64))
                vals.append(lv)
                sigs.append(sg)
            if not np.array_equal(sigs[0], sigs[1]):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grads[key][idx]) <= 1e-5 * max(abs(fd), abs(grads[key][idx]), 1e-3), (key, idx)
            checked += 1
    assert checked >= 20


def test_static_path_equals_4d_path_and_is_time_independent(rend, device):
    g = W.static_gaussians(20000, 3)
    views = [W.view((0.3, -0.2, -4.0), 300, 200, 250.0, 0.1), W.view((0.3, -0.2, -4.0), 300, 200, 250.0, 7.0)]
    st = dict(W.settings(), mode="fused")
    p = to_dev(g, device)
    a, _ = rend.forward_static(p, views, st)
    assert torch.equal(a[0], a[1])                  # no time dependence
    q = p["quats"]
    n = q.shape[1]
    zero = torch.zeros(n, device=device)
    g4 = {"means": torch.cat([p["means"], torch.zeros(1, n, device=device)]).contiguous(),
          "log_scales": torch.cat([p["log_scales"], torch.full((1, n), 40.0, device=device)]).contiguous(),
          "rotors": torch.stack([q[0], -q[3], q[2], -q[1], zero, zero, zero, zero]).contiguous(),
          "opacity": p["opacity"], "sh": p["sh"], "sh_degree": 3}
    b, _ = rend.forward(g4, views[:1], st)
    d = float((a[0] - b[0]).abs().max())
    print(f"static vs 4D path: max diff {d:.3g}")
    assert d <= 2e-5


def test_static_and_4d_states_do_not_mix(r4d, rend, device):
    g = W.static_gaussians(100, 0)
    v = W.view((0.0, 0.0, -4.0), 32, 32, 40.0, 0.5)
    p = to_dev(g, device)
    _, saved = rend.forward_static(p, [v], W.settings())
    g4 = W.gaussians(100, 0)
    p4 = {k: torch.as_tensor(g4[k]).to(device) for k in ("means", "log_scales", "rotors", "opacity", "sh")}
    p4["sh_degree"] = 0
    with pytest.raises(r4d.R4DError):
        rend.backward(p4, [v], W.settings(), saved, [torch.zeros(3, 32, 32, device=device)])
