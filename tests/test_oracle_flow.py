"""Pins for the oracle's speed field (Sec. 3.2.2: the slice moves with speed
V/W; its projection, composited like a colour, is the rendered optical flow of
the paper's flow figure).

* the per-Gaussian flow equals the time derivative of the projected mean,
  taken by central differences of the oracle's own preprocess at t +- h;
* an x-t rotor on the optical axis moves at the hand-derived speed
  cos(phi) sin(phi) (st^2 - sx^2) / W, so its flow is fx * that / z, and its
  flow image is that flow times the closed-form alpha of the single Gaussian;
* Gaussians with no temporal rotor part do not move (flow exactly 0).
"""
import math

import numpy as np
import torch

import workloads as W
from oracle import render as O

from test_oracle_composite import _scene


def test_flow_is_time_derivative_of_projected_mean():
    g = W.gaussians(400, 1)
    v = W.view((0.3, -0.2, -3.0), 96, 80, 90.0, 0.5)
    P = O.params_to_torch(g)
    st = O.settings_dict({})
    pre = O.preprocess(P, v, st)
    h = 1e-5
    plus = O.preprocess(P, dict(v, t=v["t"] + h), st)["mean2"]
    minus = O.preprocess(P, dict(v, t=v["t"] - h), st)["mean2"]
    fd = (plus - minus) / (2 * h)
    flow = pre["flow"]
    ok = pre["depth"] > 0.5          # away from the camera plane
    assert int(ok.sum()) > 300
    err = (flow - fd)[ok].abs().max() / flow[ok].abs().max()
    assert float(err) < 1e-7
    # the speed is really non-zero for these rotors
    assert float(flow[ok].abs().max()) > 1.0


def test_xt_rotor_on_axis_closed_form_flow_image():
    f, z, o = 150.0, 4.0, 0.8
    th, sx, sy, sz, st_ = 0.35, 0.08, 0.05, 0.05, 0.3
    w2c = np.concatenate([np.eye(3), np.array([[0.0], [0.0], [z]])], 1)   # camera at (0,0,-4)
    g, view = _scene([{"xyz": (0, 0, 0), "o": o, "c": (1, 1, 1), "t": 0.5,
                       "rotor": (math.cos(th), 0, 0, 0, math.sin(th), 0, 0, 0)}],
                     f=f, w=96, h=96, w2c=w2c)
    g["log_scales"][:, 0] = np.log([sx, sy, sz, st_])
    phi = 2 * th
    Wt = math.sin(phi) ** 2 * sx ** 2 + math.cos(phi) ** 2 * st_ ** 2
    vx = math.cos(phi) * math.sin(phi) * (st_ ** 2 - sx ** 2) / Wt
    out = O.render(g, view, {}, flow=True)
    pre = out["pre"]
    assert abs(float(pre["flow"][0, 0]) - f * vx / z) < 1e-12 * f
    assert abs(float(pre["flow"][0, 1])) < 1e-15
    # sliced at t = mu_t: centre on the axis, 2D covariance of the x-t slice
    var_x = (f / z) ** 2 * sx ** 2 * st_ ** 2 / Wt + 0.3
    var_y = (f / z) ** 2 * sy ** 2 + 0.3
    ys, xs = np.mgrid[0:96, 0:96]
    q = (xs + 0.5 - 48) ** 2 / var_x + (ys + 0.5 - 48) ** 2 / var_y
    a = np.minimum(0.99, o * np.exp(-0.5 * q))
    a = np.where((q <= 9) & (a >= 1 / 255), a, 0.0)
    fl = out["flow"].numpy()
    assert np.abs(fl[0] - f * vx / z * a).max() < 1e-10
    assert np.abs(fl[1]).max() < 1e-14
    # the same weights as the colour (white on black)
    assert np.abs(out["image"].numpy()[0] - a).max() < 1e-12


def test_static_gaussians_have_zero_flow():
    rng = np.random.default_rng(4)
    gs = []
    for _ in range(12):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        gs.append({"xyz": tuple(rng.uniform(-0.3, 0.3, 3) + [0, 0, 3]), "o": 0.8,
                   "c": (0.5, 0.5, 0.5), "rotor": tuple(q) + (0, 0, 0, 0), "scale": 0.05})
    g, view = _scene(gs, w=32, h=32, f=40.0)
    out = O.render(g, view, {}, flow=True)
    assert float(out["pre"]["flow"].abs().max()) == 0.0
    assert float(out["flow"].abs().max()) == 0.0
    assert float(out["image"].abs().max()) > 0.1


def test_flow_gradient_matches_central_differences():
    """Autograd through the composited flow (a loss on flow channels only)
    against central differences on a few parameters."""
    g = W.gaussians(24, 0)
    v = W.view((0.0, 0.0, -3.0), 20, 20, 30.0, 0.5)
    rng = np.random.default_rng(5)
    wts = torch.as_tensor(rng.uniform(-1, 1, (2, 400)))
    P = O.params_to_torch(g, requires_grad=True)
    loss = (O.render(g, v, {}, P=P, flow=True)["flow"].reshape(2, -1) * wts).sum()
    loss.backward()

    def value(key, idx, dv):
        P2 = O.params_to_torch(g)
        with torch.no_grad():
            P2[key][idx] += dv
        return float((O.render(g, v, {}, P=P2, flow=True)["flow"].reshape(2, -1) * wts).sum())

    checked = 0
    for key, idx in (("means", (0, 3)), ("means", (3, 5)), ("rotors", (4, 7)), ("rotors", (6, 2)),
                     ("log_scales", (3, 9)), ("log_scales", (0, 11))):
        grad = float(P[key].grad[idx])
        h = 1e-6
        fd = (value(key, idx, h) - value(key, idx, -h)) / (2 * h)
        if abs(fd) > 1e-8:
            checked += 1
        assert abs(grad - fd) <= 1e-5 * max(1.0, abs(fd)), (key, idx, grad, fd)
    assert checked >= 3
