"""Pins for the oracle's compositing and whole-render behaviour (Sec. 3.1
blending equation; Sec. 3.2.2 time cull; Sec. 3.2.1 static reduction).

The golden cases in tests/golden/composite_cases.json were derived by hand;
the single-Gaussian image is checked against the closed-form 2D covariance of
an isotropic Gaussian on the optical axis, not against the oracle's own
projection code.
"""
import json
import math
import os

import numpy as np
import torch

from oracle import render as O

HERE = os.path.dirname(os.path.abspath(__file__))
C0 = 0.5 / math.sqrt(math.pi)


def _scene(gs, f=64.0, w=16, h=16, t=0.5, w2c=None, sh_degree=0):
    """Gaussians given by camera-space centre (x, y, z) with identity rotor,
    isotropic scale, opacity and base colour; float64 arrays."""
    n = len(gs)
    k = (sh_degree + 1) ** 2
    means = np.zeros((4, n))
    ls = np.zeros((4, n))
    rot = np.zeros((8, n))
    op = np.zeros(n)
    sh = np.zeros((3 * k, n))
    for i, gg in enumerate(gs):
        means[:3, i] = gg["xyz"]
        means[3, i] = gg.get("t", t)
        ls[:3, i] = math.log(gg.get("scale", 0.01))
        ls[3, i] = math.log(gg.get("scale_t", 0.1))
        rot[:, i] = gg.get("rotor", (1, 0, 0, 0, 0, 0, 0, 0))
        op[i] = gg["o"]
        sh[0:3, i] = (np.asarray(gg["c"], dtype=np.float64) - 0.5) / C0
    g = {"means": means, "log_scales": ls, "rotors": rot, "opacity": op, "sh": sh,
         "sh_degree": sh_degree}
    if w2c is None:
        w2c = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    view = {"width": w, "height": h, "fx": f, "fy": f, "cx": w / 2, "cy": h / 2,
            "world_to_cam": w2c, "t": t, "bg": (0, 0, 0)}
    return g, view


def test_golden_composite_cases():
    data = json.load(open(os.path.join(HERE, "golden", "composite_cases.json")))
    px, py = 5, 9
    for case in data["cases"]:
        gs = []
        for gg in case["gaussians"]:
            z = float(gg["depth"])
            xyz = ((px + 0.5 - 8) * z / 64.0, (py + 0.5 - 8) * z / 64.0, z)
            gs.append({"xyz": xyz, "o": gg["o"], "c": gg["c"]})
        g, view = _scene(gs)
        view["bg"] = tuple(case["bg"])
        out = O.render(g, view, {}, pixels=np.array([py * 16 + px]))
        col = out["image"][:, 0].numpy()
        assert np.allclose(col, case["colour"], atol=1e-12), (case["name"], col)
        assert abs(float(out["T_final"][0]) - case["T_final"]) < 1e-12, case["name"]
        assert int(out["n_contrib"][0]) == case["n_contrib"], case["name"]
        assert not bool(out["ambiguous"][0])


def test_single_gaussian_image_closed_form():
    f, z, s, o = 150.0, 4.0, 0.05, 0.8
    colour = (0.9, 0.3, 0.1)
    bg = (0.05, 0.1, 0.2)
    w2c = np.concatenate([np.eye(3), np.array([[0.0], [0.0], [z]])], 1)   # camera at (0,0,-4)
    g, view = _scene([{"xyz": (0, 0, 0), "o": o, "c": colour, "scale": s}], f=f, w=128, h=128,
                     w2c=w2c)
    view["bg"] = bg
    img = O.render(g, view, {})["image"].numpy()
    var = (f * s / z) ** 2 + 0.3
    ys, xs = np.mgrid[0:128, 0:128]
    q = ((xs + 0.5 - 64) ** 2 + (ys + 0.5 - 64) ** 2) / var
    a = np.minimum(0.99, o * np.exp(-0.5 * q))
    use = (q <= 9) & (a >= 1 / 255)
    a = np.where(use, a, 0.0)
    for ch in range(3):
        expect = colour[ch] * a + bg[ch] * (1 - a)
        assert np.abs(img[ch] - expect).max() < 1e-12


def test_time_cull_threshold():
    # lambda dt^2 = dt^2 / s_t^2 with an identity rotor; tau = 4
    st = {"time_cull": 4.0}
    res = []
    for dt in (0.195, 0.205):                  # lambda dt^2 = 3.8025 / 4.2025
        g, view = _scene([{"xyz": (4 / 128, 4 / 128, 4.0), "o": 0.9, "c": (1, 1, 1), "t": 0.5 - dt}])
        out = O.render(g, view, st, pixels=np.array([8 * 16 + 8]))
        res.append(float(out["image"][0, 0]))
    expect_visible = 0.9 * math.exp(-0.5 * 3.8025)   # colour 1 on black
    assert abs(res[0] - expect_visible) < 1e-9
    assert res[1] == 0.0


def test_near_plane_cull():
    out = []
    for z in (0.19, 0.21):
        g, view = _scene([{"xyz": (z / 128, z / 128, z), "o": 0.9, "c": (1, 1, 1), "scale": 0.0005}])
        r = O.render(g, view, {}, pixels=np.array([8 * 16 + 8]))
        out.append(float(r["image"][0, 0]))
    assert out[0] == 0.0 and abs(out[1] - 0.9) < 1e-12


def test_static_reduction_to_3d_gaussian():
    """Zero temporal rotor components, sliced at t = mu_t: the sliced Gaussian is
    the 3D Gaussian R3 diag(s^2) R3^T of the corresponding quaternion, with the
    full opacity (Sec. 3.2.1: the rotor reduces to a quaternion)."""
    rng = np.random.default_rng(9)
    gs = []
    for _ in range(16):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        gs.append({"xyz": tuple(rng.uniform(-1, 1, 3) + [0, 0, 5]), "o": 0.7, "c": (0.5, 0.5, 0.5),
                   "rotor": tuple(q) + (0, 0, 0, 0), "scale": 0.05})
    g, view = _scene(gs)
    g["log_scales"][:3] = np.log(rng.uniform(0.01, 0.1, size=(3, 16)))
    P = O.params_to_torch(g)
    pre = O.preprocess(P, view, {})
    for i in range(16):
        s, b01, b02, b12 = g["rotors"][:4, i]
        w, x, y, z = s, -b12, b02, -b01
        R3 = np.array([
            [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
            [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
            [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        cov = R3 @ np.diag(np.exp(2 * g["log_scales"][:3, i])) @ R3.T
        assert np.allclose(pre["cov3"][i].numpy(), cov, atol=1e-15)
        assert np.allclose(pre["mu3"][i].numpy(), g["means"][:3, i], atol=1e-15)
        assert abs(float(pre["opacity"][i]) - 0.7) < 1e-15
