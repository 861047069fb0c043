"""Parity of the speed-field (optical flow) render of the HIP path with the
FP64 CPU oracle (Sec. 3.2.2: each Gaussian's sliced mean moves with speed
V / W; its projection is composited with the colour weights, background 0).

Tolerances (FP32 GPU vs FP64 oracle), derived like the colour ones:
  * per-Gaussian flow: |GPU - oracle| <= 1e-4 (|oracle| + kappa), kappa the
    size of the terms the FP32 speed V / W and its projection are summed from
    (they can cancel; see _flow_condition).  The oracle's own formulas run in
    float32 on this scene reach 5.3e-5 of (|oracle| + kappa), the GPU 1.6e-5;
  * flow images: max |GPU - oracle| <= 1e-4 * max_i |flow_i| on every pixel the
    oracle does not flag as ambiguous -- the colour bound (1e-4 for values in
    [0, 1]) scaled by the largest value a Gaussian contributes;
  * colour images of a flow render: bit-identical to those of the plain render;
  * gradients of a loss on colour and flow: per parameter group
    ||g - g_ref|| / ||g_ref|| <= 1e-3, as for colour alone; the float64
    instantiation agrees with central differences of its own forward to 1e-5.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import render as O

from helpers import image_errors, to_device

pytestmark = pytest.mark.gpu

PARAMS = ("means", "log_scales", "rotors", "opacity", "sh")


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


@pytest.fixture(scope="module")
def scene2k_flow():
    g, views, st = W.scene_2k()
    ref = O.render(g, views[0], st, flow=True)
    return g, views, st, ref


def _flow_condition(g, view, pre):
    """Per Gaussian, the size of the terms the FP32 flow is formed from:
    (fx / z) (1 + |x/z| + |y/z|) (sum_i sum_k |R_ik R_3k| s_k^2) / W.  The speed
    V / W sums products of rotation entries that can cancel, so its rounding
    error scales with these terms, not with the flow itself."""
    R = pre["R"].detach().numpy()
    s2 = np.exp(2 * g["log_scales"].astype(np.float64)).T
    vmag = np.einsum("nik,nk->n", np.abs(R[:, :3, :] * R[:, 3:4, :]), s2)
    w = np.einsum("nk,nk->n", R[:, 3, :] ** 2, s2)
    m2 = pre["mean2"].detach().numpy()
    z = np.abs(pre["depth"].detach().numpy()) + 1e-30
    xz = (m2[:, 0] - view["cx"]) / view["fx"]
    yz = (m2[:, 1] - view["cy"]) / view["fy"]
    return view["fx"] / z * (1 + np.abs(xz) + np.abs(yz)) * vmag / w


def _flow_errors(gpu: np.ndarray, ref: np.ndarray, ambiguous: np.ndarray):
    keep = ~ambiguous.reshape(-1)
    err = np.abs(gpu.reshape(2, -1) - ref.reshape(2, -1))[:, keep]
    return float(err.max()) if err.size else 0.0


def test_flow_render_2k_matches_oracle(r4d, scene2k_flow, device):
    g, views, st, ref = scene2k_flow
    print("case: flow 2k scene 128x128 tile 16", flush=True)
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    imgs, flows, saved = rend.forward(p, views, st, flow=True)
    plain, psaved = rend.forward(p, views, st)
    torch.cuda.synchronize()
    # the colour pass of a flow render is the plain render
    assert torch.equal(imgs[0], plain[0])
    assert torch.equal(saved.copy(0, r4d.BUF_TFINAL, 0), psaved.copy(0, r4d.BUF_TFINAL, 0))
    assert torch.equal(saved.copy(0, r4d.BUF_NCONTRIB, 0), psaved.copy(0, r4d.BUF_NCONTRIB, 0))
    # per-Gaussian flow of the visible Gaussians
    n = g["opacity"].shape[0]
    keys = saved.copy(0, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32)
    vis = keys != 0xFFFFFFFF
    vis &= ~O.gaussian_margin_flags(ref["pre"], st).numpy()
    assert vis.sum() > 500
    gf = saved.copy(0, r4d.BUF_FLOW, n).cpu().numpy().astype(np.float64)[vis]
    rf = ref["pre"]["flow"].numpy()[vis]
    scale = np.abs(rf).max()
    assert scale > 10.0
    d = np.abs(gf - rf)
    kappa = _flow_condition(g, views[0], ref["pre"])[vis][:, None]
    ratio = d / (np.abs(rf) + kappa)
    print(f"per-Gaussian flow: max err {d.max():.3g} (max |flow| {scale:.3g}), "
          f"max err / (|flow| + kappa) {ratio.max():.3g}")
    assert np.all(ratio <= 1e-4)
    # flow image
    err = _flow_errors(flows[0].cpu().numpy().astype(np.float64), ref["flow"].numpy(),
                       ref["ambiguous"].numpy())
    n_amb = int(ref["ambiguous"].sum())
    print(f"flow image: max err {err:.3g}, tol {1e-4 * scale:.3g}, ambiguous {n_amb}")
    assert n_amb <= 0.01 * 128 * 128
    assert err <= 1e-4 * scale
    assert float(flows[0].abs().max()) > 1.0


def test_flow_render_modes_and_ragged_views_agree(r4d, device):
    """Per-view, fused and graph modes render the same flow images for two
    views of different (non-tile-multiple) sizes; the oracle checks one."""
    g = W.gaussians(3000, 1)
    views = [W.view((0.4, -0.2, -4.0), 83, 61, 70.0, 0.3),
             W.view((-1.0, 0.5, -3.8), 50, 77, 60.0, 0.7)]
    st = W.settings()
    p = to_device(g, device)
    rend = r4d.Renderer(device)
    outs = {}
    for mode in ("per_view", "fused", "graph"):
        s = dict(st, mode=mode)
        imgs, flows, saved = rend.forward(p, views, s, flow=True)
        torch.cuda.synchronize()
        saved.check()
        outs[mode] = ([i.clone() for i in imgs], [f.clone() for f in flows])
    for mode in ("fused", "graph"):
        for a, b in zip(outs[mode][0] + outs[mode][1], outs["per_view"][0] + outs["per_view"][1]):
            assert torch.equal(a, b), mode
    ref = O.render(g, views[1], st, flow=True)
    scale = float(ref["pre"]["flow"][ref["pre"]["valid"]].abs().max())
    err = _flow_errors(outs["fused"][1][1].cpu().numpy().astype(np.float64), ref["flow"].numpy(),
                       ref["ambiguous"].numpy())
    assert err <= 1e-4 * scale
    err, _ = image_errors(outs["fused"][0][1].cpu().numpy().astype(np.float64),
                          ref["image"].numpy(), ref["ambiguous"].numpy())
    assert err <= 1e-4


def _flow_loss_refs(g, views, st, w_img, w_flow):
    ref = O.render(g, views[0], st, requires_grad=True, flow=True)
    loss = (ref["image"] * torch.as_tensor(w_img)).sum() + (ref["flow"] * torch.as_tensor(w_flow)).sum()
    loss.backward()
    return ref


def test_flow_gradients_vs_oracle(r4d, device):
    g, views, st = W.scene_fd_subset()
    rng = np.random.default_rng(7)
    w_img = rng.uniform(-1, 1, (3, 32, 32))
    w_flow = rng.uniform(-1, 1, (2, 32, 32)) * 0.1
    ref = _flow_loss_refs(g, views, st, w_img, w_flow)
    p = to_device(g, device)
    for k in PARAMS:
        p[k].requires_grad_(True)
    imgs, flows = r4d.render_flow(p, views, st)
    scale = float(ref["pre"]["flow"].detach()[ref["pre"]["valid"]].abs().max())
    err = _flow_errors(flows[0].detach().cpu().numpy().astype(np.float64),
                       ref["flow"].detach().numpy(), ref["ambiguous"].numpy())
    assert err <= 1e-4 * scale
    loss = (imgs[0] * torch.as_tensor(w_img, dtype=torch.float32, device=device)).sum() + \
        (flows[0] * torch.as_tensor(w_flow, dtype=torch.float32, device=device)).sum()
    loss.backward()
    for k in PARAMS:
        gg = p[k].grad.cpu().numpy().astype(np.float64)
        gr = ref["params"][k].grad.numpy()
        rel = float(np.linalg.norm(gg - gr) / max(np.linalg.norm(gr), 1e-30))
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-3, k
        assert np.all(np.abs(gg - gr) <= 1e-3 * (np.abs(gr) + 1e-2 * np.abs(gr).max()) + 1e-7), k


def test_flow_gradients_fp64_match_central_differences(r4d, device):
    """float64 flow backward vs central differences of its own forward, on a
    loss that weights the flow channels only (the colour part is covered by
    the colour-only check)."""
    g, views, st = W.scene_fd_subset()
    g64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    w_flow = torch.as_tensor(np.random.default_rng(8).uniform(-1, 1, (2, 32, 32)),
                             dtype=torch.float64, device=device)
    zero_img = torch.zeros(3, 32, 32, dtype=torch.float64, device=device)
    rend = r4d.Renderer(device)
    p = to_device(g64, device, torch.float64)
    _, _, saved = rend.forward(p, views, st, flow=True)
    grads = rend.backward(p, views, st, saved, [zero_img], [w_flow])
    grads = {k: v.cpu().numpy() for k, v in grads.items()}
    live = np.nonzero(np.abs(grads["means"]).sum(0))[0]
    assert live.size >= 10
    rng = np.random.default_rng(9)

    def loss_and_sig(pp):
        _, fl, sv = rend.forward(pp, views, st, flow=True)
        nc = sv.copy(0, r4d.BUF_NCONTRIB, 0).cpu().numpy()
        return float((fl[0] * w_flow).sum()), nc

    checked = 0
    for key in ("means", "log_scales", "rotors", "opacity"):
        arr = g64[key]
        for gi in rng.choice(live, size=8, replace=False):
            comp = int(rng.integers(0, arr.shape[0])) if arr.ndim == 2 else None
            idx = (comp, gi) if comp is not None else (gi,)
            theta = arr[idx]
            h = 1e-6 * max(1.0, abs(theta))
            vals, sigs = [], []
            for sgn in (1, -1):
                q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g64.items()}
                q[key][idx] = theta + sgn * h
                lv, sg = loss_and_sig(to_device(q, device, torch.float64))
                vals.append(lv)
                sigs.append(sg)
            if not np.array_equal(sigs[0], sigs[1]):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = grads[key][idx]
            assert abs(fd - ad) <= 1e-5 * max(abs(fd), abs(ad), 1e-3), (key, idx, fd, ad)
            checked += 1
    assert checked >= 20
    # SH coefficients do not move the flow
    assert np.all(grads["sh"] == 0.0)


def test_flow_state_errors_and_colour_only_backward(r4d, device):
    g, views, st = W.scene_fd_subset()
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    w = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, (3, 32, 32)),
                        dtype=torch.float32, device=device)
    wf = torch.ones(2, 32, 32, dtype=torch.float32, device=device)
    # flow gradients need a flow forward
    _, saved = rend.forward(p, views, st)
    with pytest.raises(r4d.R4DError):
        rend.backward(p, views, st, saved, [w], [wf])
    with pytest.raises(r4d.R4DError):
        saved.copy(0, r4d.BUF_FLOW, g["opacity"].shape[0])
    plain = {k: v.clone() for k, v in rend.backward(p, views, st, saved, [w]).items()}
    # a flow forward's state serves the colour-only backward, with the same result
    _, _, fsaved = rend.forward(p, views, st, flow=True)
    col = rend.backward(p, views, st, fsaved, [w])
    for k in PARAMS:
        a, b = col[k].double(), plain[k].double()
        assert float((a - b).norm()) <= 1e-6 * max(float(b.norm()), 1e-30), k
    # and a zero flow gradient adds nothing
    both = rend.backward(p, views, st, fsaved, [w], [torch.zeros_like(wf)])
    for k in PARAMS:
        a, b = both[k].double(), plain[k].double()
        assert float((a - b).norm()) <= 1e-6 * max(float(b.norm()), 1e-30), k
