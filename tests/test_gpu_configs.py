"""Parity on the large scene and on the orbit renders, in the launch
configuration the benchmark times them in (graph mode, every render of the
workload in one call), plus the 4096-pixel image check of the 500k scene.

Large scene: 3,000,000 Gaussians with means in [-4, 4]^3, SH degree 3,
1920x1080, f = 1400, 8 timestamps x 2 views from radius 4.  The cameras sit
on the faces of the cloud, so Gaussians lie nearer than the near plane and far
outside the image (where the projection's Jacobian is taken at the guard-band
clamp, Sec. 3.1 with the 3DGS conventions), and the time cull is the lossy
tau = 9 (Sec. 3.2.2 drops a slice whose temporal falloff lambda dt^2 exceeds the
threshold).  Checked on two renders:
  * every Gaussian the GPU keeps is valid in the oracle, and every Gaussian the
    oracle drops by the near plane or by tau = 9 (outside the FP32 margins) is
    dropped on the GPU; both drops hit Gaussians that would have been blended;
  * the records (2D mean, conic, opacity, depth, colour) of kept Gaussians,
    including those whose Jacobian is clamped, against the oracle's;
  * binning and the (tile, depth, index) order, bit-exact on whole tile rows
    against the CPU re-derivation from the GPU's records, and the total entry
    count over the whole frame;
  * sampled pixels against the oracle (1e-4 on unambiguous pixels, at most 8%
    ambiguous), some of them reached by clamped Gaussians.
A 40,000-Gaussian set with the same geometry checks the gradients of a
sampled-pixel loss (1e-3 relative per parameter group).
Orbit: 300,000 Gaussians, 30 renders at t in [0, 1]; sampled pixels of three.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import render as O

from helpers import (PARAM_KEYS, cpu_tile_rows, depth_positions, front_cut, image_errors,
                     kept_tiles, to_device)

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4
AMB_MAX = 0.08
LARGE_RENDERS = (0, 9)       # t = 0 from -z; t = 4/7 from +x
LARGE_PIXELS = 384


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


@pytest.fixture(scope="module")
def large(r4d, device):
    g, views, st = W.scene_3m_large()
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    print("case: 3M large scene, 16 renders, graph mode", flush=True)
    imgs, saved = rend.forward(p, views, dict(st, mode="graph"), save=True)
    saved.check()
    imgs = [i.clone() for i in imgs]
    n = g["opacity"].shape[0]
    out = {}
    for v in LARGE_RENDERS:
        out[v] = {
            "image": imgs[v],
            "rec": saved.copy(v, r4d.BUF_RECORDS, n).cpu().numpy().astype(np.float64),
            "rect": saved.copy(v, r4d.BUF_RECT, n).cpu().numpy().view(np.uint16),
            "key": saved.copy(v, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32),
            "vals": saved.copy(v, r4d.BUF_VALUES, n).cpu().numpy().view(np.uint32),
            "rng": saved.copy(v, r4d.BUF_RANGES, n).cpu().numpy().view(np.uint32),
            "rest": saved.copy(v, r4d.BUF_REST, n).cpu().numpy().view(np.uint32),
            "stats": saved.stats(v),
            "settings": dict(r4d.default_settings(), **saved.settings),
        }
    cfg = saved.config()
    saved.release()
    del p
    torch.cuda.empty_cache()
    return g, views, st, out, cfg


def _clamped(pre, view, st):
    """Gaussians whose x/z or y/z lies beyond the guard band (the Jacobian is
    taken at the clamp)."""
    s = O.settings_dict(st)
    m2 = pre["mean2"].detach().numpy()
    xz = (m2[:, 0] - view["cx"]) / view["fx"]
    yz = (m2[:, 1] - view["cy"]) / view["fy"]
    limx = s["guard_band"] * 0.5 * view["width"] / view["fx"]
    limy = s["guard_band"] * 0.5 * view["height"] / view["fy"]
    return (np.abs(xz) > limx) | (np.abs(yz) > limy)


U32 = 2.0 ** -24   # unit roundoff of float32


def _fp32_scales(g, pre, view):
    """Magnitudes that set the float32 error of each Gaussian's record, from
    the oracle's FP64 intermediates (the record is computed in float32 from
    float32 inputs); a rounding contributes the unit roundoff times them:
      * p_scale: of the camera-space position.  The rotation R from the
        normalised rotor has entries of unit scale, each carrying roundings of
        1 (absolute, however small the entry), so an entry of Sigma_4 =
        R S^2 R^T, sum_k R_ik R_jk s_k^2, carries them of
        sum_k (|R_ik| + |R_jk|) s_k^2; mu(t) = mu_xyz + (t - mu_t) V / W then
        carries them of |t - mu_t| (V_terms + |V| W_terms / W) / W and of
        |mu(t)|; p = M mu(t) + t_w, of |M| |mu(t)| + |t_w| on top;
      * gamma: cancellation factor of Sigma_3D = U - V V^T / W, the magnitude
        of the terms over the magnitude of the result;
      * kappa: condition number of the (dilated) Sigma_2D, by which the
        inversion to the conic multiplies relative errors."""
    R = pre["R"].detach().numpy()
    s2 = np.exp(2.0 * g["log_scales"].T.astype(np.float64))
    aR = np.abs(R)
    terms = np.einsum("nik,nk->ni", aR, s2)[:, :, None] + np.einsum("njk,nk->nj", aR, s2)[:, None, :]
    cov4 = np.einsum("nik,njk,nk->nij", R, R, s2)
    V, W = cov4[:, :3, 3], cov4[:, 3, 3]
    dt = np.abs(view["t"] - g["means"][3].astype(np.float64))
    vel_rel = (terms[:, :3, 3] + np.abs(V) * terms[:, 3, 3][:, None] / W[:, None]) / W[:, None]
    mu3 = pre["mu3"].detach().numpy()
    M = view["world_to_cam"].astype(np.float64).reshape(3, 4)
    mu_scale = dt[:, None] * vel_rel + np.abs(mu3)
    absM = np.abs(M[:, :3])[None]
    p_scale = (absM @ mu_scale[..., None])[..., 0] + \
        (absM @ np.abs(mu3)[..., None])[..., 0] + np.abs(M[:, 3])
    cov3 = pre["cov3"].detach().numpy()
    sch = terms[:, :3, :3] + np.abs(V)[:, :, None] * np.abs(V)[:, None, :] / W[:, None, None]
    gamma = sch.reshape(-1, 9).max(1) / np.abs(cov3).reshape(-1, 9).max(1)
    ev = np.linalg.eigvalsh(pre["cov2"].detach().numpy())
    kappa = ev[:, 1] / ev[:, 0]
    return p_scale.max(1), gamma, kappa


@pytest.mark.parametrize("vi", LARGE_RENDERS)
def test_3m_culls_and_records(large, vi):
    g, views, st, out, _ = large
    view, o = views[vi], out[vi]
    s = O.settings_dict(st)
    with torch.no_grad():
        pre = O.preprocess(O.params_to_torch(g), view, s)
    key, rec = o["key"], o["rec"]
    vis = key != 0xFFFFFFFF
    valid = pre["valid"].numpy()
    lam = pre["lam_dt2"].numpy()
    dep = pre["depth"].detach().numpy()
    op = pre["opacity"].detach().numpy()
    # decisions within FP32 rounding of a threshold may go either way
    margin = (np.abs(lam - s["time_cull"]) < 1e-5 * s["time_cull"]) | \
        (np.abs(dep - s["near_plane"]) < 1e-6)
    assert not np.any(vis & ~valid & ~margin), "the GPU keeps a Gaussian the oracle drops"
    # time cull at tau = 9: Gaussians between 9 and 16 would be blended at tau = 16
    t_drop = (lam > s["time_cull"] * (1 + 1e-5)) & (lam <= 16.0) & (op >= s["alpha_min"])
    # near plane: in front of the camera but nearer than 0.2
    n_drop = (lam <= s["time_cull"] * (1 - 1e-5)) & (dep > 0) & (dep < s["near_plane"] - 1e-6)
    print(f"render {vi}: kept {int(vis.sum())}, dropped by tau=9 {int(t_drop.sum())}, "
          f"by the near plane {int(n_drop.sum())}", flush=True)
    assert t_drop.sum() > 1000 and n_drop.sum() > 1000
    assert not np.any(vis & t_drop) and not np.any(vis & n_drop)
    # near-plane Gaussians opaque enough to be blended somewhere
    assert np.sum(n_drop & (op >= s["alpha_min"])) > 100

    clamped = _clamped(pre, view, s) & vis
    print(f"render {vi}: {int(clamped.sum())} kept Gaussians with a clamped Jacobian", flush=True)
    assert clamped.sum() > 100
    m2 = pre["mean2"].detach().numpy()
    cn = pre["conic"].detach().numpy()
    rgb = pre["rgb"].detach().numpy()
    i = np.nonzero(vis & valid)[0]
    # 2D mean f x / z + c: the camera-space error scaled by f / z and, through
    # 1 / z, by 1 + |x / z| + |y / z|; the two products and the reciprocal add 3
    # roundings relative to f x / z and the sum with c half an ulp of the result
    # (the 1e-3 floor covers |mean| < 1.6e4); 16 roundings of the position scale
    p_scale, gamma, kappa = _fp32_scales(g, pre, view)
    p_scale, gamma, kappa = p_scale[i], gamma[i], kappa[i]
    z = dep[i]
    xy = np.abs(m2[i] - np.array([view["cx"], view["cy"]])) / view["fx"]
    tol_m2 = (1e-3 + 16 * U32 * view["fx"] * p_scale / z * (1 + xy.sum(1)) +
              3 * U32 * view["fx"] * xy.max(1))
    err_m2 = np.abs(rec[i, 0:2] - m2[i]).max(1)
    w = int(np.argmax(err_m2 / tol_m2))
    print(f"2D mean: worst error / bound {(err_m2 / tol_m2).max():.3g} (error "
          f"{err_m2[w]:.3g}, z {z[w]:.4g}, |x/z| + |y/z| {xy[w].sum():.3g}, "
          f"position scale {p_scale[w]:.3g})", flush=True)
    assert np.all(err_m2 <= tol_m2)
    # conic = Sigma_2D^-1: Sigma_2D carries the Schur complement's cancellation
    # (gamma) on top of a few roundings, and the inversion multiplies relative
    # errors by kappa; relative to the conic's largest diagonal entry
    cscale = np.maximum(np.abs(cn[i, 0]), np.abs(cn[i, 2]))
    tol_cn = 1e-4 + 64 * U32 * (gamma + 1.0) * kappa
    for c, j in ((2, 0), (3, 1), (4, 2)):
        err = np.abs(rec[i, c] - cn[i, j]) / cscale
        w = int(np.argmax(err / tol_cn))
        print(f"conic[{j}] worst relative {err.max():.3g}; clamped "
              f"{err[clamped[i]].max():.3g}; worst / bound {(err / tol_cn).max():.3g} "
              f"(gamma {gamma[w]:.3g}, kappa {kappa[w]:.3g})", flush=True)
        assert np.all(err <= tol_cn)
    assert (np.abs(rec[i, 5] - op[i]) / op[i]).max() < 1e-5
    # depth = camera-space z: 16 roundings of the position scale
    err_d = np.abs(rec[i, 6] - dep[i])
    tol_d = 16 * U32 * p_scale + U32 * dep[i]
    print(f"depth: worst error / bound {(err_d / tol_d).max():.3g}", flush=True)
    assert np.all(err_d <= tol_d)
    # colour: SH of the unit direction from the camera centre to mu(t), whose
    # error is the position's over the distance (higher bands ~ N(0, 0.05): the
    # colour moves by less than its direction)
    w2c = view["world_to_cam"].astype(np.float64).reshape(3, 4)
    centre = -(w2c[:, :3].T @ w2c[:, 3])
    dist = np.linalg.norm(pre["mu3"].detach().numpy()[i] - centre, axis=1)
    err_c = np.abs(rec[i, 8:11] - rgb[i]).max(1)
    tol_c = 1e-5 + 16 * U32 * p_scale / dist
    print(f"colour: worst error / bound {(err_c / tol_c).max():.3g}", flush=True)
    assert np.all(err_c <= tol_c)


@pytest.mark.parametrize("vi", LARGE_RENDERS)
def test_3m_binning_bit_exact_on_tile_rows(large, vi):
    g, views, st, out, cfg = large
    view, o = views[vi], out[vi]
    s = o["stats"]
    tx, ty = s["tiles_x"], s["tiles_y"]
    rows = sorted({0, ty // 3, ty // 2, (2 * ty) // 3, ty - 1})
    total, lists = cpu_tile_rows(o["rec"], o["rect"], o["key"], tx, rows, cfg["tile_size"],
                                 view["width"], view["height"])
    print(f"render {vi}: D = {s['n_dup']} (CPU {total}), visible {s['n_visible']}, front "
          f"lists {s['n_front']}, rests {s['rest_tiles']}", flush=True)
    assert s["n_dup"] == total
    assert s["n_visible"] == int((o["key"] != 0xFFFFFFFF).sum())
    rng, vals, rest_rng = o["rng"], o["vals"], o["rest"]
    # front lists: a kept tile's whole list, any other tile's entries from depth
    # positions below the cut (the rest, when collected, is the remainder)
    r0 = front_cut(s["n_visible"], o["settings"], tx, ty)
    pos = depth_positions(o["key"])
    kept = (kept_tiles(o["rect"], o["key"], tx, ty, int(o["settings"]["front_keep"]), r0)
            if r0 is not None else np.ones(tx * ty, dtype=bool))
    checked = 0
    for t, ref in lists.items():
        front = kept[t] | (pos[ref.astype(np.int64)] < (r0 if r0 is not None else 1 << 62))
        a, b = int(rng[t, 0]), int(rng[t, 1])
        got = vals[a:b] if b > a else np.zeros(0, np.uint32)
        assert np.array_equal(got, ref[front]), f"tile {t}"
        a, b = int(rest_rng[t, 0]), int(rest_rng[t, 1])
        if b > a:
            assert np.array_equal(vals[a:b], ref[~front]), f"rest of tile {t}"
        checked += ref.size
    print(f"{checked} entries on {len(lists)} tiles equal", flush=True)
    assert checked > 0
    # ranges partition [0, n_front) in tile order
    lens = (rng[:, 1].astype(np.int64) - rng[:, 0].astype(np.int64))
    assert lens.sum() == s["n_front"]
    nz = lens > 0
    assert np.all(rng[nz][1:, 0] == rng[nz][:-1, 1])


@pytest.mark.parametrize("vi", LARGE_RENDERS)
def test_3m_sampled_pixels(large, vi):
    g, views, st, out, _ = large
    view = views[vi]
    pix = W.pixel_sample(view["height"], view["width"], LARGE_PIXELS, seed=7 + vi)
    with torch.no_grad():
        ref = O.render(g, view, st, pixels=pix)
    gpu = out[vi]["image"].reshape(3, -1)[:, torch.as_tensor(pix, device=out[vi]["image"].device)]
    err, n_amb = image_errors(gpu.cpu().numpy().astype(np.float64), ref["image"].numpy(),
                              ref["ambiguous"].numpy())
    # pixels some clamped Gaussian is blended into (alpha >= alpha_min inside the extent)
    pre = ref["pre"]
    s = O.settings_dict(st)
    cl = np.nonzero(_clamped(pre, view, s) & pre["valid"].numpy())[0]
    m2 = pre["mean2"].detach().numpy()[cl]
    cn = pre["conic"].detach().numpy()[cl]
    o_t = pre["opacity"].detach().numpy()[cl]
    px = np.stack([pix % view["width"], pix // view["width"]], 1) + 0.5
    reached = 0
    for k in range(0, px.shape[0], 32):
        d = m2[None] - px[k:k + 32, None]
        q = cn[:, 0] * d[..., 0] ** 2 + 2 * cn[:, 1] * d[..., 0] * d[..., 1] + cn[:, 2] * d[..., 1] ** 2
        hit = (q <= 9.0) & (o_t * np.exp(-0.5 * q) >= s["alpha_min"])
        reached += int(hit.any(1).sum())
    print(f"render {vi}: sampled max err {err:.3g}, ambiguous {n_amb}/{pix.size}, "
          f"pixels reached by clamped Gaussians {reached}", flush=True)
    assert n_amb <= AMB_MAX * pix.size
    assert reached > 0
    assert err <= IMG_TOL


def test_3m_geometry_gradients_reduced_set(r4d, device):
    """40,000 Gaussians in [-4, 4]^3 seen from the large scene's cameras at
    t = 0 and t = 4/7, tau = 9, graph mode: gradients of a loss on 160
    sampled pixels of each render against the oracle's autograd."""
    _, views, st = W.scene_3m_large(n=8)      # the cameras and settings only
    views = [views[i] for i in LARGE_RENDERS]
    g = W.gaussians(40_000, 3, xyz_half_extent=4.0)
    gst = dict(st, mode="graph")
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    imgs, saved = rend.forward(p, views, gst)
    saved.check()
    imgs = [i.clone() for i in imgs]
    P = None
    total = None
    dl = []
    rng = np.random.default_rng(5)
    worst, clamped_blended = 0.0, 0
    for j, v in enumerate(views):
        pix = W.pixel_sample(v["height"], v["width"], 160, seed=31 + j)
        ref = O.render(g, v, st, pixels=pix, requires_grad=True, P=P)
        P = ref["params"]
        keep = ~ref["ambiguous"].numpy()
        assert keep.sum() >= (1 - AMB_MAX) * pix.size
        gpu = imgs[j].reshape(3, -1)[:, torch.as_tensor(pix, device=device)].cpu().numpy()
        err = np.abs(gpu.astype(np.float64) - ref["image"].detach().numpy())[:, keep].max()
        worst = max(worst, err)
        w = rng.uniform(-1, 1, (3, pix.size)) * keep[None, :]
        term = (ref["image"] * torch.as_tensor(w)).sum()
        total = term if total is None else total + term
        d = torch.zeros(3, v["height"] * v["width"], dtype=torch.float32)
        d[:, torch.as_tensor(pix)] = torch.as_tensor(w, dtype=torch.float32)
        dl.append(d.reshape(3, v["height"], v["width"]).to(device))
        clamped_blended += int((_clamped(ref["pre"], v, st) & ref["pre"]["valid"].numpy()).sum())
    print(f"sampled image error {worst:.3g}; clamped valid Gaussians {clamped_blended}", flush=True)
    assert worst <= IMG_TOL
    total.backward()
    grads = rend.backward(p, views, gst, saved, dl)
    saved.check()
    for k in PARAM_KEYS:
        a = grads[k].double().cpu().numpy()
        b = P[k].grad.numpy()
        rel = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        print(f"{k}: rel {rel:.3g}", flush=True)
        assert rel <= 1e-3, k


@pytest.fixture(scope="module")
def orbit(r4d, device):
    g, views, st = W.scene_300k_orbit()
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    print("case: 300k orbit, 30 renders, graph mode", flush=True)
    imgs, saved = rend.forward(p, views, dict(st, mode="graph"), save=True)
    saved.check()
    imgs = [i.clone() for i in imgs]
    saved.release()
    return g, views, st, imgs


@pytest.mark.parametrize("vi", (0, 11, 23))
def test_orbit_sampled_pixels(orbit, vi):
    g, views, st, imgs = orbit
    view = views[vi]
    pix = W.pixel_sample(view["height"], view["width"], 1024, seed=40 + vi)
    with torch.no_grad():
        ref = O.render(g, view, st, pixels=pix)
    gpu = imgs[vi].reshape(3, -1)[:, torch.as_tensor(pix, device=imgs[vi].device)]
    err, n_amb = image_errors(gpu.cpu().numpy().astype(np.float64), ref["image"].numpy(),
                              ref["ambiguous"].numpy())
    print(f"orbit render {vi} (t = {view['t']:.3f}): max err {err:.3g}, ambiguous "
          f"{n_amb}/{pix.size}", flush=True)
    assert n_amb <= AMB_MAX * pix.size
    assert err <= IMG_TOL


def test_500k_4096_sampled_pixels(r4d, device):
    """The headline render (500k Gaussians, 1352x1014, tile 16) on the 4096
    pixels of the fixed sample, image only (the oracle's dense path)."""
    g, views, st = W.scene_500k_step()
    view = views[0]
    rend = r4d.Renderer(device)
    imgs, _ = rend.forward(to_device(g, device), views, st, save=False)
    pix = W.pixel_sample(view["height"], view["width"], 4096)
    with torch.no_grad():
        ref = O.render(g, view, st, pixels=pix)
    gpu = imgs[0].reshape(3, -1)[:, torch.as_tensor(pix, device=device)]
    err, n_amb = image_errors(gpu.cpu().numpy().astype(np.float64), ref["image"].numpy(),
                              ref["ambiguous"].numpy())
    print(f"500k: 4096 sampled pixels, max err {err:.3g}, ambiguous {n_amb}", flush=True)
    assert n_amb <= AMB_MAX * pix.size
    assert err <= IMG_TOL
