"""Parity of the HIP render path (through the C ABI) with the FP64 CPU oracle.

Tolerances (FP32 GPU vs FP64 oracle):
  * images: max |GPU - oracle| <= 1e-4 per channel on every pixel the oracle
    does not flag as ambiguous (a cut-off decision within FP32 rounding of its
    threshold, with enough weight to matter);
  * tile assignment and (tile, depth, index) order: bit-exact against a CPU
    re-derivation from the GPU's own integer rectangles and depth keys;
  * gradients: per parameter group ||g - g_ref|| / ||g_ref|| <= 1e-3.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import render as O

from helpers import image_errors, tile_lists, to_device

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


@pytest.fixture(scope="module")
def scene2k():
    g, views, st = W.scene_2k()
    ref = O.render(g, views[0], st)
    return g, views, st, ref


def _render(r4d, g, views, st, device, save=True, dtype=torch.float32):
    rend = r4d.Renderer(device)
    p = to_device(g, device, dtype)
    imgs, saved = rend.forward(p, views, st, save=save)
    torch.cuda.synchronize()
    return rend, p, imgs, saved


def test_image_2k_full_frame(r4d, scene2k, device):
    g, views, st, ref = scene2k
    print("case: 2k scene 128x128 tile 16", flush=True)
    _, _, imgs, _ = _render(r4d, g, views, st, device)
    err, n_amb = image_errors(imgs[0].cpu().numpy().astype(np.float64), ref["image"].numpy(),
                              ref["ambiguous"].numpy())
    print(f"max err {err:.3g}, ambiguous {n_amb}")
    assert n_amb <= 0.01 * 128 * 128
    assert err <= IMG_TOL


def test_blend_and_evaluation_counts_2k(r4d, scene2k, device):
    """The measurement build's per-pixel counts: Gaussians blended equal the
    oracle's contributor count on every unambiguous pixel; entries evaluated
    and entries up to the last contributor bound it from above."""
    g, views, st, ref = scene2k
    print("case: 2k scene blend / evaluation counts", flush=True)
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    rend.set_timing(True)
    imgs, saved = rend.forward(p, views, dict(st, mode="per_view"), save=True)
    rend.set_timing(False)
    n = g["opacity"].shape[0]
    blend = saved.copy(0, r4d.BUF_NBLEND, n).cpu().numpy().astype(np.int64)
    evals = saved.copy(0, r4d.BUF_NEVAL, n).cpu().numpy().astype(np.int64)
    ncon = saved.copy(0, r4d.BUF_NCONTRIB, n).cpu().numpy().astype(np.int64)
    amb = ref["ambiguous"].numpy().reshape(-1)
    want = ref["n_contrib"].numpy().reshape(-1)
    print(f"blended pairs {blend.sum()}, evaluated {evals.sum()}, walked {ncon.sum()}")
    assert np.array_equal(blend[~amb], want[~amb])
    assert (evals >= ncon).all() and (ncon >= blend).all()
    assert blend.sum() > 10 * 128 * 128 // 100


def test_preprocess_records_2k(r4d, scene2k, device):
    g, views, st, ref = scene2k
    _, _, _, saved = _render(r4d, g, views, st, device)
    n = g["opacity"].shape[0]
    rec = saved.copy(0, r4d.BUF_RECORDS, n).cpu().numpy().astype(np.float64)
    key = saved.copy(0, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32)
    pre = ref["pre"]
    vis = key != 0xFFFFFFFF
    valid = pre["valid"].numpy()
    # every Gaussian the GPU keeps is valid in the oracle
    assert not np.any(vis & ~valid)
    m2 = pre["mean2"].detach().numpy()
    cn = pre["conic"].detach().numpy()
    dep = pre["depth"].detach().numpy()
    op = pre["opacity"].detach().numpy()
    rgb = pre["rgb"].detach().numpy()
    i = np.nonzero(vis)[0]
    assert i.size > 100
    assert np.abs(rec[i, 0] - m2[i, 0]).max() < 1e-3
    assert np.abs(rec[i, 1] - m2[i, 1]).max() < 1e-3
    cscale = np.maximum(np.abs(cn[i, 0]), np.abs(cn[i, 2]))
    for c, j in ((2, 0), (3, 1), (4, 2)):
        assert (np.abs(rec[i, c] - cn[i, j]) / cscale).max() < 1e-4
    assert (np.abs(rec[i, 5] - op[i]) / op[i]).max() < 1e-5
    assert (np.abs(rec[i, 6] - dep[i]) / dep[i]).max() < 1e-6
    assert np.abs(rec[i, 8:11] - rgb[i]).max() < 1e-5
    # qmax: min(extent^2, 2 ln(o / alpha_min)) of the record's opacity, rounded up to float32
    # (ln alpha_min is held in float32: differences of a few 1e-8 are allowed)
    qd = np.minimum(st["extent_sigma"] ** 2, 2.0 * (np.log(rec[i, 5]) - np.log(st["alpha_min"])))
    assert np.all(np.abs(rec[i, 7] - qd) <= 1e-6 * np.maximum(qd, 1.0))
    # depth keys are the float32 bit patterns of the record depths
    assert np.array_equal(key[i], rec[i, 6].astype(np.float32).view(np.uint32))


def test_binning_and_sort_bit_exact_2k(r4d, scene2k, device):
    g, views, st, _ = scene2k
    for ts in (8, 16, 32):
        _, _, _, saved = _render(r4d, g, views, dict(st, tile_size=ts), device)
        n = g["opacity"].shape[0]
        vals, rng, ref_vals, ref_rng, s = tile_lists(r4d, saved, 0, n)
        key = saved.copy(0, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32)
        assert s["n_front"] == ref_vals.size
        assert np.array_equal(vals, ref_vals), f"tile {ts}: order differs"
        assert np.array_equal(rng, ref_rng), f"tile {ts}: ranges differ"
        assert s["n_visible"] == int((key != 0xFFFFFFFF).sum())


def test_tile_lists_are_conservative_2k(r4d, scene2k, device):
    """Every pixel where a Gaussian can pass the extent and alpha tests lies in a
    tile whose list holds the Gaussian (evaluated on the GPU's own FP32
    record), and the lists hold fewer entries than the tile bounding boxes."""
    g, views, st, _ = scene2k
    for ts in (8, 16, 32):
        _, _, _, saved = _render(r4d, g, views, dict(st, tile_size=ts), device)
        n = g["opacity"].shape[0]
        rec = saved.copy(0, r4d.BUF_RECORDS, n).cpu().numpy().astype(np.float64)
        key = saved.copy(0, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32)
        vals, rng, _, _, s = tile_lists(r4d, saved, 0, n)
        tx = s["tiles_x"]
        lens = (rng[:, 1] - rng[:, 0]).astype(np.int64)
        listed = np.repeat(np.arange(lens.size), lens) * n + vals.astype(np.int64)
        ys, xs = np.mgrid[0:128, 0:128]
        cx, cy = xs.ravel() + 0.5, ys.ravel() + 0.5
        need = []
        for i in np.nonzero(key != 0xFFFFFFFF)[0]:
            mx, my, a, b, c, o = rec[i, :6]
            dx, dy = mx - cx, my - cy
            q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
            reach = (q <= 9.0 * (1 + 1e-5)) & (o * np.exp(-0.5 * q) >= (1 / 255) * (1 - 1e-5))
            t = (ys.ravel()[reach] // ts) * tx + xs.ravel()[reach] // ts
            need.append(np.unique(t) * n + i)
        need = np.concatenate(need)
        assert need.size > 0
        missing = need[~np.isin(need, listed)]
        assert missing.size == 0, f"tile {ts}: {missing.size} (tile, Gaussian) pairs missing"
        rect = saved.copy(0, r4d.BUF_RECT, n).cpu().numpy().view(np.uint16).astype(np.int64)
        box = int(((rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1])).sum())
        print(f"tile {ts}: {vals.size} entries, {box} in the runs' bounding boxes", flush=True)
        assert vals.size <= box


RASTER_CONFIGS = ((8, 1), (16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4))


def test_tile_size_invariance_2k(r4d, scene2k, device):
    """Every (tile size, pixels per lane) gives the same image bit for bit, and
    the same gradients up to the order of float atomics."""
    g, views, st, _ = scene2k
    out, grads = [], []
    dl = torch.as_tensor(np.random.default_rng(3).uniform(-1, 1, (3, 128, 128)),
                         dtype=torch.float32, device=device)
    for ts, ppt in RASTER_CONFIGS:
        cfg = dict(st, tile_size=ts, fwd_pixels_per_thread=ppt, bwd_pixels_per_thread=ppt)
        rend, p, imgs, saved = _render(r4d, g, views, cfg, device)
        out.append(imgs[0].cpu().numpy())
        grads.append({k: v.cpu().numpy().astype(np.float64)
                      for k, v in rend.backward(p, views, cfg, saved, [dl]).items()})
    for o in out[1:]:
        assert np.array_equal(out[0], o)
    # the per-Gaussian sums are float atomics in a different order per config
    for gr in grads[1:]:
        for k in gr:
            ref = grads[0][k]
            assert _rel(gr[k], ref) <= 1e-4, k
            assert np.all(np.abs(gr[k] - ref) <= 1e-3 * (np.abs(ref) + 1e-2 * np.abs(ref).max())), k


def test_unsupported_raster_config_is_rejected(r4d, device):
    g, views, st = W.scene_2k()
    rend = r4d.Renderer(device)
    with pytest.raises(r4d.R4DError, match="INVALID_ARG"):
        rend.forward(to_device(g, device), views, dict(st, tile_size=8, fwd_pixels_per_thread=2))


def test_ragged_image_and_multi_view(r4d, device):
    """Non-multiple-of-tile sizes; several views in one call equal one call each."""
    g, _, st = W.scene_2k()
    views = [W.view((0.0, 0.0, -4.0), 100, 70, 120.0, 0.3),
             W.view((1.0, 0.5, -3.5), 37, 53, 60.0, 0.8, bg=(0.2, 0.4, 0.6))]
    _, _, imgs, _ = _render(r4d, g, views, st, device, save=False)
    for v, im in zip(views, imgs):
        _, _, single, _ = _render(r4d, g, [v], st, device, save=False)
        assert torch.equal(im, single[0])
        ref = O.render(g, v, st)
        err, n_amb = image_errors(im.cpu().numpy().astype(np.float64), ref["image"].numpy(),
                                  ref["ambiguous"].numpy())
        assert err <= IMG_TOL and n_amb <= 0.01 * v["width"] * v["height"]


def test_empty_and_all_culled_scenes_give_background(r4d, device):
    st = W.settings()
    v = W.view((0.0, 0.0, -4.0), 40, 24, 50.0, 0.5, bg=(0.1, 0.2, 0.3))
    g0 = W.gaussians(0, 0)
    _, _, imgs, saved = _render(r4d, g0, [v], st, device)
    bg = torch.tensor([0.1, 0.2, 0.3], dtype=torch.float32).view(3, 1, 1)
    assert torch.equal(imgs[0].cpu(), bg.expand(3, 24, 40))
    # every Gaussian far outside its time window (time cull)
    g = W.gaussians(50, 0)
    g["means"][3] = 50.0
    _, _, imgs, saved = _render(r4d, g, [v], st, device)
    assert torch.equal(imgs[0].cpu(), bg.expand(3, 24, 40))
    assert saved.stats(0)["n_dup"] == 0


def test_invalid_arguments_report_errors(r4d, device):
    g, views, st = W.scene_2k()
    rend = r4d.Renderer(device)
    p = to_device(g, device)
    with pytest.raises(r4d.R4DError, match="INVALID_ARG"):
        rend.forward(p, views, dict(st, tile_size=12))
    bad = dict(views[0], width=0)
    with pytest.raises(r4d.R4DError, match="INVALID_ARG"):
        rend.forward(p, [bad], st)


def test_l1_loss_grad_matches_torch(r4d, device):
    rend = r4d.Renderer(device)
    gen = torch.Generator().manual_seed(0)
    img = torch.rand(3, 37, 53, generator=gen).to(device)
    tgt = torch.rand(3, 37, 53, generator=gen).to(device)
    tgt.view(-1)[:10] = img.view(-1)[:10]
    loss, grad = rend.l1_loss_grad(img, tgt)
    ref = torch.sign(img - tgt) / img.numel()
    assert torch.equal(grad, ref)
    assert abs(float(loss) - float((img - tgt).abs().mean())) < 1e-6


# ---------------------------------------------------------------------------
# gradients


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_gradients_fd_scene_vs_oracle(r4d, device):
    g, views, st = W.scene_fd_subset()
    weight = np.random.default_rng(2).uniform(-1, 1, (3, 32, 32))
    ref = O.render(g, views[0], st, requires_grad=True)
    (ref["image"] * torch.as_tensor(weight)).sum().backward()
    p = to_device(g, device)
    for k in ("means", "log_scales", "rotors", "opacity", "sh"):
        p[k].requires_grad_(True)
    img = r4d.render(p, views, st)[0]
    err, _ = image_errors(img.detach().cpu().numpy().astype(np.float64), ref["image"].detach().numpy(),
                          ref["ambiguous"].numpy())
    assert err <= IMG_TOL
    (img * torch.as_tensor(weight, dtype=torch.float32, device=device)).sum().backward()
    for k in ("means", "log_scales", "rotors", "opacity", "sh"):
        gg = p[k].grad.cpu().numpy().astype(np.float64)
        gr = ref["params"][k].grad.numpy()
        rel = _rel(gg, gr)
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-3, k
        assert np.all(np.abs(gg - gr) <= 1e-3 * (np.abs(gr) + 1e-2 * np.abs(gr).max()) + 1e-7), k


@pytest.mark.parametrize("k", [1, 2, 63, 65])
def test_few_visible_gaussians_vs_oracle(r4d, device, k):
    """k of 200 Gaussians left after the time cull (the others far past the
    render time): single-key and partial-wavefront segments in every stage
    (histogram, depth sort, counts, emission, tile sort, both rasterisers);
    the visible count exact, image and gradients against the oracle (the
    loss weighted off the pixels the oracle flags as ambiguous)."""
    g = W.gaussians(200, 3, xyz_half_extent=0.5)
    g["means"][3, :k] = 0.5
    g["means"][3, k:] = 50.0
    v = W.view((0.0, 0.0, -4.0), 64, 48, 60.0, 0.5)
    st = W.settings()
    print(f"case: {k} visible of 200, 64x48", flush=True)
    _, _, _, saved = _render(r4d, g, [v], st, device)
    assert saved.stats(0)["n_visible"] == k
    saved.release()
    weight = np.random.default_rng(5).uniform(-1, 1, (3, 48, 64))
    ref = O.render(g, v, st, requires_grad=True)
    weight[:, ref["ambiguous"].numpy().astype(bool)] = 0.0  # no weight where a decision is a tie
    (ref["image"] * torch.as_tensor(weight)).sum().backward()
    p = to_device(g, device)
    for key in ("means", "log_scales", "rotors", "opacity", "sh"):
        p[key].requires_grad_(True)
    img = r4d.render(p, [v], st)[0]
    err, n_amb = image_errors(img.detach().cpu().numpy().astype(np.float64),
                              ref["image"].detach().numpy(), ref["ambiguous"].numpy())
    assert err <= IMG_TOL and n_amb <= 8
    (img * torch.as_tensor(weight, dtype=torch.float32, device=device)).sum().backward()
    for key in ("means", "log_scales", "rotors", "opacity", "sh"):
        gg = p[key].grad.cpu().numpy().astype(np.float64)
        gr = ref["params"][key].grad.numpy()
        assert not np.any(gg[..., k:]) and not np.any(gr[..., k:]), key
        rel = _rel(gg, gr)
        print(f"{key}: rel {rel:.3g}")
        assert rel <= 1e-3, key


@pytest.mark.parametrize("mode", ["fused", "graph"])
@pytest.mark.parametrize("k", [0, 1, 63])
def test_empty_and_tiny_segments_in_one_call(r4d, device, mode, k):
    """Two renders in one call whose visible sets split 200 Gaussians into k
    and 200 - k (the second render's time is where the others live): empty
    and single-key segments next to full ones in the segmented sorts.  Each
    render equals the same render made alone, bit for bit, and its visible
    count is exact."""
    g = W.gaussians(200, 3, xyz_half_extent=0.5)
    g["means"][3, :k] = 0.5
    g["means"][3, k:] = 50.0
    views = [W.view((0.0, 0.0, -4.0), 64, 48, 60.0, 0.5),
             W.view((0.3, -0.2, -4.0), 56, 40, 55.0, 50.0, bg=(0.1, 0.2, 0.3))]
    st = dict(W.settings(), mode=mode)
    print(f"case: {mode}, {k} and {200 - k} visible", flush=True)
    for rep in range(2 if mode == "graph" else 1):  # a graph is captured, then replayed
        _, _, imgs, saved = _render(r4d, g, views, st, device)
        assert [saved.stats(v)["n_visible"] for v in range(2)] == [k, 200 - k]
        imgs = [i.clone() for i in imgs]
        saved.release()
        for v, im in zip(views, imgs):
            _, _, single, s1 = _render(r4d, g, [v], W.settings(), device)
            s1.release()
            assert torch.equal(im, single[0]), (rep, v["t"])


def test_degenerate_rotors_vs_oracle(r4d, device):
    """Rotors whose squared norm is below 1e-12 before the App. A update (0,
    all 1e-7) or after it (1 +- e0123 and a scaled copy) render as the
    identity rotation and get an exactly zero rotor gradient, on five
    Gaussians that contribute to the image; the rest of the scene keeps the
    oracle's image and gradients."""
    g, views, st = W.scene_fd_subset()
    weight = np.random.default_rng(2).uniform(-1, 1, (3, 32, 32))
    probe = O.render(g, views[0], st, requires_grad=True)
    (probe["image"] * torch.as_tensor(weight)).sum().backward()
    live = np.nonzero(probe["params"]["opacity"].grad.numpy())[0]
    assert live.size >= 5
    pick = live[:5]
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    rot = g["rotors"]
    rot[:, pick] = 0.0
    rot[:, pick[1]] = 1e-7
    rot[0, pick[2]], rot[7, pick[2]] = 1.0, 1.0
    rot[0, pick[3]], rot[7, pick[3]] = 1.0, -1.0
    rot[0, pick[4]], rot[7, pick[4]] = 3.0, 3.0
    print(f"case: degenerate rotors at {pick.tolist()}", flush=True)
    ref = O.render(g, views[0], st, requires_grad=True)
    (ref["image"] * torch.as_tensor(weight)).sum().backward()
    assert np.all(ref["params"]["rotors"].grad.numpy()[:, pick] == 0.0)
    p = to_device(g, device)
    for k in ("means", "log_scales", "rotors", "opacity", "sh"):
        p[k].requires_grad_(True)
    img = r4d.render(p, views, st)[0]
    err, n_amb = image_errors(img.detach().cpu().numpy().astype(np.float64),
                              ref["image"].detach().numpy(), ref["ambiguous"].numpy())
    print(f"max err {err:.3g}, ambiguous {n_amb}")
    assert err <= IMG_TOL
    (img * torch.as_tensor(weight, dtype=torch.float32, device=device)).sum().backward()
    gro = p["rotors"].grad.cpu().numpy()
    assert np.all(np.isfinite(gro))
    assert np.all(gro[:, pick] == 0.0)
    for k in ("means", "log_scales", "rotors", "opacity", "sh"):
        gg = p[k].grad.cpu().numpy().astype(np.float64)
        gr = ref["params"][k].grad.numpy()
        rel = _rel(gg, gr)
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-3, k


def test_gradients_fp64_match_central_differences(r4d, device):
    """The float64 instantiation of the same kernels: backward vs central
    differences of its own forward (h = 1e-6 max(1, |theta|))."""
    g, views, st = W.scene_fd_subset()
    g64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    weight = torch.as_tensor(np.random.default_rng(2).uniform(-1, 1, (3, 32, 32)),
                             dtype=torch.float64, device=device)
    rend = r4d.Renderer(device)
    p = to_device(g64, device, torch.float64)
    imgs, saved = rend.forward(p, views, st, save=True)
    grads = rend.backward(p, views, st, saved, [weight])
    grads = {k: v.cpu().numpy() for k, v in grads.items()}
    live = np.nonzero(grads["opacity"])[0]
    assert live.size >= 10
    rng = np.random.default_rng(5)
    checked = 0

    def loss_and_sig(pp):
        im, sv = rend.forward(pp, views, st, save=True)
        nc = sv.copy(0, r4d.BUF_NCONTRIB, 0).cpu().numpy()
        return float((im[0] * weight).sum()), nc

    for key in ("means", "log_scales", "rotors", "opacity", "sh"):
        arr = g64[key]
        for gi in rng.choice(live, size=8, replace=False):
            comp = int(rng.integers(0, arr.shape[0])) if arr.ndim == 2 else None
            idx = (comp, gi) if comp is not None else (gi,)
            theta = arr[idx]
            h = 1e-6 * max(1.0, abs(theta))
            vals = []
            sigs = []
            for sgn in (1, -1):
                q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g64.items()}
                q[key][idx] = theta + sgn * h
                l, s = loss_and_sig(to_device(q, device, torch.float64))
                vals.append(l)
                sigs.append(s)
            if not np.array_equal(sigs[0], sigs[1]):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            ad = grads[key][idx]
            assert abs(fd - ad) <= 1e-5 * max(abs(fd), abs(ad), 1e-3), (key, idx, fd, ad)
            checked += 1
    assert checked >= 25


def test_saved_state_may_outlive_its_context(r4d, device):
    """Releasing a saved state after its renderer was destroyed frees only the
    handle (the context's destroy already freed the device memory)."""
    g, views, st = W.scene_2k()
    rend = r4d.Renderer(device)
    _, saved = rend.forward(to_device(g, device), views, st, save=True)
    rend.close()
    saved.release()
    with pytest.raises(r4d.R4DError):
        saved.stats(0)


def test_binning_paths_agree_on_large_image(r4d, device):
    """A 2048x1152 frame (36,864 tiles of 8 px: tile ids need 16 radix bits,
    two full passes; 9,216 tiles of 16 px: 14 bits).  Both orders are bit-exact
    and the images identical."""
    g, _, st = W.scene_2k()
    v = W.view((0.0, 0.0, -3.0), 2048, 1152, 900.0, 0.5)
    images = []
    for ts in (8, 16):
        _, _, imgs, saved = _render(r4d, g, [v], dict(st, tile_size=ts), device)
        n = g["opacity"].shape[0]
        vals, rng, ref_vals, ref_rng, s = tile_lists(r4d, saved, 0, n)
        assert s["n_front"] == ref_vals.size > 0
        assert np.array_equal(vals, ref_vals), f"tile {ts}: order differs"
        assert np.array_equal(rng, ref_rng), f"tile {ts}: ranges differ"
        images.append(imgs[0].cpu().numpy())
    assert np.array_equal(images[0], images[1])
