"""The no-allocation forward (r4d_render_forward_noalloc), called through the
C ABI, against the allocating forward (r4d_render_forward) on the same inputs:
images equal, on two calls in a row, the second with a smaller input (fewer
Gaussians, fewer and smaller views), in fused and per-view mode.  Inputs too
large for the library's fixed region are rejected with R4D_ERR_CAPACITY, both
before anything is launched (per-Gaussian buffers) and after the preprocess
(tile lists), and the next call still renders correctly.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

from helpers import to_device

pytestmark = pytest.mark.gpu

R4D_ERR_CAPACITY = -4


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


def _views_large():
    return [W.view((0.0, 0.0, -3.0), 320, 240, 300.0, 0.5),
            W.view((2.5, -1.0, -2.0), 177, 131, 160.0, 0.2),
            W.view((-1.0, 0.5, 3.0), 200, 64, 180.0, 0.9)]


def _views_small():
    return [W.view((0.5, 0.0, -3.5), 96, 80, 110.0, 0.7)]


def _noalloc(r4d, rend, p, views, st, out):
    """Raw C-ABI call; returns the status."""
    lib = r4d.library()
    n = int(p["opacity"].shape[0])
    g = r4d._Gaussians(n, int(p["sh_degree"]), *[r4d._ptr(p[k]) for k in r4d._PARAM_KEYS])
    varr = r4d._views_array(views)
    s = r4d._settings_struct(st)
    return lib.r4d_render_forward_noalloc(rend.handle, ctypes.byref(g), varr, len(views),
                                          ctypes.byref(s), r4d._ptr(out),
                                          r4d._stream(rend.device))


def _reference(rend, p, views, st):
    imgs, _ = rend.forward(p, views, st, save=False, flat=True)
    return imgs.clone()


@pytest.mark.parametrize("mode", ["fused", "per_view"])
def test_noalloc_matches_forward_two_calls(r4d, device, mode):
    rend = r4d.Renderer(device)
    st = W.settings(mode=mode)
    cases = [(W.gaussians(20_000, 3, seed=11), _views_large()),
             (W.gaussians(3_000, 1, seed=12), _views_small())]
    for ci, (g, views) in enumerate(cases):
        print(f"case: no-alloc {mode}, call {ci}, n={g['opacity'].shape[0]}, "
              f"{len(views)} view(s)", flush=True)
        p = to_device(g, device)
        total = sum(3 * v["height"] * v["width"] for v in views)
        out = torch.full((total,), float("nan"), dtype=torch.float32, device=device)
        assert _noalloc(r4d, rend, p, views, st, out) == 0, rend_error(r4d, rend)
        ref = _reference(rend, p, views, st)
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        b = ref.cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        assert (b > 0).any()  # something was drawn
    rend.check_pending()
    rend.close()


def rend_error(r4d, rend):
    return r4d.library().r4d_last_error(rend.handle).decode()


def test_noalloc_rejects_oversized_inputs(r4d, device):
    rend = r4d.Renderer(device)
    st = W.settings(mode="fused")
    # per-Gaussian buffers beyond the region: refused before any launch
    n_big = 4_000_000
    big = {"means": torch.zeros((4, n_big), device=device),
           "log_scales": torch.zeros((4, n_big), device=device),
           "rotors": torch.zeros((8, n_big), device=device),
           "opacity": torch.zeros((n_big,), device=device),
           "sh": torch.zeros((3, n_big), device=device), "sh_degree": 0}
    views = _views_small()
    out = torch.empty((3 * 96 * 80,), device=device)
    print("case: no-alloc oversized Gaussian count", flush=True)
    assert _noalloc(r4d, rend, big, views, st, out) == R4D_ERR_CAPACITY
    assert "no-allocation region" in rend_error(r4d, rend)
    del big
    # tile lists beyond the region: refused after the preprocess
    g = W.gaussians(200_000, 0, seed=13)
    g["log_scales"][:3] += 2.0            # large footprints: many tiles each
    p = to_device(g, device)
    wide = [W.view((0.0, 0.0, -3.0), 1920, 1080, 1000.0, 0.5)]
    out = torch.empty((3 * 1920 * 1080,), device=device)
    print("case: no-alloc oversized tile lists", flush=True)
    assert _noalloc(r4d, rend, p, wide, st, out) == R4D_ERR_CAPACITY
    assert "tile entries" in rend_error(r4d, rend)
    # the region is usable again afterwards
    g2 = W.gaussians(2_000, 0, seed=14)
    p2 = to_device(g2, device)
    out2 = torch.empty((3 * 96 * 80,), device=device)
    print("case: no-alloc after a refusal", flush=True)
    assert _noalloc(r4d, rend, p2, views, st, out2) == 0, rend_error(r4d, rend)
    ref = _reference(rend, p2, views, st)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)
    rend.check_pending()
    rend.close()


def test_noalloc_argument_errors(r4d, device):
    rend = r4d.Renderer(device)
    g = W.gaussians(100, 0, seed=15)
    p = to_device(g, device)
    views = _views_small()
    out = torch.empty((3 * 96 * 80,), device=device)
    assert _noalloc(r4d, rend, p, views, W.settings(tile_size=0), out) == -1
    assert _noalloc(r4d, rend, p, views, W.settings(mode="graph"), out) == -1
    rend.close()
