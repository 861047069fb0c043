"""Parity of the 4D KNN and the 4D consistency loss (Sec. 3.3) of the HIP path
with the CPU oracle.

* KNN: bit-exact neighbour lists (index order included) against the oracle's
  float32 brute force, which takes the same float32 decisions -- for several
  sizes, k, scene scales, exact ties, duplicates and degenerate layouts; at
  500k (the headline scene) on sampled queries.
* Loss (float32 GPU vs FP64 oracle, the same neighbour lists): relative 1e-5;
  gradients per parameter group ||g - g_ref|| / ||g_ref|| <= 1e-4, and
  elementwise |g - g_ref| <= 1e-3 (|g_ref| + 0.01 max |g_ref|) as for the
  render gradients, on every Gaussian not touched by a sign decision within float32
  reach of 0 (|d| <= 1e-4 of the speeds it is formed from); the float64
  instantiation matches central differences of its own loss.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import consistency as C
from oracle import render as O

from helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def r4d():
    import paper_2402_03307_amd as mod
    return mod


@pytest.fixture(scope="module")
def rend(r4d, device):
    return r4d.Renderer(device)


def _knn_gpu(rend, means, k, ss=1.0, ts=1.0):
    m = torch.as_tensor(np.ascontiguousarray(means, dtype=np.float32)).to(rend.device)
    out = rend.knn4d(m, k, ss, ts)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("n,k,scales", [(3000, 8, (1.0, 1.0)), (20000, 8, (1.0, 1.0)),
                                        (5000, 8, (2.0, 0.25)), (2000, 1, (1.0, 1.0)),
                                        (2000, 5, (1.0, 1.0)), (2000, 16, (0.5, 3.0)),
                                        (1500, 32, (1.0, 1.0))])
def test_knn_bit_exact(rend, n, k, scales):
    print(f"case: knn n={n} k={k} scales={scales}", flush=True)
    g = W.gaussians(n, 0)
    got = _knn_gpu(rend, g["means"], k, *scales)
    ref = C.knn4d(g["means"], k, *scales)
    bad = np.nonzero((got != ref).any(1))[0]
    assert bad.size == 0, (bad[:5], got[bad[:2]], ref[bad[:2]])


def test_knn_ties_duplicates_and_degenerate_layouts(rend):
    rng = np.random.default_rng(11)
    # a coarse lattice: many exactly equal distances, ranked by index
    lat = rng.integers(0, 6, size=(4, 3000)).astype(np.float32) * np.float32(0.25)
    assert np.array_equal(_knn_gpu(rend, lat, 8), C.knn4d(lat, 8))
    # exact duplicates of a few points
    base = rng.uniform(-1, 1, size=(4, 40)).astype(np.float32)
    dup = base[:, rng.integers(0, 40, size=1200)]
    assert np.array_equal(_knn_gpu(rend, dup, 8), C.knn4d(dup, 8))
    # all points equal: the k smallest other indices
    same = np.ones((4, 100), dtype=np.float32)
    got = _knn_gpu(rend, same, 4)
    assert np.array_equal(got, C.knn4d(same, 4))
    assert got[0].tolist() == [1, 2, 3, 4] and got[3].tolist() == [0, 1, 2, 4]
    # points on a 2D plane (two coordinates constant), and on a line in t
    plane = rng.uniform(-1, 1, size=(4, 2500)).astype(np.float32)
    plane[1] = 0.3
    plane[3] = 0.5
    assert np.array_equal(_knn_gpu(rend, plane, 8), C.knn4d(plane, 8))
    line = np.zeros((4, 800), dtype=np.float32)
    line[3] = rng.uniform(0, 1, size=800).astype(np.float32)
    assert np.array_equal(_knn_gpu(rend, line, 6), C.knn4d(line, 6))
    # one far outlier stretches the grid
    out = rng.uniform(-1, 1, size=(4, 3000)).astype(np.float32)
    out[:, 17] = (50.0, -40.0, 30.0, 20.0)
    assert np.array_equal(_knn_gpu(rend, out, 8), C.knn4d(out, 8))
    # the smallest case: n = k + 1
    tiny = rng.uniform(-1, 1, size=(4, 9)).astype(np.float32)
    assert np.array_equal(_knn_gpu(rend, tiny, 8), C.knn4d(tiny, 8))


def test_knn_full_size_sampled(rend):
    g, _, _ = W.scene_500k_step()
    print("case: knn 500k k=8 (sampled queries)", flush=True)
    got = _knn_gpu(rend, g["means"], 8)
    assert got.shape == (500_000, 8)
    q = np.random.default_rng(12).choice(500_000, size=192, replace=False)
    ref = C.knn4d(g["means"], 8, queries=q, chunk=8)
    assert np.array_equal(got[q], ref)
    # properties at every point: in range, no self, no repeats
    assert got.min() >= 0 and got.max() < 500_000
    assert not (got == np.arange(500_000)[:, None]).any()
    s = np.sort(got, axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()


def test_knn_rejects_bad_arguments(r4d, rend):
    m = torch.zeros(4, 10, dtype=torch.float32, device=rend.device)
    for k, ss in ((0, 1.0), (10, 1.0), (33, 1.0), (4, 0.0), (4, float("nan"))):
        with pytest.raises(r4d.R4DError):
            rend.knn4d(m, k, ss, 1.0)


def _ambiguous_gaussians(P, nb, rel=1e-4):
    """Gaussians whose gradient depends on a sign(d) decision within float32
    reach of 0: i itself and its neighbours, for every such component."""
    s = C.speeds(P).detach().numpy()
    m = s[nb].mean(axis=1)
    d = s - m
    mag = np.abs(s) + np.abs(s[nb]).mean(axis=1)
    amb = (np.abs(d) <= rel * mag).any(axis=1)
    touched = np.zeros(s.shape[0], dtype=bool)
    idx = np.nonzero(amb)[0]
    touched[idx] = True
    touched[nb[idx].reshape(-1)] = True
    return touched


def test_loss_and_gradients_vs_oracle(rend, device):
    g = W.gaussians(4000, 1)
    nb = C.knn4d(g["means"], 8)
    P = O.params_to_torch(g, requires_grad=True)
    ref = C.consistency_loss(P, nb)
    ref.backward()
    p = to_device(g, device)
    w = 0.05
    grads = {k: torch.zeros_like(p[k]) for k in ("rotors", "log_scales")}
    loss, grads = rend.consistency4d(p, torch.as_tensor(nb).to(device), w, grads)
    torch.cuda.synchronize()
    assert abs(float(loss) - float(ref)) <= 1e-5 * float(ref)
    skip = _ambiguous_gaussians(P, nb)
    print(f"loss {float(loss):.6g} vs {float(ref):.6g}; ambiguous Gaussians {int(skip.sum())}")
    assert skip.sum() <= 0.01 * 4000
    for k in ("rotors", "log_scales"):
        gg = grads[k].cpu().numpy().astype(np.float64)[:, ~skip]
        gr = w * P[k].grad.numpy()[:, ~skip]
        rel = float(np.linalg.norm(gg - gr) / np.linalg.norm(gr))
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-4, k
        assert np.all(np.abs(gg - gr) <= 1e-3 * (np.abs(gr) + 1e-2 * np.abs(gr).max())), k
    # the gradient is added: a second call doubles it
    before = {k: v.clone() for k, v in grads.items()}
    rend.consistency4d(p, torch.as_tensor(nb).to(device), w, grads)
    for k in grads:
        assert torch.allclose(grads[k], 2 * before[k], rtol=1e-6, atol=0)


@pytest.mark.parametrize("n", [5000, 1_100_000])
def test_loss_with_arbitrary_lists_both_sign_sum_paths(rend, device, n):
    """Any neighbour lists (seeded random, repeats allowed) through the packed
    sign sums (n <= 2^20) and the per-component ones (n > 2^20)."""
    print(f"case: consistency n={n} random lists", flush=True)
    g = W.gaussians(n, 0)
    nb = np.random.default_rng(14).integers(0, n, size=(n, 8))
    P = O.params_to_torch(g, requires_grad=True)
    ref = C.consistency_loss(P, nb)
    ref.backward()
    p = to_device(g, device)
    loss, grads = rend.consistency4d(p, torch.as_tensor(nb).to(device), 1.0)
    torch.cuda.synchronize()
    assert abs(float(loss) - float(ref)) <= 1e-5 * float(ref)
    skip = _ambiguous_gaussians(P, nb)
    assert skip.sum() <= 0.01 * n
    for k in ("rotors", "log_scales"):
        gg = grads[k].cpu().numpy().astype(np.float64)[:, ~skip]
        gr = P[k].grad.numpy()[:, ~skip]
        rel = float(np.linalg.norm(gg - gr) / np.linalg.norm(gr))
        print(f"{k}: rel {rel:.3g}")
        assert rel <= 1e-4, k


def test_gpu_neighbours_feed_the_loss(rend, device):
    """KNN and loss chained on the device, as a training step would: the
    result equals the oracle with its own neighbour lists."""
    g = W.gaussians(6000, 0)
    p = to_device(g, device)
    nb = rend.knn4d(p["means"], 8, 1.0, 1.0)
    loss, _ = rend.consistency4d(p, nb, 1.0, need_grad=False)
    ref = C.consistency_loss(O.params_to_torch(g), C.knn4d(g["means"], 8))
    assert abs(float(loss) - float(ref)) <= 1e-5 * float(ref)


def test_static_gaussians_zero_loss_and_gradient(rend, device):
    g = W.gaussians(500, 0)
    g["rotors"][4:] = 0.0
    p = to_device(g, device)
    nb = rend.knn4d(p["means"], 8)
    loss, grads = rend.consistency4d(p, nb, 1.0)
    assert float(loss) == 0.0
    assert float(grads["rotors"].abs().max()) == 0.0
    assert float(grads["log_scales"].abs().max()) == 0.0


def test_fp64_gradient_matches_central_differences(rend, device):
    g = W.gaussians(300, 0)
    g64 = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    nb = torch.as_tensor(C.knn4d(g["means"], 8)).to(device)
    p = to_device(g64, device, torch.float64)
    _, grads = rend.consistency4d(p, nb, 1.0)
    grads = {k: v.cpu().numpy() for k, v in grads.items()}
    rng = np.random.default_rng(13)

    def loss_of(q):
        return float(rend.consistency4d(to_device(q, device, torch.float64), nb, 1.0,
                                        need_grad=False)[0])

    nb_np = nb.cpu().numpy()

    def residual_signs(q):
        # signs of every residual component s_i - mean_j s_j (oracle, FP64):
        # |.| has a kink where one of them changes sign
        sp = C.speeds(O.params_to_torch(q))
        return torch.sign(sp - sp[torch.as_tensor(nb_np)].mean(dim=1)).numpy()

    for key, rows in (("rotors", 8), ("log_scales", 4)):
        for _ in range(12):
            idx = (int(rng.integers(0, rows)), int(rng.integers(0, 300)))
            h = 1e-6 * max(1.0, abs(g64[key][idx]))
            # shrink h until no residual changes sign inside [theta - h, theta + h]
            while True:
                qs = []
                for sgn in (1, -1):
                    q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g64.items()}
                    q[key][idx] += sgn * h
                    qs.append(q)
                if np.array_equal(residual_signs(qs[0]), residual_signs(qs[1])) or h < 1e-11:
                    break
                h *= 0.1
            assert np.array_equal(residual_signs(qs[0]), residual_signs(qs[1])), (key, idx)
            fd = (loss_of(qs[0]) - loss_of(qs[1])) / (2 * h)
            ad = grads[key][idx]
            # rounding of the FP64 loss (about 1, a mean of 900 terms) over 2h
            roundoff = 1e-15 / h
            assert abs(fd - ad) <= 1e-5 * max(abs(fd), abs(ad), 1e-3) + roundoff, (key, idx, fd, ad, h)
