"""Pins for the oracle's 4D consistency loss (Sec. 3.3, "4D Consistency Loss").

* the float32 brute-force KNN agrees with scipy's k-d tree in float64 on the
  scaled coordinates (the same index sets wherever the k-th and (k+1)-th
  distances are not within float32 reach of each other), for unit and
  non-unit scene scales;
* equal distances are ranked by index, and a Gaussian is not its own
  neighbour (hand-built lattice);
* on a line of x-t rotors with hand-derived speeds cos(phi) sin(phi)
  (s_t^2 - s_x^2) / W (the survey's x-t rotation: R00 = R33 = cos phi,
  R03 = -R30 = sin phi), the neighbour lists and the loss equal their values
  worked out by hand;
* Gaussians without a temporal rotor part do not move: loss and gradient 0;
* the autograd gradient equals central differences.
"""

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import workloads as W
from oracle import consistency as C
from oracle import render as O


@pytest.mark.parametrize("scales", [(1.0, 1.0), (2.0, 0.25)])
def test_knn_matches_kdtree(scales):
    g = W.gaussians(3000, 0)
    k = 8
    nb = C.knn4d(g["means"], k, *scales)
    u = g["means"].astype(np.float64).T / np.array([scales[0]] * 3 + [scales[1]])
    dist, idx = cKDTree(u).query(u, k=k + 2)
    agree = gapped = 0
    for i in range(u.shape[0]):
        d, j = dist[i], idx[i]
        keep = j != i
        d, j = d[keep][:k + 1], j[keep][:k + 1]
        if d[k] - d[k - 1] > 1e-5 * d[k]:
            gapped += 1
            agree += set(j[:k].tolist()) == set(nb[i].tolist())
        # the oracle's ranks come in increasing distance
        dn = np.linalg.norm(u[nb[i]] - u[i], axis=1)
        assert np.all(np.diff(dn) >= -1e-6 * dn[1:])
        assert i not in nb[i]
    assert gapped >= 0.99 * u.shape[0]
    assert agree == gapped


def test_knn_ties_by_index_and_no_self():
    # points on a lattice: 0 at the origin, 1..4 at distance 1 (equal), 5 at 2
    pts = np.array([[0, 0, 0, 0], [1, 0, 0, 0], [0, -1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
                    [2, 0, 0, 0]], dtype=np.float32).T
    nb = C.knn4d(pts, 3)
    assert nb[0].tolist() == [1, 2, 3]
    # from 1: the origin (1), then 5 (1) -- tie, index order -- then 2, 3, 4 (sqrt 2)
    assert nb[1].tolist() == [0, 5, 2]
    # duplicates: distance 0 to each other, ranked by index
    dup = np.zeros((4, 5), dtype=np.float32)
    dup[0, 4] = 3.0
    nb = C.knn4d(dup, 3)
    assert nb[2].tolist() == [0, 1, 3]
    assert nb[4].tolist() == [0, 1, 2]


def _xt_line(thetas, sx=0.08, st=0.3):
    n = len(thetas)
    g = W.gaussians(n, 0)
    g["means"][:] = 0.0
    g["means"][0] = np.arange(n, dtype=np.float32)
    g["means"][3] = 0.5
    g["log_scales"][:] = np.log(np.array([sx, 0.05, 0.05, st], dtype=np.float32))[:, None]
    g["rotors"][:] = 0.0
    g["rotors"][0] = np.cos(thetas)
    g["rotors"][4] = np.sin(thetas)          # b03: the x-t plane
    return g


def test_loss_closed_form_on_a_line_of_xt_rotors():
    thetas = np.array([0.1, -0.35, 0.5, 0.2, -0.15, 0.4])
    sx, st = 0.08, 0.3
    g = _xt_line(thetas, sx, st)
    nb = C.knn4d(g["means"], 2)
    assert nb.tolist() == [[1, 2], [0, 2], [1, 3], [2, 4], [3, 5], [4, 3]]
    # the stored (float32) rotor angles and scales
    phi = 2 * np.arctan2(g["rotors"][4].astype(np.float64), g["rotors"][0].astype(np.float64))
    sx, st = np.exp(g["log_scales"][0, 0].astype(np.float64)), np.exp(g["log_scales"][3, 0].astype(np.float64))
    w = np.sin(phi) ** 2 * sx ** 2 + np.cos(phi) ** 2 * st ** 2
    v = np.cos(phi) * np.sin(phi) * (st ** 2 - sx ** 2) / w
    lists = [[1, 2], [0, 2], [1, 3], [2, 4], [3, 5], [4, 3]]
    expect = np.mean([abs(v[i] - 0.5 * (v[a] + v[b])) for i, (a, b) in enumerate(lists)])
    P = O.params_to_torch(g)
    sp = C.speeds(P).numpy()
    assert np.abs(sp[:, 0] - v).max() < 1e-12 * np.abs(v).max()
    assert np.abs(sp[:, 1:]).max() < 1e-15
    loss = float(C.consistency_loss(P, nb))
    assert abs(loss - expect) < 1e-12 * expect


def test_static_gaussians_have_zero_loss_and_gradient():
    g = W.gaussians(200, 0)
    g["rotors"][4:] = 0.0                    # no x-t, y-t, z-t or e0123 part
    nb = C.knn4d(g["means"], 8)
    P = O.params_to_torch(g, requires_grad=True)
    loss = C.consistency_loss(P, nb)
    assert float(loss) == 0.0
    loss.backward()
    # |.| has no derivative at 0; torch takes 0 there
    assert float(P["rotors"].grad.abs().max()) == 0.0
    assert float(P["log_scales"].grad.abs().max()) == 0.0


def test_gradient_matches_central_differences():
    g = W.gaussians(60, 0)
    nb = C.knn4d(g["means"], 4)
    P = O.params_to_torch(g, requires_grad=True)
    C.consistency_loss(P, nb).backward()
    rng = np.random.default_rng(3)
    for key, rows in (("rotors", 8), ("log_scales", 4)):
        for _ in range(8):
            idx = (int(rng.integers(0, rows)), int(rng.integers(0, 60)))
            h = 1e-6

            def val(dv):
                P2 = O.params_to_torch(g)
                with torch.no_grad():
                    P2[key][idx] += dv
                return float(C.consistency_loss(P2, nb))
            fd = (val(h) - val(-h)) / (2 * h)
            ad = float(P[key].grad[idx])
            assert abs(fd - ad) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, ad)
    # the means only choose the neighbours: no gradient reaches them
    assert P["means"].grad is None or float(P["means"].grad.abs().max()) == 0.0
