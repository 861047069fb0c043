"""Pins for the oracle's temporal slicing (Sec. 3.2.2, Eq. center-motion; App. A).

The slice is pinned to the definition it abbreviates: a 4D Gaussian density
restricted to the hyperplane at time t factors into a temporal term times a 3D
Gaussian.  The test evaluates the 4D density with an explicit numpy inverse of
Sigma_4 and compares it with exp(-lambda dt^2/2) * G_3D(x; mu(t), Sigma_3D).
"""
import math

import numpy as np
import torch

from oracle import render as O


def _random_gaussians(n, seed):
    g = np.random.default_rng(seed)
    mu4 = torch.as_tensor(np.concatenate([g.uniform(-1, 1, (n, 3)), g.uniform(0, 1, (n, 1))], 1))
    ls = torch.as_tensor(np.concatenate([g.normal(-3, .5, (n, 3)), g.normal(-1.5, .5, (n, 1))], 1))
    r = torch.as_tensor(g.normal(size=(n, 8)))
    R = O.rotor_to_matrix(O.rotor_normalize(r))
    cov4 = O.covariance_4d(R, ls)
    return mu4, ls, R, cov4


def test_covariance_factorisation():
    mu4, ls, R, cov4 = _random_gaussians(200, 0)
    s2 = torch.exp(2 * ls)
    # eigenvalues of Sigma_4 are the squared scales
    ev = torch.linalg.eigvalsh(cov4)
    assert torch.allclose(torch.sort(ev, -1).values, torch.sort(s2, -1).values, rtol=1e-10, atol=0)


def test_slice_matches_4d_density():
    mu4, ls, R, cov4 = _random_gaussians(100, 1)
    g = np.random.default_rng(11)
    for t in (0.1, 0.5, 0.93):
        mu3, cov3, lam_dt2, decay = O.slice_at_time(mu4, cov4, t)
        for i in range(mu4.shape[0]):
            S4 = cov4[i].numpy()
            inv4 = np.linalg.inv(S4)
            inv3 = np.linalg.inv(cov3[i].numpy())
            for _ in range(4):
                x = mu3[i].numpy() + g.normal(scale=0.05, size=3)
                d4 = np.concatenate([x, [t]]) - mu4[i].numpy()
                g4 = math.exp(-0.5 * d4 @ inv4 @ d4)
                d3 = x - mu3[i].numpy()
                g3 = float(decay[i]) * math.exp(-0.5 * d3 @ inv3 @ d3)
                assert abs(g4 - g3) <= 1e-9 * max(g4, 1e-300) + 1e-300


def test_schur_complement_equals_inverse_of_precision_block():
    mu4, ls, R, cov4 = _random_gaussians(300, 2)
    _, cov3, _, _ = O.slice_at_time(mu4, cov4, 0.5)
    A = torch.linalg.inv(cov4)[:, :3, :3]
    assert torch.allclose(torch.linalg.inv(A), cov3, rtol=1e-9, atol=1e-15)
    # det Sigma_4 = W det Sigma_3D
    W = cov4[:, 3, 3]
    assert torch.allclose(torch.linalg.det(cov4), W * torch.linalg.det(cov3), rtol=1e-9, atol=0)
    # lambda = 1/W equals the temporal precision left after the spatial part
    Z = torch.linalg.inv(cov4)[:, 3, 3]
    Mv = torch.linalg.inv(cov4)[:, :3, 3]
    lam = Z - (Mv[:, None, :] @ torch.linalg.solve(A, Mv[:, :, None]))[:, 0, 0]
    assert torch.allclose(lam, 1.0 / W, rtol=1e-9)


def test_motion_is_linear_and_opacity_peaks_at_mu_t():
    mu4, ls, R, cov4 = _random_gaussians(50, 3)
    ts = [0.0, 0.25, 0.5, 0.75, 1.0]
    mus = [O.slice_at_time(mu4, cov4, t)[0] for t in ts]
    vel = (mus[1] - mus[0]) / 0.25
    for t, m in zip(ts, mus):
        assert torch.allclose(m, mus[0] + t * vel, atol=1e-12)
    _, _, _, decay_at_mu = O.slice_at_time(mu4, cov4, 0.0)
    for i in range(5):
        mu3, _, lam, dec = O.slice_at_time(mu4[i:i + 1], cov4[i:i + 1], float(mu4[i, 3]))
        assert abs(float(dec[0]) - 1.0) < 1e-15 and float(lam[0]) == 0.0
        assert torch.allclose(mu3[0], mu4[i, :3], atol=1e-15)


def test_uncorrelated_gaussian_is_static():
    # V = 0: static 3D Gaussian with Gaussian-in-t opacity of std s_t
    n = 20
    g = np.random.default_rng(4)
    q = g.normal(size=(n, 4))
    r = torch.zeros(n, 8, dtype=torch.float64)
    r[:, :4] = torch.as_tensor(q)
    ls = torch.as_tensor(g.normal(-2, .5, (n, 4)))
    mu4 = torch.as_tensor(g.uniform(0, 1, (n, 4)))
    cov4 = O.covariance_4d(O.rotor_to_matrix(O.rotor_normalize(r)), ls)
    for t in (0.0, 0.6):
        mu3, cov3, lam_dt2, decay = O.slice_at_time(mu4, cov4, t)
        assert torch.allclose(mu3, mu4[:, :3], atol=1e-15)
        assert torch.allclose(cov3, cov4[:, :3, :3], atol=1e-15)
        st = torch.exp(ls[:, 3])
        expect = torch.exp(-0.5 * ((t - mu4[:, 3]) / st) ** 2)
        assert torch.allclose(decay, expect, rtol=1e-12)


def test_xt_rotor_closed_form():
    # rotor (cos th, b03 = sin th): rotation by phi = 2 th in the x-t plane.  By hand:
    # W = sin^2 phi sx^2 + cos^2 phi st^2,  V_x = cos phi sin phi (st^2 - sx^2),
    # Sigma_3D,xx = sx^2 st^2 / W, the y, z axes untouched.
    for th in (0.2, 0.7, 1.3):
        for (sx, sy, sz, st_) in ((0.05, 0.07, 0.03, 0.2), (0.3, 0.1, 0.2, 0.02)):
            r = torch.zeros(1, 8, dtype=torch.float64)
            r[0, 0], r[0, 4] = math.cos(th), math.sin(th)
            ls = torch.log(torch.tensor([[sx, sy, sz, st_]], dtype=torch.float64))
            cov4 = O.covariance_4d(O.rotor_to_matrix(O.rotor_normalize(r)), ls)
            mu4 = torch.zeros(1, 4, dtype=torch.float64)
            mu3, cov3, lam_dt2, _ = O.slice_at_time(mu4, cov4, 0.1)
            phi = 2 * th
            W = math.sin(phi) ** 2 * sx ** 2 + math.cos(phi) ** 2 * st_ ** 2
            vx = math.cos(phi) * math.sin(phi) * (st_ ** 2 - sx ** 2) / W
            assert abs(float(mu3[0, 0]) - 0.1 * vx) < 1e-14
            assert abs(float(cov3[0, 0, 0]) - sx ** 2 * st_ ** 2 / W) < 1e-14
            assert abs(float(cov3[0, 1, 1]) - sy ** 2) < 1e-15
            assert abs(float(cov3[0, 2, 2]) - sz ** 2) < 1e-15
            assert abs(float(lam_dt2[0]) - 0.01 / W) < 1e-12 * (0.01 / W)
