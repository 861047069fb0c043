"""Pins for the oracle's EWA projection (Sec. 3.1) and spherical-harmonic
colour (Sec. 3.1).

Projection: the 2D covariance must equal (Jfd Wv) Sigma (Jfd Wv)^T + dilation I
with Jfd a finite-difference Jacobian of the pinhole map, must reduce to the
closed form for an isotropic Gaussian on the optical axis, and must match the
profile of the exact line integral of the 3D Gaussian along pixel rays for a
small far Gaussian (the affine approximation EWA makes).
SH: the basis must be orthonormal (quadrature) and equal, up to one sign per
function, to real harmonics built from scipy's complex spherical harmonics.
"""
import math

import numpy as np
import pytest
import torch

from oracle import render as O

ST = O.settings_dict({})


def _view(w=512, h=512, f=4000.0, w2c=None):
    if w2c is None:
        w2c = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)
    return {"width": w, "height": h, "fx": f, "fy": f, "cx": w / 2, "cy": h / 2,
            "world_to_cam": w2c, "t": 0.0, "bg": (0, 0, 0)}


def _rand_rotation(g):
    q, _ = np.linalg.qr(g.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


def _rand_spd(g, scale):
    A = g.normal(size=(3, 3)) * scale
    return A @ A.T + 1e-4 * scale ** 2 * np.eye(3)


def test_ewa_covariance_against_numerical_jacobian():
    g = np.random.default_rng(0)
    for _ in range(20):
        Rw = _rand_rotation(g)
        tw = g.normal(size=3) + np.array([0, 0, 6.0])
        view = _view(w2c=np.concatenate([Rw, tw[:, None]], 1), f=800.0)
        mu = g.normal(size=3) * 0.5
        cov = _rand_spd(g, 0.05)
        _, mean2, depth, cov2 = O.project_ewa(torch.as_tensor(mu)[None], torch.as_tensor(cov)[None],
                                              view, ST)
        pc = Rw @ mu + tw

        def pin(p):
            return np.array([800.0 * p[0] / p[2] + 256, 800.0 * p[1] / p[2] + 256])
        h = 1e-6
        Jfd = np.stack([(pin(pc + h * e) - pin(pc - h * e)) / (2 * h) for e in np.eye(3)], 1)
        expect = (Jfd @ Rw) @ cov @ (Jfd @ Rw).T + 0.3 * np.eye(2)
        assert np.allclose(cov2[0].numpy(), expect, rtol=1e-7, atol=1e-9)
        assert np.allclose(mean2[0].numpy(), pin(pc), atol=1e-10)
        assert abs(float(depth[0]) - pc[2]) < 1e-12


def test_isotropic_on_axis_closed_form():
    for (sigma, z, f) in ((0.05, 4.0, 1000.0), (0.01, 2.0, 150.0)):
        view = _view(128, 128, f)
        cov = torch.eye(3, dtype=torch.float64)[None] * sigma ** 2
        mu = torch.tensor([[0.0, 0.0, z]], dtype=torch.float64)
        _, mean2, _, cov2 = O.project_ewa(mu, cov, view, ST)
        expect = ((f * sigma / z) ** 2 + 0.3) * np.eye(2)
        assert np.allclose(cov2[0].numpy(), expect, rtol=1e-14)
        assert np.allclose(mean2[0].numpy(), [64, 64])


def test_projection_matches_ray_integral_profile():
    """Exact line integral of a 3D Gaussian along each pixel ray, normalised at
    the projected centre, versus the EWA profile exp(-q/2) (dilation 0)."""
    from scipy import integrate
    g = np.random.default_rng(3)
    st = dict(ST, dilation=0.0)
    view = _view()
    f = view["fx"]
    mu = np.array([0.9, -0.6, 20.0])                      # off axis: tests J's third column
    Rg = _rand_rotation(g)
    cov = Rg @ np.diag([0.004 ** 2, 0.006 ** 2, 0.05 ** 2]) @ Rg.T
    inv = np.linalg.inv(cov)
    _, mean2, _, cov2 = O.project_ewa(torch.as_tensor(mu)[None], torch.as_tensor(cov)[None], view, st)
    conic = np.linalg.inv(cov2[0].numpy())
    m2 = mean2[0].numpy()

    def ray_integral(u, v, numeric=False):
        d = np.array([(u - 256) / f, (v - 256) / f, 1.0])
        if numeric:
            fn = lambda s: math.exp(-0.5 * (s * d - mu) @ inv @ (s * d - mu))
            val, _ = integrate.quad(fn, 19.0, 21.0, epsabs=0, epsrel=1e-12, limit=200)
            return val
        a = d @ inv @ d
        b = d @ inv @ mu
        c = mu @ inv @ mu
        return math.sqrt(2 * math.pi / a) * math.exp(-0.5 * (c - b * b / a))

    i0 = ray_integral(*m2)
    assert abs(ray_integral(*m2, numeric=True) - i0) < 1e-9 * i0
    worst = 0.0
    for _ in range(300):
        dlt = g.normal(size=2) * np.sqrt(np.diag(cov2[0].numpy())) * 1.5
        q = dlt @ conic @ dlt
        if q > 9:
            continue
        ratio = ray_integral(*(m2 + dlt)) / i0
        worst = max(worst, abs(ratio - math.exp(-0.5 * q)))
    assert worst < 3e-3
    # a sign error in J's third column would move the profile by O(1e-1)
    assert worst > 0.0


# ---------------------------------------------------------------------------


def _scipy_real_sh(l, m, dirs):
    from scipy import special
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    Y = special.sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Y.real
    return math.sqrt(2) * (-1) ** m * Y.imag


def test_sh_basis_equals_scipy_real_harmonics_up_to_sign():
    g = np.random.default_rng(5)
    dirs = g.normal(size=(400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    B = O.sh_basis(torch.as_tensor(dirs), 3).numpy()
    col = 0
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _scipy_real_sh(l, m, dirs)
            sign = np.sign(np.dot(B[:, col], ref))
            assert sign != 0
            assert np.abs(B[:, col] - sign * ref).max() < 1e-12, (l, m)
            col += 1


def test_sh_basis_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for the degree-6 products
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * 2 * math.pi / 24
    ct, ph = np.meshgrid(xs, phis, indexing="ij")
    w = (ws[:, None] * np.full_like(ph, 2 * math.pi / 24)).ravel()
    stt = np.sqrt(1 - ct ** 2)
    dirs = np.stack([stt * np.cos(ph), stt * np.sin(ph), ct], -1).reshape(-1, 3)
    B = O.sh_basis(torch.as_tensor(dirs), 3).numpy()
    G = (B * w[:, None]).T @ B
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_degree_zero_colour():
    dc = torch.tensor([[[0.3, -1.0, 2.0]]], dtype=torch.float64)   # [n=1, k=1, 3]
    mu = torch.tensor([[0.1, 0.2, 0.3]], dtype=torch.float64)
    rgb = O.sh_colour(dc, 0, mu, torch.zeros(3, dtype=torch.float64))
    c0 = 0.5 / math.sqrt(math.pi)
    expect = np.maximum(0, c0 * np.array([0.3, -1.0, 2.0]) + 0.5)
    assert np.allclose(rgb[0].numpy(), expect, rtol=1e-15)
