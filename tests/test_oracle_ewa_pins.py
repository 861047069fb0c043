"""Pins for the parts of the oracle's EWA projection and compositing that the
axis-aligned closed forms leave free (Sec. 3.1, with the 3DGS conventions the
paper defers to for the projection):

* the cross term of the conic (the inverse 2D covariance) and the order of the
  camera rotation in J Wv Sigma Wv^T J^T: a strongly anisotropic Gaussian,
  rotated about the optical axis by its own rotor or by a camera roll, renders
  the closed-form image built from the rotated covariance, inverted by hand
  through its eigen-decomposition (not by a matrix inverse);
* the guard-band clamp of the projection's Jacobian: a Gaussian whose centre
  lies beyond the guard band gets the 2D covariance of J evaluated at the
  clamped x/z, y/z, written out as numbers here, and its footprint in the image
  follows that covariance;
* the whole forward on a tiny scene: six small, far, rotated Gaussians seen by
  a rolled and tilted camera match a brute-force render that integrates each
  3D density numerically along every pixel ray (peak-normalised) and
  composites front to back.

The planted-mistake tests in test_oracle_mutations.py show that a flipped cross
term, a dropped clamp or a transposed camera rotation fails these pins.
"""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import render as O

C0 = 0.5 / math.sqrt(math.pi)


def _single(xyz, o, colour, log_scales, rotor, t=0.5):
    g = {
        "means": np.array([[xyz[0]], [xyz[1]], [xyz[2]], [t]], dtype=np.float64),
        "log_scales": np.array(log_scales, dtype=np.float64).reshape(4, 1),
        "rotors": np.array(rotor, dtype=np.float64).reshape(8, 1),
        "opacity": np.array([o], dtype=np.float64),
        "sh": ((np.asarray(colour, dtype=np.float64) - 0.5) / C0).reshape(3, 1),
        "sh_degree": 0,
    }
    return g


def _view(w, h, f, w2c, t=0.5, bg=(0.0, 0.0, 0.0)):
    return {"width": w, "height": h, "fx": f, "fy": f, "cx": w / 2, "cy": h / 2,
            "world_to_cam": np.asarray(w2c, dtype=np.float64), "t": t, "bg": bg}


def _rot2(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def _closed_form_image(w, h, mean2, theta, lam, o, colour, bg):
    """Single-Gaussian image for a 2D covariance Rot(theta) diag(lam) Rot(theta)^T:
    q = u1^2/lam1 + u2^2/lam2 with u = Rot(theta)^T (p - mean2); blended when
    q <= 9 and a = min(.99, o e^{-q/2}) >= 1/255."""
    ys, xs = np.mgrid[0:h, 0:w]
    dx = xs + 0.5 - mean2[0]
    dy = ys + 0.5 - mean2[1]
    c, s = math.cos(theta), math.sin(theta)
    u1 = c * dx + s * dy
    u2 = -s * dx + c * dy
    q = u1 * u1 / lam[0] + u2 * u2 / lam[1]
    a = np.minimum(0.99, o * np.exp(-0.5 * q))
    use = (q <= 9.0) & (a >= 1.0 / 255.0)
    a = np.where(use, a, 0.0)
    img = np.stack([colour[ch] * a + bg[ch] * (1.0 - a) for ch in range(3)])
    near = (np.abs(q - 9.0) < 1e-9) | (np.abs(a - 1.0 / 255.0) < 1e-12)
    return img, q, near


def test_rotated_anisotropic_gaussian_by_rotor():
    """A rotor in the x-y plane (s, b01) = (cos th/2, -sin th/2) turns the
    Gaussian about the optical axis by th (the quaternion reduction of the rotor,
    Sec. 3.2.1); on the axis J = (f/z) [I | 0], so the 2D covariance is
    Rot(th) diag((f s_x / z)^2 + .3, (f s_y / z)^2 + .3) Rot(th)^T."""
    f, z, w, h = 150.0, 4.0, 64, 64
    sx, sy, sz = 0.2, 0.02, 0.05
    o, colour, bg = 0.85, (0.9, 0.3, 0.1), (0.05, 0.1, 0.2)
    for theta in (math.radians(30.0), math.radians(-55.0), math.radians(100.0)):
        rotor = (math.cos(theta / 2), -math.sin(theta / 2), 0, 0, 0, 0, 0, 0)
        g = _single((0.0, 0.0, z), o, colour,
                    (math.log(sx), math.log(sy), math.log(sz), math.log(0.1)), rotor)
        view = _view(w, h, f, np.concatenate([np.eye(3), np.zeros((3, 1))], 1), bg=bg)
        out = O.render(g, view, {})
        lam = ((f * sx / z) ** 2 + 0.3, (f * sy / z) ** 2 + 0.3)
        expect, q, near = _closed_form_image(w, h, (w / 2, h / 2), theta, lam, o, colour, bg)
        img = out["image"].numpy()
        assert (q <= 9).sum() > 150          # an elongated footprint of many pixels
        err = np.abs(img - expect)[:, ~near].max()
        assert err < 1e-12, (theta, err)
        # the conic itself: Rot diag(1/lam) Rot^T, off-diagonal included
        R2 = _rot2(theta)
        conic = R2 @ np.diag([1 / lam[0], 1 / lam[1]]) @ R2.T
        cn = out["pre"]["conic"][0].numpy()
        assert np.allclose(cn, [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=1e-12, atol=0)
        assert abs(conic[0, 1]) > 0.1 * max(conic[0, 0], conic[1, 1])


def test_rotated_anisotropic_gaussian_by_camera_roll():
    """An axis-aligned Gaussian seen by a camera rolled about its optical axis by
    phi (world-to-camera rotation Rot_z(phi)): its camera-space covariance is
    Rot_z(phi) diag(s^2) Rot_z(phi)^T, so the footprint turns by +phi."""
    f, z, w, h = 150.0, 4.0, 64, 64
    sx, sy, sz = 0.03, 0.25, 0.05
    o, colour, bg = 0.6, (0.2, 0.8, 0.4), (0.0, 0.0, 0.0)
    for phi in (math.radians(20.0), math.radians(-70.0)):
        Rz = np.eye(3)
        Rz[:2, :2] = _rot2(phi)
        g = _single((0.0, 0.0, z), o, colour,
                    (math.log(sx), math.log(sy), math.log(sz), math.log(0.1)),
                    (1, 0, 0, 0, 0, 0, 0, 0))
        view = _view(w, h, f, np.concatenate([Rz, np.zeros((3, 1))], 1), bg=bg)
        img = O.render(g, view, {})["image"].numpy()
        lam = ((f * sx / z) ** 2 + 0.3, (f * sy / z) ** 2 + 0.3)
        expect, q, near = _closed_form_image(w, h, (w / 2, h / 2), phi, lam, o, colour, bg)
        assert (q <= 9).sum() > 150
        assert np.abs(img - expect)[:, ~near].max() < 1e-12, phi


# The guard band: x/z and y/z enter J clamped to +-1.3 (W/2)/fx, +-1.3 (H/2)/fy.
# 128x128, f = 100: both limits are 1.3 * 64 / 100 = 0.832.


def test_guard_band_clamps_jacobian():
    view = _view(128, 128, 100.0, np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    A = np.array([[0.04, 0.01, -0.006], [0.01, 0.02, 0.004], [-0.006, 0.004, 0.03]])
    cov = torch.as_tensor(A)[None]
    # centre (3, -2.5, 2): x/z = 1.5 and y/z = -1.25, both beyond 0.832, so J is
    # taken at x' = 0.832 * 2 = 1.664, y' = -1.664:
    # J = [[100/2, 0, -100 * 1.664 / 4], [0, 100/2, 100 * 1.664 / 4]]
    J = np.array([[50.0, 0.0, -41.6], [0.0, 50.0, 41.6]])
    _, mean2, depth, cov2 = O.project_ewa(torch.tensor([[3.0, -2.5, 2.0]], dtype=torch.float64),
                                          cov, view, O.settings_dict({}))
    expect = J @ A @ J.T + 0.3 * np.eye(2)
    assert np.allclose(cov2[0].numpy(), expect, rtol=1e-13, atol=0)
    # the mean is the unclamped pinhole projection
    assert np.allclose(mean2[0].numpy(), [100 * 1.5 + 64, 100 * -1.25 + 64], rtol=0, atol=1e-12)
    # J at the unclamped x, y would differ by far more than rounding
    Jfree = np.array([[50.0, 0.0, -75.0], [0.0, 50.0, 62.5]])
    assert np.abs(Jfree @ A @ Jfree.T - expect).max() > 10.0
    # one coordinate inside, one outside: x/z = 0.5 is used as is
    # J = [[100/2, 0, -100 * 1 / 4], [0, 100/2, 100 * 1.664 / 4]]
    _, _, _, cov2b = O.project_ewa(torch.tensor([[1.0, -2.5, 2.0]], dtype=torch.float64), cov,
                                   view, O.settings_dict({}))
    Jb = np.array([[50.0, 0.0, -25.0], [0.0, 50.0, 41.6]])
    assert np.allclose(cov2b[0].numpy(), Jb @ A @ Jb.T + 0.3 * np.eye(2), rtol=1e-13, atol=0)
    # a non-square image has different limits per axis: 160 x 96, f = 100:
    # 1.3 * 80 / 100 = 1.04 in x, 1.3 * 48 / 100 = 0.624 in y; centre
    # (2, 1, 2) has x/z = 1 (inside) and y/z = 0.5 (inside), (2.4, 1.6, 2) has
    # x/z = 1.2 -> 1.04 * 2 = 2.08 and y/z = 0.8 -> 0.624 * 2 = 1.248
    v2 = _view(160, 96, 100.0, np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    _, _, _, c3 = O.project_ewa(torch.tensor([[2.4, 1.6, 2.0]], dtype=torch.float64), cov, v2,
                                O.settings_dict({}))
    Jc = np.array([[50.0, 0.0, -100 * 2.08 / 4], [0.0, 50.0, -100 * 1.248 / 4]])
    assert np.allclose(c3[0].numpy(), Jc @ A @ Jc.T + 0.3 * np.eye(2), rtol=1e-13, atol=0)


def test_guard_band_footprint_in_image():
    """A large Gaussian centred past the right guard band (x/z = 0.8 against a
    limit of 1.3 * 32 / 64 = 0.65 on a 64x64 image, f = 64, z = 2) still
    reaches into the image; its footprint there follows the clamped Jacobian
    J = [[32, 0, -64 * 1.3 / 4], [0, 32, 0]]: with Sigma = 0.09 I,
    Sigma_2D = diag(0.09 (32^2 + 20.8^2) + .3, 0.09 * 32^2 + .3)."""
    f, z, w, h = 64.0, 2.0, 64, 64
    o, colour, bg = 0.9, (1.0, 0.5, 0.0), (0.0, 0.2, 0.4)
    g = _single((1.6, 0.0, z), o, colour, (math.log(0.3),) * 3 + (math.log(0.1),),
                (1, 0, 0, 0, 0, 0, 0, 0))
    view = _view(w, h, f, np.concatenate([np.eye(3), np.zeros((3, 1))], 1), bg=bg)
    img = O.render(g, view, {})["image"].numpy()
    lam = (0.09 * (32.0 ** 2 + 20.8 ** 2) + 0.3, 0.09 * 32.0 ** 2 + 0.3)
    mean2 = (64 * 0.8 + 32, 32.0)
    expect, q, near = _closed_form_image(w, h, mean2, 0.0, lam, o, colour, bg)
    assert (q <= 9).sum() > 100              # the footprint covers the right edge
    assert np.abs(img - expect)[:, ~near].max() < 1e-12
    # the unclamped Jacobian (x' = 1.6: -64 * 1.6 / 4 = -25.6) gives another image
    lam_free = (0.09 * (32.0 ** 2 + 25.6 ** 2) + 0.3, lam[1])
    other, _, _ = _closed_form_image(w, h, mean2, 0.0, lam_free, o, colour, bg)
    assert np.abs(other - expect).max() > 0.02


# ---------------------------------------------------------------------------
# Tiny scene against brute-force ray integration


def _tiny_scene():
    """Six small far Gaussians, rotated and anisotropic, overlapping in the
    image at different depths, seen by a camera rolled and tilted away from
    the world axes.  Rotors have zero temporal part (a quaternion, pinned in
    the rotor tests) and the render is at each Gaussian's own time."""
    rng = np.random.default_rng(11)
    n = 6
    cam = np.array([0.3, -0.2, -1.0])
    # camera rotation: yaw 10 deg, pitch -8 deg, roll 25 deg
    Rwc = Rotation.from_euler("zyx", [25.0, 10.0, -8.0], degrees=True).as_matrix()
    tw = -Rwc @ cam
    means = np.zeros((4, n))
    ls = np.zeros((4, n))
    rot = np.zeros((8, n))
    depth = np.array([18.0, 19.5, 21.0, 22.5, 24.0, 25.5])
    f = 2000.0
    offs = np.array([[0.0, 0.0], [6.0, 4.0], [-5.0, 6.0], [4.0, -7.0], [-7.0, -3.0],
                     [2.0, 8.0]])                  # pixels from the image centre
    for i in range(n):
        pc = np.array([offs[i, 0] * depth[i] / f, offs[i, 1] * depth[i] / f, depth[i]])
        means[:3, i] = Rwc.T @ (pc - tw)
        means[3, i] = 0.5
        ls[:3, i] = np.log(rng.uniform(0.02, 0.07, 3))
        ls[3, i] = math.log(0.2)
        q = rng.normal(size=4)
        rot[:4, i] = q / np.linalg.norm(q)
    op = rng.uniform(0.5, 0.9, n)
    colours = rng.uniform(0, 1, (n, 3))
    g = {"means": means, "log_scales": ls, "rotors": rot, "opacity": op,
         "sh": ((colours.T - 0.5) / C0), "sh_degree": 0}
    view = _view(48, 48, f, np.concatenate([Rwc, tw[:, None]], 1), bg=(0.1, 0.15, 0.2))
    return g, view, colours, cam, Rwc, tw


def _brute_force_render(g, view, colours, cam, Rwc, tw):
    """For every pixel ray x(s) = cam + s d (d = Rwc^T K^{-1} (u, v, 1), so s is
    the camera depth), integrate each Gaussian's 3D density numerically
    (trapezoid rule over +-12 of its largest std around its depth, 4001 nodes),
    normalise by the integral along the ray through the pinhole projection of
    its centre, multiply by the opacity, and composite front to back by the
    camera depth of the centres."""
    n = g["opacity"].shape[0]
    w, h = view["width"], view["height"]
    f, cx, cy = view["fx"], view["cx"], view["cy"]
    ys, xs = np.mgrid[0:h, 0:w]
    u = (xs + 0.5).ravel()
    v = (ys + 0.5).ravel()

    def rays(uu, vv):
        dc = np.stack([(uu - cx) / f, (vv - cy) / f, np.ones_like(uu)], 1)
        return dc @ Rwc                       # rows: Rwc^T dc

    D = rays(u, v)
    alphas = np.zeros((n, u.size))
    zc = np.zeros(n)
    for i in range(n):
        s0, b01, b02, b12 = g["rotors"][:4, i]
        # quaternion (w, x, y, z) = (s, -b12, b02, -b01); scipy takes (x, y, z, w)
        R3 = Rotation.from_quat([-b12, b02, -b01, s0]).as_matrix()
        S2 = np.exp(2 * g["log_scales"][:3, i])
        inv = R3 @ np.diag(1.0 / S2) @ R3.T
        mu = g["means"][:3, i]
        pc = Rwc @ mu + tw
        zc[i] = pc[2]
        sig = math.sqrt(S2.max())
        s = np.linspace(pc[2] - 12 * sig, pc[2] + 12 * sig, 4001)

        def integral(Dr):
            X = cam[None, None, :] + s[None, :, None] * Dr[:, None, :] - mu
            e = np.einsum("psi,ij,psj->ps", X, inv, X)
            return np.trapezoid(np.exp(-0.5 * e), s, axis=1)

        u0 = f * pc[0] / pc[2] + cx
        v0 = f * pc[1] / pc[2] + cy
        peak = integral(rays(np.array([u0]), np.array([v0])))[0]
        alphas[i] = g["opacity"][i] * integral(D) / peak
    order = np.argsort(zc, kind="stable")
    T = np.ones(u.size)
    C = np.zeros((3, u.size))
    for i in order:
        C += colours[i][:, None] * alphas[i][None] * T[None]
        T *= 1.0 - alphas[i]
    C += np.asarray(view["bg"])[:, None] * T[None]
    return C.reshape(3, h, w), alphas


def test_tiny_scene_matches_ray_integration():
    g, view, colours, cam, Rwc, tw = _tiny_scene()
    # no cut-offs and no dilation: the EWA image of the densities themselves
    st = {"dilation": 0.0, "alpha_min": 1e-30, "extent_sigma": 1e3, "T_min": 1e-30}
    img = O.render(g, view, st)["image"].numpy()
    ref, alphas = _brute_force_render(g, view, colours, cam, Rwc, tw)
    # the scene is not trivial: overlapping footprints, most of the frame covered
    assert (alphas > 0.05).sum(0).max() >= 3
    assert ((alphas > 0.05).any(0)).mean() > 0.3
    err = np.abs(img - ref).max()
    # the affine (EWA) approximation of perspective is off by O(sigma/z) of the
    # profile here (sigma/z <= 4e-3; measured 6e-4)
    assert err < 2e-3, err
