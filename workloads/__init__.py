"""Seeded synthetic inputs for the 4D-rotor Gaussian renderer.

This module only draws random numbers and builds camera poses; it holds none
of the renderer's arithmetic.  Both the FP64 CPU oracle and the HIP library are
fed from here, so the two sides see bit-identical FP32 inputs.

Layouts (all float32, component-major "SoA": element (c, i) at arr[c, i]):
  means      [4, n]    x, y, z, t
  log_scales [4, n]    log s_x, log s_y, log s_z, log s_t
  rotors     [8, n]    s, b01, b02, b12, b03, b13, b23, p  (raw, unnormalised;
                       the component order of the rotor definition in
                       Sec. 3.2.1 of the paper)
  opacity    [n]       already activated, in (0, 1)
  sh         [3k, n]   row = coefficient * 3 + channel, k = (degree + 1)^2

A view is a dict: width, height, fx, fy, cx, cy, world_to_cam (3x4 row-major
[R|t], OpenCV axes: x right, y down, z forward), t (time), bg (3 floats).

Draw order and distributions follow the synthetic stand-ins for the paper's
workloads (Plenoptic 1352x1014, HyperNeRF 960x540): numpy PCG64 generators,
Gaussian seed 0, camera seed 1, target/pixel-sample seed 2, draws made in
float64 and rounded to float32.
"""
from __future__ import annotations

import math

import numpy as np

GAUSSIAN_SEED = 0
CAMERA_SEED = 1
TARGET_SEED = 2
PIXEL_SAMPLE_SEED = 7

# Degree-0 real spherical-harmonic constant 1/(2 sqrt(pi)); used only to encode
# a desired base colour c as a DC coefficient (c - 0.5) / Y00 for the 2k scene.
_Y00 = 0.28209479177387814


def sh_coeffs(degree: int) -> int:
    return (degree + 1) ** 2


def gaussians(n: int, sh_degree: int, *, seed: int = GAUSSIAN_SEED,
              xyz_half_extent: float = 1.0, base_colour_dc: bool = False) -> dict:
    """Draw n 4D Gaussians.

    Draw order: mu_xyz, mu_t, log s_xyz, log s_t, q1 (rotor[0:4]), q2 (rotor[4:8]),
    opacity logits, SH DC, SH rest.
    mu_xyz ~ U[-e, e]^3, mu_t ~ U[0,1], log s_xyz ~ N(-3, .5), log s_t ~ N(-1.5, .5),
    q1, q2 ~ normalise(N(0, I4)), opacity = sigmoid(N(0,1)).
    base_colour_dc: colour c ~ U[0,1]^3 encoded as DC = (c - .5)/Y00 (degree 0
    scene); otherwise DC ~ U[0,1] and higher bands ~ N(0, 0.05).
    """
    rng = np.random.default_rng(seed)
    k = sh_coeffs(sh_degree)
    mu_xyz = rng.uniform(-xyz_half_extent, xyz_half_extent, size=(3, n))
    mu_t = rng.uniform(0.0, 1.0, size=(1, n))
    ls_xyz = rng.normal(-3.0, 0.5, size=(3, n))
    ls_t = rng.normal(-1.5, 0.5, size=(1, n))
    q1 = rng.normal(0.0, 1.0, size=(4, n))
    q1 /= np.linalg.norm(q1, axis=0, keepdims=True)
    q2 = rng.normal(0.0, 1.0, size=(4, n))
    q2 /= np.linalg.norm(q2, axis=0, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=n)
    opacity = 1.0 / (1.0 + np.exp(-logits))
    sh = np.zeros((k, 3, n))
    if base_colour_dc:
        colour = rng.uniform(0.0, 1.0, size=(3, n))
        sh[0] = (colour - 0.5) / _Y00
    else:
        sh[0] = rng.uniform(0.0, 1.0, size=(3, n))
        if k > 1:
            sh[1:] = rng.normal(0.0, 0.05, size=(k - 1, 3, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {
        "means": f32(np.concatenate([mu_xyz, mu_t], axis=0)),
        "log_scales": f32(np.concatenate([ls_xyz, ls_t], axis=0)),
        "rotors": f32(np.concatenate([q1, q2], axis=0)),
        "opacity": f32(opacity),
        "sh": f32(sh.reshape(3 * k, n)),
        "sh_degree": int(sh_degree),
    }


def static_gaussians(n: int, sh_degree: int, *, seed: int = GAUSSIAN_SEED,
                     xyz_half_extent: float = 1.0) -> dict:
    """Draw n static 3D Gaussians (a 3D Gaussian Splatting scene).

    Draw order: mu ~ U[-e, e]^3, log s ~ N(-3, .5)^3, q ~ N(0, I4) (stored as
    drawn, (w, x, y, z)), opacity = sigmoid(N(0,1)), SH DC ~ U[0,1], higher
    bands ~ N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    k = sh_coeffs(sh_degree)
    mu = rng.uniform(-xyz_half_extent, xyz_half_extent, size=(3, n))
    ls = rng.normal(-3.0, 0.5, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))
    sh = np.zeros((k, 3, n))
    sh[0] = rng.uniform(0.0, 1.0, size=(3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, 0.05, size=(k - 1, 3, n))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {"means": f32(mu), "log_scales": f32(ls), "quats": f32(q), "opacity": f32(opacity),
            "sh": f32(sh.reshape(3 * k, n)), "sh_degree": int(sh_degree)}


def scene_static_500k(n: int = 500_000):
    """500k static 3D Gaussians, SH degree 3, 1352x1014, f=1000, camera (0,0,-4)."""
    g = static_gaussians(n, 3)
    v = view(orbit_position(0), 1352, 1014, 1000.0, 0.5)
    return g, [v], settings()


def subset(g: dict, count: int) -> dict:
    """The first `count` Gaussians of a set (used for the finite-difference scene)."""
    out = {key: (np.ascontiguousarray(v[..., :count]) if isinstance(v, np.ndarray) else v)
           for key, v in g.items()}
    return out


def look_at(position, target=(0.0, 0.0, 0.0), world_down=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World-to-camera [R|t] (3x4) for a camera at `position` looking at `target`.

    OpenCV axes: camera z points at the target, y is world "down" (+y, i.e. world
    up is (0,-1,0)) projected orthogonally, x = y cross z.
    """
    c = np.asarray(position, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - c
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(world_down, dtype=np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    rot = np.stack([x, y, z], axis=0)
    trans = -rot @ c
    return np.concatenate([rot, trans[:, None]], axis=1)


def view(position, width: int, height: int, focal: float, t: float,
         bg=(0.0, 0.0, 0.0)) -> dict:
    w2c = look_at(position)
    return {
        "width": int(width), "height": int(height),
        "fx": float(focal), "fy": float(focal),
        "cx": width / 2.0, "cy": height / 2.0,
        "world_to_cam": np.asarray(w2c, dtype=np.float32),
        "t": float(np.float32(t)),
        "bg": tuple(float(b) for b in bg),
    }


def orbit_position(k: int, count: int = 30, radius: float = 4.0):
    phi = 2.0 * math.pi * k / count
    return (radius * math.sin(phi), 0.0, -radius * math.cos(phi))


def target_image(height: int, width: int, seed: int = TARGET_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(3, height, width)), dtype=np.float32)


def pixel_sample(height: int, width: int, count: int = 4096,
                 seed: int = PIXEL_SAMPLE_SEED) -> np.ndarray:
    """Fixed random sample of distinct pixel indices (row-major y*W+x), sorted."""
    rng = np.random.default_rng(seed)
    count = min(count, height * width)
    return np.sort(rng.choice(height * width, size=count, replace=False)).astype(np.int64)


# ---------------------------------------------------------------------------
# Named workloads.  Each returns (gaussians, [views], settings-overrides).

DEFAULT_SETTINGS = {
    "tile_size": 16,
    "near_plane": 0.2,
    "time_cull": 16.0,
    "extent_sigma": 3.0,
    "alpha_min": 1.0 / 255.0,
    "alpha_max": 0.99,
    "T_min": 1e-4,
    "dilation": 0.3,
    "guard_band": 1.3,
}


def settings(**overrides) -> dict:
    s = dict(DEFAULT_SETTINGS)
    s.update(overrides)
    return s


def scene_2k():
    """2,000 Gaussians, SH degree 0, 128x128, camera at (0,0,-4), f=150, t=0.5."""
    g = gaussians(2000, 0, base_colour_dc=True)
    v = view((0.0, 0.0, -4.0), 128, 128, 150.0, 0.5)
    return g, [v], settings()


def scene_300k_orbit(n: int = 300_000):
    """300k Gaussians, SH degree 3, 1352x1014, f=1000, 30 orbit views, t in linspace(0,1,30)."""
    g = gaussians(n, 3)
    ts = np.linspace(0.0, 1.0, 30)
    views = [view(orbit_position(k), 1352, 1014, 1000.0, ts[k]) for k in range(30)]
    return g, views, settings()


def scene_500k_step(n: int = 500_000):
    """500k Gaussians, SH degree 3, 1352x1014, f=1000, camera (0,0,-4), t=0.5."""
    g = gaussians(n, 3)
    v = view(orbit_position(0), 1352, 1014, 1000.0, 0.5)
    return g, [v], settings()


def scene_fd_subset(count: int = 64):
    """First 64 Gaussians of the 500k scene, camera (0,0,-4), f=40, 32x32, t=0.5."""
    g = subset(gaussians(500_000, 3), count)
    v = view((0.0, 0.0, -4.0), 32, 32, 40.0, 0.5)
    return g, [v], settings()


BATCH_RESOLUTIONS = ((800, 800), (1014, 1352), (1352, 1014), (960, 540))


def scene_200k_batch(n: int = 200_000, renders: int = 16):
    """200k Gaussians, 16 renders: camera on the radius-4 sphere, t ~ U[0,1],
    resolution drawn from BATCH_RESOLUTIONS (W x H), f = 1000."""
    g = gaussians(n, 3)
    rng = np.random.default_rng(CAMERA_SEED)
    views = []
    for _ in range(renders):
        d = rng.normal(0.0, 1.0, size=3)
        pos = 4.0 * d / np.linalg.norm(d)
        t = rng.uniform(0.0, 1.0)
        w, h = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
        views.append(view(pos, w, h, 1000.0, t))
    return g, views, settings()


def scene_3m_large(n: int = 3_000_000):
    """3M Gaussians in [-4,4]^3, SH 3, 1920x1080, f=1400, 8 timestamps x 2 views
    (phi in {0, pi/2}, radius 4), time cull at 9."""
    g = gaussians(n, 3, xyz_half_extent=4.0)
    views = []
    for t in np.linspace(0.0, 1.0, 8):
        for phi in (0.0, 0.5 * math.pi):
            pos = (4.0 * math.sin(phi), 0.0, -4.0 * math.cos(phi))
            views.append(view(pos, 1920, 1080, 1400.0, t))
    return g, views, settings(time_cull=9.0)
