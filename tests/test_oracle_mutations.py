"""Planted mistakes in the oracle must fail its pins.

Each case swaps one step of the CPU oracle (in memory, for the duration of the
test) for a plausible mistake and checks that at least one pin of
test_oracle_ewa_pins.py then fails:

* the conic's cross term with the wrong sign (q = a dx^2 - 2 b dx dy + c dy^2
  instead of + 2 b dx dy, Sec. 3.1 inverse of the 2D covariance);
* the guard-band clamp of x/z, y/z in the projection's Jacobian dropped;
* the camera rotation transposed in J Wv Sigma Wv^T J^T.

Nothing here touches the HIP library.
"""
import pytest
import torch

import test_oracle_ewa_pins as P
from oracle import render as O


def _flipped_conic(cov2):
    a, b, c = cov2[:, 0, 0], cov2[:, 0, 1], cov2[:, 1, 1]
    det = a * c - b * b
    return torch.stack([c / det, b / det, a / det], dim=-1), det


def _fails(fn):
    try:
        fn()
    except AssertionError:
        return True
    return False


def test_flipped_cross_term_is_caught(monkeypatch):
    monkeypatch.setattr(O, "conic_of", _flipped_conic)
    assert _fails(P.test_rotated_anisotropic_gaussian_by_rotor)
    assert _fails(P.test_rotated_anisotropic_gaussian_by_camera_roll)
    assert _fails(P.test_tiny_scene_matches_ray_integration)


def test_dropped_guard_band_is_caught(monkeypatch):
    orig = O.project_ewa
    monkeypatch.setattr(O, "project_ewa",
                        lambda mu3, cov3, view, st: orig(mu3, cov3, view, dict(st, guard_band=1e9)))
    assert _fails(P.test_guard_band_clamps_jacobian)
    assert _fails(P.test_guard_band_footprint_in_image)


def test_transposed_camera_rotation_is_caught(monkeypatch):
    orig = O.project_ewa

    def transposed(mu3, cov3, view, st):
        # Wv^T in place of Wv for the covariance only (the mean stays right)
        v = dict(view)
        w2c = O._to64(view["world_to_cam"]).reshape(3, 4).clone()
        w2c[:, :3] = w2c[:, :3].T.clone()
        v["world_to_cam"] = w2c.numpy()
        _, _, _, cov2 = orig(mu3, cov3, v, st)
        pc, mean2, depth, _ = orig(mu3, cov3, view, st)
        return pc, mean2, depth, cov2

    monkeypatch.setattr(O, "project_ewa", transposed)
    assert _fails(P.test_rotated_anisotropic_gaussian_by_camera_roll)
    assert _fails(P.test_tiny_scene_matches_ray_integration)


def test_unmodified_oracle_passes():
    for fn in (P.test_rotated_anisotropic_gaussian_by_rotor,
               P.test_rotated_anisotropic_gaussian_by_camera_roll,
               P.test_guard_band_clamps_jacobian, P.test_guard_band_footprint_in_image):
        fn()
