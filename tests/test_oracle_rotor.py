"""Pins for the oracle's rotor normalisation (F_norm) and rotor-to-matrix map
(F_map), App. A of the paper.

The strongest pin is an independent brute-force geometric-algebra product in
Cl(4,0) (basis blades as bit masks): the rotation is defined by u' = r u r^dagger
(App. A, rotor-to-rotation), so F_map's columns must equal r e_j r^dagger, and
r r^dagger must equal l^2 + 2 eps e0123 (App. A, expansion of r r^dagger).
"""
import math

import numpy as np
import torch

from oracle import render as O

# blade bit masks for the storage order s, b01, b02, b12, b03, b13, b23, p
BLADES = (0b0000, 0b0011, 0b0101, 0b0110, 0b1001, 0b1010, 0b1100, 0b1111)


def _reorder_sign(a: int, b: int) -> int:
    a >>= 1
    swaps = 0
    while a:
        swaps += bin(a & b).count("1")
        a >>= 1
    return -1 if swaps & 1 else 1


def ga_mul(x: dict, y: dict) -> dict:
    """Geometric product of multivectors {blade mask: coefficient}, e_i^2 = +1."""
    out = {}
    for a, ca in x.items():
        for b, cb in y.items():
            m = a ^ b
            out[m] = out.get(m, 0.0) + _reorder_sign(a, b) * ca * cb
    return out


def rotor_mv(r):
    return {BLADES[i]: float(r[i]) for i in range(8)}


def reverse_mv(x: dict) -> dict:
    out = {}
    for m, c in x.items():
        k = bin(m).count("1")
        out[m] = c * (-1 if (k * (k - 1) // 2) % 2 else 1)
    return out


def rand_rotors(n, seed=0):
    g = np.random.default_rng(seed)
    return torch.as_tensor(g.normal(size=(n, 8)), dtype=torch.float64)


def test_rr_dagger_expansion_pins_epsilon():
    r = rand_rotors(50)
    eps = O.rotor_epsilon(r)
    l2 = (r * r).sum(-1)
    for i in range(r.shape[0]):
        rv = rotor_mv(r[i])
        prod = ga_mul(rv, reverse_mv(rv))
        assert abs(prod.get(0, 0.0) - float(l2[i])) < 1e-12
        assert abs(prod.get(0b1111, 0.0) - 2.0 * float(eps[i])) < 1e-12
        for m, c in prod.items():
            if m not in (0, 0b1111):
                assert abs(c) < 1e-12


def test_epsilon_gradient_matches_finite_difference():
    r = rand_rotors(20, seed=3)
    g = O.rotor_epsilon_gradient(r)
    h = 1e-6
    for j in range(8):
        e = torch.zeros(8, dtype=torch.float64)
        e[j] = h
        fd = (O.rotor_epsilon(r + e) - O.rotor_epsilon(r - e)) / (2 * h)
        assert torch.allclose(fd, g[:, j], atol=1e-9)


def test_normalize_satisfies_both_conditions():
    r = rand_rotors(2000, seed=1)
    rn = O.rotor_normalize(r)
    assert O.rotor_epsilon(rn).abs().max() < 1e-14
    assert ((rn * rn).sum(-1) - 1).abs().max() < 1e-14
    # existence condition |2 eps| <= l^2 (AM-GM) holds for every draw
    assert bool((2 * O.rotor_epsilon(r).abs() <= (r * r).sum(-1) + 1e-15).all())


def test_normalize_is_idempotent_and_scale_invariant_on_valid_rotors():
    rn = O.rotor_normalize(rand_rotors(500, seed=2))
    assert (O.rotor_normalize(rn) - rn).abs().max() < 1e-14
    # a normalised rotor scaled by 3 normalises back to itself (eps scales, delta = 0)
    assert (O.rotor_normalize(3.0 * rn) - rn).abs().max() < 1e-13


def test_one_update_step_zeroes_epsilon_before_rescale():
    # eps(r + delta grad eps) = eps (1 + delta^2) + l^2 delta; with the chosen root it is 0
    r = rand_rotors(500, seed=4)
    eps = O.rotor_epsilon(r)
    l2 = (r * r).sum(-1)
    delta = -2 * eps / (l2 + torch.sqrt(l2 * l2 - 4 * eps * eps))
    r1 = r + delta[:, None] * O.rotor_epsilon_gradient(r)
    assert O.rotor_epsilon(r1).abs().max() < 1e-13
    # the root tends to 0 as eps -> 0 (sign choice of App. A)
    assert bool((delta.abs() <= 1.0 + 1e-12).all())


def test_degenerate_rotor_maps_to_identity():
    r = torch.zeros(2, 8, dtype=torch.float64)
    r[1, 3] = 1e-9
    rn = O.rotor_normalize(r)
    expect = torch.zeros(2, 8, dtype=torch.float64)
    expect[:, 0] = 1
    assert torch.equal(rn, expect)


def test_degenerate_rotors_have_zero_gradient():
    """Identity with zero gradient for rotors of squared norm below 1e-12
    before the update (0, all 1e-7) or after it: r = 1 +- e0123, i.e.
    (s, p) = (1, +-1), has 2|eps| = l^2, the step lands on 0 (the updated squared
    norm is (l^4 - 4 eps^2) / l^2); also a scaled copy.  A regular rotor
    beside them keeps a finite, nonzero gradient."""
    r = torch.zeros(6, 8, dtype=torch.float64)
    r[1] = 1e-7
    r[2, 0], r[2, 7] = 1.0, 1.0
    r[3, 0], r[3, 7] = 1.0, -1.0
    r[4, 0], r[4, 7] = 3.0, 3.0
    r[5] = torch.tensor([0.3, -0.2, 0.5, 0.1, 0.4, -0.3, 0.2, 0.6], dtype=torch.float64)
    r.requires_grad_(True)
    rn = O.rotor_normalize(r)
    ident = torch.zeros(8, dtype=torch.float64)
    ident[0] = 1
    for i in range(5):
        assert torch.equal(rn[i].detach(), ident), i
    w = torch.as_tensor(np.random.default_rng(0).normal(size=(6, 8)))
    (rn * w).sum().backward()
    assert bool(torch.isfinite(r.grad).all())
    assert torch.equal(r.grad[:5], torch.zeros(5, 8, dtype=torch.float64))
    assert float(r.grad[5].abs().max()) > 1e-3


def test_fmap_equals_sandwich_product():
    rn = O.rotor_normalize(rand_rotors(40, seed=5))
    R = O.rotor_to_matrix(rn)
    for i in range(rn.shape[0]):
        rv = rotor_mv(rn[i])
        rd = reverse_mv(rv)
        for j in range(4):
            img = ga_mul(ga_mul(rv, {1 << j: 1.0}), rd)
            for m, c in img.items():
                if bin(m).count("1") == 1:
                    row = m.bit_length() - 1
                    assert abs(c - float(R[i, row, j])) < 1e-12, (i, row, j)
                else:
                    assert abs(c) < 1e-12


def test_fmap_is_proper_rotation():
    R = O.rotor_to_matrix(O.rotor_normalize(rand_rotors(2000, seed=6)))
    eye = torch.eye(4, dtype=torch.float64)
    assert (R @ R.transpose(-1, -2) - eye).abs().max() < 1e-13
    assert (torch.linalg.det(R) - 1).abs().max() < 1e-13


def _quat_matrix(w, x, y, z):
    """Textbook rotation matrix of a unit quaternion (w, x, y, z)."""
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def test_spatial_rotor_reduces_to_quaternion_rotation():
    # Sec. 3.2.1: zero temporal components -> a 3D rotation (quaternion)
    g = np.random.default_rng(7)
    for _ in range(50):
        q = g.normal(size=4)
        q /= np.linalg.norm(q)
        r = torch.zeros(8, dtype=torch.float64)
        r[:4] = torch.as_tensor(q)                 # s, b01, b02, b12
        R = O.rotor_to_matrix(O.rotor_normalize(r[None]))[0].numpy()
        s, b01, b02, b12 = q
        expect = _quat_matrix(s, -b12, b02, -b01)
        assert np.abs(R[:3, :3] - expect).max() < 1e-13
        assert np.abs(R[3, :3]).max() < 1e-15 and np.abs(R[:3, 3]).max() < 1e-15
        assert abs(R[3, 3] - 1) < 1e-14


def test_xt_rotor_rotates_by_twice_the_angle():
    for theta in (0.1, 0.3, 1.0, 2.5):
        r = torch.zeros(1, 8, dtype=torch.float64)
        r[0, 0] = math.cos(theta)
        r[0, 4] = math.sin(theta)                  # b03
        R = O.rotor_to_matrix(O.rotor_normalize(r))[0]
        c, s = math.cos(2 * theta), math.sin(2 * theta)
        assert abs(R[0, 0] - c) < 1e-14 and abs(R[3, 3] - c) < 1e-14
        assert abs(R[0, 3] - s) < 1e-14 and abs(R[3, 0] + s) < 1e-14
        assert abs(R[1, 1] - 1) < 1e-14 and abs(R[2, 2] - 1) < 1e-14
