"""CPU oracle for the 4D consistency loss (Sec. 3.3 "4D Consistency Loss").

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library.

What the paper defines:
  * every Gaussian i has a speed s_i = V_i / W_i (the motion of its slice,
    Sec. 3.2.2; V the space-time block of Sigma_4, W its time variance);
  * Omega_i: its K nearest Gaussians in 4D (x, y, z, t), Euclidean distance
    after dividing the spatial coordinates by the spatial scene scale and t by
    the temporal scene scale;
  * L = (1/N) sum_i || s_i - (1/K) sum_{j in Omega_i} s_j ||_1.

Readings (listed in the design notes): Omega_i excludes i itself; the K
nearest are ranked by distance, ties by the smaller index; the nearest-
neighbour decision is a discrete choice taken in float32 (the precision of the
stored means), with the scaled coordinates u = x * fl32(1 / scale) and the
squared distance summed in the order ((d0^2 + d1^2) + d2^2) + d3^2, each
operation rounded to float32; the loss and its gradient are FP64 with the
neighbour lists fixed (no gradient flows through the choice of neighbours).
"""
from __future__ import annotations

import numpy as np
import torch

from . import render as R


def inverse_scales(spatial_scale: float, temporal_scale: float) -> np.ndarray:
    """float32 reciprocals of the scene scales, as (x, y, z, t) multipliers:
    the reciprocal of the float32 scale, rounded once to float32."""
    ss = float(np.float32(spatial_scale))
    ts = float(np.float32(temporal_scale))
    if not (ss > 0 and ts > 0):
        raise ValueError("scene scales must be positive")
    inv_s, inv_t = np.float32(1.0 / ss), np.float32(1.0 / ts)
    return np.array([inv_s, inv_s, inv_s, inv_t], dtype=np.float32)


def scaled_coords(means: np.ndarray, spatial_scale: float, temporal_scale: float) -> np.ndarray:
    """[n, 4] float32 scaled 4D coordinates of means ([4, n] float32)."""
    m = np.asarray(means, dtype=np.float32)
    return (m.T * inverse_scales(spatial_scale, temporal_scale)[None, :]).astype(np.float32)


def squared_distances_f32(uq: np.ndarray, u: np.ndarray) -> np.ndarray:
    """[q, n] float32 squared distances, summed in the fixed order."""
    d = uq[:, None, :] - u[None, :, :]
    sq = d * d
    return ((sq[..., 0] + sq[..., 1]) + sq[..., 2]) + sq[..., 3]


def knn4d(means: np.ndarray, k: int, spatial_scale: float = 1.0, temporal_scale: float = 1.0,
          queries: np.ndarray | None = None, chunk: int = 256) -> np.ndarray:
    """Brute-force K nearest neighbours in scaled 4D space.

    means: [4, n] float32.  Returns [q, k] int64: for each query index (all
    Gaussians, or `queries`), the indices of its k nearest other Gaussians,
    nearest first, ties by the smaller index."""
    u = scaled_coords(means, spatial_scale, temporal_scale)
    n = u.shape[0]
    if not (1 <= k < n):
        raise ValueError("need 1 <= k < n")
    qs = np.arange(n) if queries is None else np.asarray(queries, dtype=np.int64)
    out = np.empty((qs.size, k), dtype=np.int64)
    for s0 in range(0, qs.size, chunk):
        q = qs[s0:s0 + chunk]
        d2 = squared_distances_f32(u[q], u)
        d2[np.arange(q.size), q] = np.inf           # not its own neighbour
        # every index within the k-th smallest distance competes; order the
        # competitors by (distance, index) and keep the first k of each row
        kth = np.partition(d2, k - 1, axis=1)[:, k - 1]
        rows, cols = np.nonzero(d2 <= kth[:, None])
        order = np.lexsort((cols, d2[rows, cols], rows))
        rows, cols = rows[order], cols[order]
        first = np.searchsorted(rows, np.arange(q.size))
        out[s0:s0 + q.size] = cols[first[:, None] + np.arange(k)[None, :]]
    return out


def speeds(P: dict) -> torch.Tensor:
    """[n, 3] FP64 speed V / W of every Gaussian (Sec. 3.2.2), from the
    normalised rotor and the scales (independent of the time)."""
    r = R.rotor_normalize(P["rotors"].T)
    cov4 = R.covariance_4d(R.rotor_to_matrix(r), P["log_scales"].T)
    return cov4[:, :3, 3] / cov4[:, 3, 3][:, None]


def consistency_loss(P: dict, neighbours: np.ndarray) -> torch.Tensor:
    """L = (1/N) sum_i || s_i - mean_{j in Omega_i} s_j ||_1 (FP64, differentiable
    w.r.t. the rotors and log-scales in P)."""
    s = speeds(P)
    nb = torch.as_tensor(np.asarray(neighbours, dtype=np.int64))
    mean_nb = s[nb].mean(dim=1)
    return (s - mean_nb).abs().sum(dim=1).mean()
