"""Shared helpers for the GPU parity tests: moving workload arrays to the
device and re-deriving the tile/sort order on the CPU from the GPU's own
integer outputs (rectangles and depth keys)."""
from __future__ import annotations

import numpy as np
import torch

PARAM_KEYS = ("means", "log_scales", "rotors", "opacity", "sh")


def to_device(g: dict, device, dtype=torch.float32) -> dict:
    out = {k: torch.as_tensor(np.ascontiguousarray(g[k])).to(device=device, dtype=dtype).contiguous()
           for k in PARAM_KEYS}
    out["sh_degree"] = int(g["sh_degree"])
    return out


def cpu_tile_lists(rects: np.ndarray, depth_keys: np.ndarray, tiles_x: int, tiles_y: int):
    """Reference binning + stable (tile, depth, index) order from integer data.

    rects: [n, 4] uint16 (x0, y0, x1, y1) tile rectangle, depth_keys: [n] uint32.
    Returns (values [D] uint32, ranges [tiles, 2] uint32)."""
    rects = rects.astype(np.int64)
    vis = np.nonzero(depth_keys != 0xFFFFFFFF)[0]
    tiles_l, idx_l, key_l = [], [], []
    for i in vis:
        x0, y0, x1, y1 = rects[i]
        ys, xs = np.mgrid[y0:y1, x0:x1]
        t = (ys * tiles_x + xs).ravel()
        tiles_l.append(t)
        idx_l.append(np.full(t.size, i, dtype=np.int64))
        key_l.append(np.full(t.size, depth_keys[i], dtype=np.int64))
    if not tiles_l:
        return np.zeros(0, np.uint32), np.zeros((tiles_x * tiles_y, 2), np.uint32)
    tiles = np.concatenate(tiles_l)
    idx = np.concatenate(idx_l)
    keys = np.concatenate(key_l)
    order = np.lexsort((idx, keys, tiles))          # last key is primary
    values = idx[order].astype(np.uint32)
    st = tiles[order]
    n_tiles = tiles_x * tiles_y
    starts = np.searchsorted(st, np.arange(n_tiles), side="left")
    ends = np.searchsorted(st, np.arange(n_tiles), side="right")
    ranges = np.stack([np.where(ends > starts, starts, 0), np.where(ends > starts, ends, 0)], 1)
    return values, ranges.astype(np.uint32)


def image_errors(gpu_img: np.ndarray, ref_img: np.ndarray, ambiguous: np.ndarray):
    """Max abs error over unambiguous pixels, and the ambiguous-pixel count.
    gpu_img/ref_img: [3, P] or [3, H, W]; ambiguous: [P] or [H, W] bool."""
    g = gpu_img.reshape(3, -1)
    r = ref_img.reshape(3, -1)
    amb = ambiguous.reshape(-1)
    keep = ~amb
    err = np.abs(g - r)[:, keep]
    return (float(err.max()) if err.size else 0.0), int(amb.sum())
