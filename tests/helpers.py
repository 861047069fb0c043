"""Shared helpers for the GPU parity tests: moving workload arrays to the
device and re-deriving the tile/sort order on the CPU from the GPU's own
outputs (records, tile boxes and depth keys)."""
from __future__ import annotations

import numpy as np
import torch

PARAM_KEYS = ("means", "log_scales", "rotors", "opacity", "sh")


def to_device(g: dict, device, dtype=torch.float32) -> dict:
    out = {k: torch.as_tensor(np.ascontiguousarray(g[k])).to(device=device, dtype=dtype).contiguous()
           for k in PARAM_KEYS}
    out["sh_degree"] = int(g["sh_degree"])
    return out


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def row_runs(rec: np.ndarray, rects: np.ndarray, ys: np.ndarray, gi: np.ndarray,
             tile_size: int, width: int, height: int):
    """Tile columns [x0, x1) of tile row ys[k] of Gaussian gi[k]: the rule the
    binning follows (a tile is listed when one of its pixel centres lies within
    one pixel of the ellipse q <= qmax), re-implemented from its definition in
    the same arithmetic (per-Gaussian constants in float64 rounded to float32,
    per-row work in float32, no fused multiply-adds), so the runs must agree
    bit for bit.  rec: [n, 12] record values (mx, my, a, b, c, o, depth, qmax,
    ...), rects: [n, 4] (x0, y0, x1, y1) boxes the runs are clipped to."""
    sh = int(tile_size).bit_length() - 1
    r = rec[gi].astype(np.float64)
    mx, my, a, b, c, Q = r[:, 0], r[:, 1], r[:, 2], r[:, 3], r[:, 4], r[:, 7]
    det = a * c - b * b
    beta = _f32(b / a)
    gamma = _f32(np.sqrt(det) / a)
    hy = _f32(np.sqrt(a * Q / det))
    ds = _f32(b * np.sqrt(Q / (c * det)))
    mxf, myf = _f32(mx), _f32(my)
    ys = ys.astype(np.int64)
    ya = (ys << sh).astype(np.float32) - np.float32(0.5)
    yb = np.minimum((ys + 1) << sh, height).astype(np.float32) + np.float32(0.5)
    lo = np.maximum(myf - yb, -hy)
    hi = np.minimum(myf - ya, hy)
    ok = lo <= hi
    dmax = np.minimum(np.maximum(ds, lo), hi)
    dmin = np.minimum(np.maximum(-ds, lo), hi)
    wmax = np.sqrt((hy - dmax) * (hy + dmax))
    wmin = np.sqrt((hy - dmin) * (hy + dmin))
    pmax = mxf + (beta * dmax + gamma * wmax)
    pmin = mxf + (beta * dmin - gamma * wmin)
    ilo = np.maximum(np.ceil(pmin - np.float32(1.5)), np.float32(0))
    ihi = np.minimum(np.floor(pmax + np.float32(0.5)), np.float32(width - 1))
    ok &= ilo <= ihi
    bx = rects[gi].astype(np.int64)
    x0 = np.maximum(np.where(ok, ilo, 0).astype(np.int64) >> sh, bx[:, 0])
    x1 = np.minimum((np.where(ok, ihi, 0).astype(np.int64) >> sh) + 1, bx[:, 2])
    ok &= x0 < x1
    return np.where(ok, x0, 0), np.where(ok, x1, 0)


def cpu_tile_lists(rec: np.ndarray, rects: np.ndarray, depth_keys: np.ndarray, tiles_x: int,
                   tiles_y: int, tile_size: int, width: int, height: int):
    """Reference binning + stable (tile, depth, index) order from the GPU's
    records, boxes and depth keys.

    rec: [n, 12] records, rects: [n, 4] uint16 (x0, y0, x1, y1) box of the row
    runs, depth_keys: [n] uint32.  Checks that every row of a box holds a run
    and that the box is the runs' bounding box.  Returns (values [D] uint32,
    ranges [tiles, 2] uint32)."""
    rects = rects.astype(np.int64)
    n_tiles = tiles_x * tiles_y
    vis = np.nonzero(depth_keys != 0xFFFFFFFF)[0]
    if vis.size == 0:
        return np.zeros(0, np.uint32), np.zeros((n_tiles, 2), np.uint32)
    nrow = rects[vis, 3] - rects[vis, 1]
    assert np.all(nrow > 0)
    gi = np.repeat(vis, nrow)
    first = np.repeat(np.cumsum(nrow) - nrow, nrow)
    ys = rects[gi, 1] + (np.arange(gi.size) - first)
    with np.errstate(invalid="ignore"):
        x0, x1 = row_runs(rec, rects, ys, gi, tile_size, width, height)
    L = x1 - x0
    assert np.all(L > 0), "a row of a box without a run"
    assert np.array_equal(np.minimum.reduceat(x0, np.cumsum(nrow) - nrow), rects[vis, 0])
    assert np.array_equal(np.maximum.reduceat(x1, np.cumsum(nrow) - nrow), rects[vis, 2])
    # entries: run k contributes tiles ys*tiles_x + x0 .. + L - 1
    run = np.repeat(np.arange(L.size), L)
    within = np.arange(run.size) - np.repeat(np.cumsum(L) - L, L)
    tiles = ys[run] * tiles_x + x0[run] + within
    idx = gi[run]
    keys = depth_keys[idx].astype(np.int64)
    order = np.lexsort((idx, keys, tiles))          # last key is primary
    values = idx[order].astype(np.uint32)
    st = tiles[order]
    starts = np.searchsorted(st, np.arange(n_tiles), side="left")
    ends = np.searchsorted(st, np.arange(n_tiles), side="right")
    ranges = np.stack([np.where(ends > starts, starts, 0), np.where(ends > starts, ends, 0)], 1)
    return values, ranges.astype(np.uint32)


def cpu_tile_rows(rec: np.ndarray, rects: np.ndarray, depth_keys: np.ndarray, tiles_x: int,
                  tile_rows, tile_size: int, width: int, height: int, chunk: int = 1 << 20):
    """The reference binning of cpu_tile_lists restricted to whole tile rows:
    (total entry count over all rows, {tile id: values in (depth, index)
    order} for every tile of `tile_rows`).  For renders whose full lists are
    too long to sort on the host; every Gaussian's row runs are still derived
    (in chunks of rows) so the total is exact."""
    rects = rects.astype(np.int64)
    vis = np.nonzero(depth_keys != 0xFFFFFFFF)[0]
    want = np.zeros(int(rects[:, 3].max(initial=0)) + 1, dtype=bool)
    for r in tile_rows:
        if r < want.size:
            want[r] = True
    nrow = rects[vis, 3] - rects[vis, 1]
    assert np.all(nrow > 0)
    total = 0
    parts_t, parts_i = [], []
    csum = np.concatenate([[0], np.cumsum(nrow)])
    g0 = 0
    while g0 < vis.size:
        g1 = int(np.searchsorted(csum, csum[g0] + chunk, side="right")) - 1
        g1 = max(g1, g0 + 1)
        v = vis[g0:g1]
        nr = nrow[g0:g1]
        gi = np.repeat(v, nr)
        first = np.repeat(np.cumsum(nr) - nr, nr)
        ys = rects[gi, 1] + (np.arange(gi.size) - first)
        with np.errstate(invalid="ignore"):
            x0, x1 = row_runs(rec, rects, ys, gi, tile_size, width, height)
        L = x1 - x0
        assert np.all(L > 0), "a row of a box without a run"
        heads = np.cumsum(nr) - nr
        assert np.array_equal(np.minimum.reduceat(x0, heads), rects[v, 0])
        assert np.array_equal(np.maximum.reduceat(x1, heads), rects[v, 2])
        total += int(L.sum())
        sel = want[ys]
        if sel.any():
            ys_s, x0_s, L_s, gi_s = ys[sel], x0[sel], L[sel], gi[sel]
            run = np.repeat(np.arange(L_s.size), L_s)
            within = np.arange(run.size) - np.repeat(np.cumsum(L_s) - L_s, L_s)
            parts_t.append(ys_s[run] * tiles_x + x0_s[run] + within)
            parts_i.append(gi_s[run])
        g0 = g1
    tiles = np.concatenate(parts_t) if parts_t else np.zeros(0, np.int64)
    idx = np.concatenate(parts_i) if parts_i else np.zeros(0, np.int64)
    keys = depth_keys[idx].astype(np.int64)
    order = np.lexsort((idx, keys, tiles))
    tiles, idx = tiles[order], idx[order]
    out = {}
    for r in tile_rows:
        for t in range(r * tiles_x, (r + 1) * tiles_x):
            lo, hi = np.searchsorted(tiles, t, "left"), np.searchsorted(tiles, t, "right")
            out[t] = idx[lo:hi].astype(np.uint32)
    return total, out


# ---- front lists (the library's depth cut of the tile lists, front.hpp)
KEEP_GRID = 16384  # cover-grid cells a render may have and still get a cut


def front_cut(n_vis: int, settings: dict, tiles_x: int, tiles_y: int):
    """Depth position from which Gaussians are listed only in kept tiles, or
    None when the render gets whole lists (front_fraction >= 1, or a cover
    grid over KEEP_GRID cells)."""
    f = float(settings.get("front_fraction", 1.0))
    if f >= 1.0 or (tiles_x + 1) * (tiles_y + 1) > KEEP_GRID:
        return None
    f16 = int(min(65536, max(1, np.ceil(np.float64(np.float32(f)) * 65536.0))))
    return min(n_vis, (n_vis * f16 + 65535) >> 16)


def depth_positions(depth_keys: np.ndarray) -> np.ndarray:
    """Position of every visible Gaussian in (depth key, index) order (-1 for
    the rest)."""
    vis = np.nonzero(depth_keys != 0xFFFFFFFF)[0]
    order = vis[np.lexsort((vis, depth_keys[vis]))]
    pos = np.full(depth_keys.size, -1, dtype=np.int64)
    pos[order] = np.arange(order.size)
    return pos


def kept_tiles(rects: np.ndarray, depth_keys: np.ndarray, tiles_x: int, tiles_y: int,
               keep: int, r0: int) -> np.ndarray:
    """Kept tiles, [tiles] bool: those covered by at most `keep` tile boxes of
    the front Gaussians (depth positions below r0)."""
    pos = depth_positions(depth_keys)
    idx = np.nonzero((pos >= 0) & (pos < r0))[0]
    cover = np.zeros((tiles_y, tiles_x), dtype=np.int64)
    for x0, y0, x1, y1 in rects[idx].astype(np.int64):
        cover[y0:y1, x0:x1] += 1
    return (cover <= keep).reshape(-1)


def front_lists(ref_vals: np.ndarray, ref_rng: np.ndarray, pos: np.ndarray, r0: int,
                kept: np.ndarray):
    """The front lists the library should emit from the whole lists: a kept
    tile's whole list, any other tile's entries from depth positions below
    r0.  Returns (values, ranges, {tile: the rest of its list})."""
    lens = (ref_rng[:, 1].astype(np.int64) - ref_rng[:, 0].astype(np.int64))
    tile = np.repeat(np.arange(lens.size), lens)
    front = kept[tile] | (pos[ref_vals.astype(np.int64)] < r0)
    counts = np.bincount(tile[front], minlength=lens.size)
    ends = np.cumsum(counts)
    rng = np.stack([np.where(counts > 0, ends - counts, 0), np.where(counts > 0, ends, 0)], 1)
    rest = {}
    for t in np.unique(tile[~front]):
        rest[int(t)] = ref_vals[(tile == t) & ~front]
    return ref_vals[front], rng.astype(np.uint32), rest


def tile_lists(r4d, saved, view: int, n: int):
    """The GPU's tile lists of one render of a saved forward and their CPU
    re-derivation: (values, ranges, ref_values, ref_ranges, stats).  With
    front lists, the values are the front lists (the first n_front entries of
    VALUES) and the reference is derived from the whole lists by the front
    rule; every rest the forward collected is checked here against the rest of
    its tile's whole list."""
    s = saved.stats(view)
    ts = saved.config()["tile_size"]
    width, height = int(saved.views[view]["width"]), int(saved.views[view]["height"])
    rec = saved.copy(view, r4d.BUF_RECORDS, n).double().cpu().numpy()
    rect = saved.copy(view, r4d.BUF_RECT, n).cpu().numpy().view(np.uint16)
    key = saved.copy(view, r4d.BUF_DEPTHKEY, n).cpu().numpy().view(np.uint32)
    vals = saved.copy(view, r4d.BUF_VALUES, n).cpu().numpy().view(np.uint32)
    rng = saved.copy(view, r4d.BUF_RANGES, n).cpu().numpy().view(np.uint32)
    ref_vals, ref_rng = cpu_tile_lists(rec, rect, key, s["tiles_x"], s["tiles_y"], ts, width,
                                       height)
    settings = dict(r4d.default_settings(), **getattr(saved, "settings", {}))
    r0 = front_cut(s["n_visible"], settings, s["tiles_x"], s["tiles_y"])
    if r0 is None:
        assert s["n_front"] == s["n_dup"] and s["rest_tiles"] == 0
        return vals, rng, ref_vals, ref_rng, s
    kept = kept_tiles(rect, key, s["tiles_x"], s["tiles_y"], int(settings["front_keep"]), r0)
    f_vals, f_rng, rest = front_lists(ref_vals, ref_rng, depth_positions(key), r0, kept)
    rest_rng = saved.copy(view, r4d.BUF_REST, n).cpu().numpy().view(np.uint32)
    got = np.nonzero(rest_rng[:, 1] > rest_rng[:, 0])[0]
    assert got.size == s["rest_tiles"]
    for t in got:
        a, b = int(rest_rng[t, 0]), int(rest_rng[t, 1])
        assert a >= s["n_front"] and a % 256 == 0
        assert np.array_equal(vals[a:b], rest.get(int(t), np.zeros(0, np.uint32))), f"rest of {t}"
    return vals[:s["n_front"]], rng, f_vals, f_rng, s


def image_errors(gpu_img: np.ndarray, ref_img: np.ndarray, ambiguous: np.ndarray):
    """Max abs error over unambiguous pixels, and the ambiguous-pixel count.
    gpu_img/ref_img: [3, P] or [3, H, W]; ambiguous: [P] or [H, W] bool."""
    g = gpu_img.reshape(3, -1)
    r = ref_img.reshape(3, -1)
    amb = ambiguous.reshape(-1)
    keep = ~amb
    err = np.abs(g - r)[:, keep]
    return (float(err.max()) if err.size else 0.0), int(amb.sum())
