// Front tile lists.
//
// A tile's list holds every Gaussian listed in the tile, in depth order, but
// the compositing rule (Sec. 3.1) stops a pixel once its transmittance would
// fall below T_min, so on a deep scene the rasteriser reads only the first
// few hundred entries of a list thousands long.  The lists are therefore
// emitted and sorted only up to a depth cut: with the visible Gaussians of a
// render numbered 0 .. n_vis - 1 in depth order, entries from depth positions
// below r0 = ceil(f n_vis) are listed everywhere; entries from later
// positions only in tiles whose whole list is kept, those covered by at most
// `keep` tile boxes of the Gaussians before r0 (a tile that few of the front
// Gaussians reach may not fill up with them: the front of a scene seen at an
// angle covers only part of the screen).  Every other tile holds a front
// list, a prefix of its full list.  The forward rasteriser walks a tile's
// list until its pixels stop; if a front list runs out first, the tile is
// queued, and a second pass collects the tile's remaining entries (the
// later Gaussians whose row run covers the tile, in depth order) into the
// render's rest area, records them as the tile's second range and renders
// the tile again over both ranges.  Either way the walk sees the full list's entries in
// the full list's order up to where it stops, so images, stop positions and
// gradients are those of the full lists.
//
// A list position p of a tile with front range [s, s + n0) and rest range
// [a, a + n1) (n1 = 0 without one) lies at s + p for p < n0, else at
// a + p - n0.  Rest ranges start at multiples of kSegment inside the render's
// segment of the list buffer, after its front entries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "r4d_internal.hpp"
#include "tileset.hpp"

namespace r4d {

// Depth cut of a render with n_vis visible Gaussians: f = front16 / 65536
// (front16 = 0: no cut).
__host__ __device__ __forceinline__ uint32_t front_cut(uint32_t n_vis, uint32_t front16) {
  if (front16 == 0u) return n_vis;
  const uint32_t r = uint32_t((uint64_t(n_vis) * front16 + 65535u) >> 16);
  return r < n_vis ? r : n_vis;
}

// Length of a render's segment of the list buffer for d entries: the whole
// lists, and with a depth cut room for each tile's rest range to start on a
// multiple of kSegment; rounded up to kSegAlign.
__host__ __device__ __forceinline__ unsigned long long seg_extent(unsigned long long d,
                                                                  const ViewSlot& sl) {
  const unsigned long long tiles =
      (unsigned long long)sl.v.tiles_x * (unsigned long long)sl.v.tiles_y;
  const unsigned long long e = d + (sl.front16 ? (unsigned long long)kSegment * (tiles + 1) : 0ull);
  return (e + kSegAlign - 1) / kSegAlign * kSegAlign;
}

// 64-bit words per row of a render's keep bitmap.
__host__ __device__ __forceinline__ uint32_t keep_words(int tiles_x) {
  return uint32_t(tiles_x + 63) >> 6;
}

// Kept tiles among columns [x0, x1) of one bitmap row (x0 < x1).
__device__ __forceinline__ uint32_t kept_in_run(const uint64_t* __restrict__ row, int x0,
                                                int x1) {
  uint32_t c = 0;
  for (int w = x0 >> 6; w <= (x1 - 1) >> 6; ++w) {
    uint64_t m = row[w];
    const int lo = w << 6;
    if (x0 > lo) m &= ~0ull << (x0 - lo);
    if (x1 - lo < 64) m &= (1ull << (x1 - lo)) - 1ull;
    c += uint32_t(__popcll(m));
  }
  return c;
}

__device__ __forceinline__ bool tile_kept(const uint64_t* __restrict__ row, int x) {
  return (row[x >> 6] >> (x & 63)) & 1ull;
}

// Whether the box [x0, x1) x [y0, y1) of a render holds a kept tile (bitmap
// rows `words` apart).
__device__ __forceinline__ bool any_kept_in_box(const uint64_t* __restrict__ bits, uint32_t words,
                                                int x0, int y0, int x1, int y1) {
  if (x0 >= x1) return false;
  for (int y = y0; y < y1; ++y)
    if (kept_in_run(bits + size_t(y) * words, x0, x1)) return true;
  return false;
}

// Run constants of a record inside its tile box (as the preprocess made them).
template <typename T>
__device__ __forceinline__ SpanGeom geom_of(const Rec<T>& r, const Rect16& box,
                                            const ViewDev& v) {
  return span_geom(double(r.mx), double(r.my), double(r.ca), double(r.cb), double(r.cc),
                   double(r.qmax), v.W, v.H, __builtin_ctz(unsigned(v.tile_size)), box.x0,
                   box.x1);
}

// Position of list entry p of a tile (see above; both ranges as [start, end)).
__device__ __forceinline__ uint32_t list_pos(uint2 front, uint2 rest, uint32_t p) {
  const uint32_t n0 = front.y - front.x;
  return p < n0 ? front.x + p : rest.x + (p - n0);
}

// Boundary-state slot (Ck) of list position m * kSegment of a tile: inside the
// front list the slot of the whole-list numbering (ck_slot); past it, one
// derived from the position in the rest area, offset past every front slot
// of the render (tile_end: one past the render's last global tile).
__device__ __forceinline__ uint32_t boundary_slot(uint2 front, uint2 rest, uint32_t gtile,
                                                  uint32_t tile_end, uint32_t m) {
  const uint32_t b = m * kSegment, n0 = front.y - front.x;
  if (b < n0) return ck_slot(front.x, gtile, m);
  return (rest.x + (b - n0)) / kSegment + tile_end + 1u;
}

}  // namespace r4d
