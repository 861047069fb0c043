// Load-balanced walk over the tile rows of the Gaussians held by a wavefront.
//
// Lane l holds one Gaussian (or none) whose listed tiles lie in rows [y0, y1).
// The rows of all 64 Gaussians are taken as one sequence, lane 0's rows first,
// and evaluated 64 at a time, one row per lane, so a lane whose Gaussian spans
// many rows does not hold the others up.  Each lane finds the holder of its
// row by a binary search over the holders' first positions (wave shuffles)
// and fetches the holder's run constants the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "tileset.hpp"

namespace r4d {

// x plus the value the DPP lane move CTRL brings, in the rows ROWS (a lane of
// another row, or one whose source lies outside its row under BOUND, adds 0).
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ uint32_t dpp_plus(uint32_t x) {
  return x + uint32_t(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROWS, 0xf, BOUND));
}

// Inclusive scan over the wavefront's 64 lanes with DPP lane moves (no LDS):
// within each row of 16 lanes by row shifts of 1, 2, 4 and 8, then across
// rows by adding lane 15 of the row before to rows 1 and 3 (row_bcast:15)
// and lane 31 to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x, int /*lane*/) {
  x = dpp_plus<0x111, 0xf, true>(x);   // row_shr:1
  x = dpp_plus<0x112, 0xf, true>(x);   // row_shr:2
  x = dpp_plus<0x114, 0xf, true>(x);   // row_shr:4
  x = dpp_plus<0x118, 0xf, true>(x);   // row_shr:8
  x = dpp_plus<0x142, 0xa, false>(x);  // row_bcast:15 into rows 1, 3
  x = dpp_plus<0x143, 0xc, false>(x);  // row_bcast:31 into rows 2, 3
  return x;
}

// Last lane o with key[o] <= p, for keys non-decreasing over the lanes and
// key[0] <= p.
__device__ __forceinline__ int wave_upper_lane(uint32_t key, uint32_t p) {
  int o = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1) {
    const uint32_t k = __shfl(key, o + step, 64);
    if (k <= p) o += step;
  }
  return o;
}

// visit(ok, holder, y, x0, x1) is called by every lane for every group of 64
// rows (ok false for the lanes past the last row; then the other arguments
// are meaningless).  Every lane must call wave_rows with its own Gaussian, and
// visit may use wave-wide operations.  sg.W, sg.H and sg.sh must be the same
// in every lane.
template <typename Visit>
__device__ __forceinline__ void wave_rows(const SpanGeom& sg, int y0, int y1, int lane,
                                          Visit visit) {
  const uint32_t R = y1 > y0 ? uint32_t(y1 - y0) : 0u;
  const uint32_t incl = wave_incl_scan_u32(R, lane);
  const uint32_t first = incl - R;
  const uint32_t total = __shfl(incl, 63, 64);
  for (uint32_t c = 0; c < total; c += 64) {
    const uint32_t p = c + uint32_t(lane);
    const int o = wave_upper_lane(first, p);
    SpanGeom g;
    g.mx = __shfl(sg.mx, o, 64);
    g.my = __shfl(sg.my, o, 64);
    g.beta = __shfl(sg.beta, o, 64);
    g.gamma = __shfl(sg.gamma, o, 64);
    g.hy = __shfl(sg.hy, o, 64);
    g.ds = __shfl(sg.ds, o, 64);
    g.x0 = __shfl(sg.x0, o, 64);
    g.x1 = __shfl(sg.x1, o, 64);
    g.W = sg.W;
    g.H = sg.H;
    g.sh = sg.sh;
    const int y = __shfl(y0, o, 64) + int(p - __shfl(first, o, 64));
    const bool ok = p < total;
    int x0 = 0, x1 = 0;
    if (ok) row_span(g, y, x0, x1);
    visit(ok, o, y, x0, x1);
  }
}

}  // namespace r4d
