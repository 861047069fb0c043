// The tiles a projected Gaussian is listed in.
//
// A pixel centre p can receive the Gaussian only if q(p) <= Q, where
// Q = min(extent^2, 2 ln(o / alpha_min)) (past Q either the extent test or the
// alpha_min test of the compositing rule, Sec. 3.1, skips the pair).  The
// Gaussian is listed in a tile when some pixel centre of the tile lies within
// one pixel of the ellipse q <= Q: that margin covers the rounding of the
// rasteriser's FP32 evaluation of q and of the exponential, and the rounding of
// the span arithmetic below (well under 1e-3 pixel).  The ellipse is convex, so
// in one row of tiles those tiles form one run of columns, which row_span
// returns; the rows with a non-empty run are consecutive.  For the elongated
// footprints of a trained scene this is about half of the bounding box.
//
// With d = mean2d - p = (dx, dy), q = a dx^2 + 2 b dx dy + c dy^2 and
// det = a c - b^2, the ellipse exists for |dy| <= hy = sqrt(a Q / det), and its
// row at offset dy covers pixel x in mx + beta dy +- gamma sqrt(hy^2 - dy^2)
// with beta = b / a, gamma = sqrt(det) / a.  The right end is concave in dy and
// peaks at dy = ds = b sqrt(Q / (c det)); the left end is convex with its
// minimum at -ds; over a band of rows each extreme is therefore at that offset
// clamped into the band.
//
// The per-Gaussian constants are computed in double and rounded to float; the
// per-row arithmetic is FP32 with contraction into fused multiply-adds
// disabled and correctly rounded square roots, so that a float32
// re-implementation gives the same tiles (the binning tests rely on it), and
// every kernel that walks the rows gets the same runs.  Tile sizes are powers
// of two (tile = pixel >> sh).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace r4d {

struct TileBox {
  int x0, y0, x1, y1;  // tiles [x0, x1) x [y0, y1)
};

struct SpanGeom {
  float mx, my, beta, gamma, hy, ds;
  int W, H, sh, x0, x1;  // image size, log2 tile size, columns the runs are clipped to
};

// Bounding box of the tiles: the ellipse's bounding box widened by one pixel.
// Returns false when it holds no pixel of the W x H image or the conic is not
// positive definite.
__host__ __device__ inline bool tile_box(double mx, double my, double a, double b, double c,
                                         double Q, int W, int H, int sh, TileBox& out) {
#pragma clang fp contract(off)
  const double det = a * c - b * b;
  if (!(det > 0.0) || !(a > 0.0) || !(Q >= 0.0)) return false;
  const double hwx = sqrt(Q * c / det) + 1.0;
  const double hwy = sqrt(Q * a / det) + 1.0;
  const double ilo = ceil(mx - hwx - 0.5), ihi = floor(mx + hwx - 0.5);
  const double jlo = ceil(my - hwy - 0.5), jhi = floor(my + hwy - 0.5);
  const double W1 = double(W - 1), H1 = double(H - 1);
  const double x0 = ilo > 0.0 ? ilo : 0.0, x1 = ihi < W1 ? ihi : W1;
  const double y0 = jlo > 0.0 ? jlo : 0.0, y1 = jhi < H1 ? jhi : H1;
  if (!(x0 <= x1) || !(y0 <= y1)) return false;
  out.x0 = int(x0) >> sh;
  out.x1 = (int(x1) >> sh) + 1;
  out.y0 = int(y0) >> sh;
  out.y1 = (int(y1) >> sh) + 1;
  return true;
}

// Per-Gaussian constants of row_span, from the record's values (a positive
// definite conic, Q >= 0).
__host__ __device__ inline SpanGeom span_geom(double mx, double my, double a, double b, double c,
                                              double Q, int W, int H, int sh, int x0, int x1) {
#pragma clang fp contract(off)
  const double det = a * c - b * b;
  SpanGeom s;
  s.mx = float(mx);
  s.my = float(my);
  s.beta = float(b / a);
  s.gamma = float(sqrt(det) / a);
  s.hy = float(sqrt(a * Q / det));
  s.ds = float(b * sqrt(Q / (c * det)));
  s.W = W;
  s.H = H;
  s.sh = sh;
  s.x0 = x0;
  s.x1 = x1;
  return s;
}

// Tile columns [x0, x1) of tile row ty, clipped to [s.x0, s.x1); empty rows
// give x0 == x1.  The band is the row's pixel centres (inside the image)
// widened by one pixel.
__host__ __device__ inline void row_span(const SpanGeom& s, int ty, int& x0, int& x1) {
#pragma clang fp contract(off)
  x0 = x1 = 0;
  const int yend = (ty + 1) << s.sh;
  const float ya = float(ty << s.sh) - 0.5f;
  const float yb = float(yend < s.H ? yend : s.H) + 0.5f;
  float lo = s.my - yb, hi = s.my - ya;
  lo = lo > -s.hy ? lo : -s.hy;
  hi = hi < s.hy ? hi : s.hy;
  if (!(lo <= hi)) return;
  float dmax = s.ds > lo ? s.ds : lo;
  dmax = dmax < hi ? dmax : hi;
  float dmin = -s.ds > lo ? -s.ds : lo;
  dmin = dmin < hi ? dmin : hi;
  const float wmax = sqrtf((s.hy - dmax) * (s.hy + dmax));
  const float wmin = sqrtf((s.hy - dmin) * (s.hy + dmin));
  const float pmax = s.mx + (s.beta * dmax + s.gamma * wmax);
  const float pmin = s.mx + (s.beta * dmin - s.gamma * wmin);
  float ilo = ceilf(pmin - 1.5f), ihi = floorf(pmax + 0.5f);
  ilo = ilo > 0.0f ? ilo : 0.0f;
  ihi = ihi < float(s.W - 1) ? ihi : float(s.W - 1);
  if (!(ilo <= ihi)) return;
  int a = int(ilo) >> s.sh, b = (int(ihi) >> s.sh) + 1;
  a = a > s.x0 ? a : s.x0;
  b = b < s.x1 ? b : s.x1;
  if (a < b) {
    x0 = a;
    x1 = b;
  }
}

}  // namespace r4d
