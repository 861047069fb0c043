// 4D nearest neighbours and the 4D consistency loss (Sec. 3.3, "4D Consistency
// Loss"): each Gaussian's speed s = V / W (Sec. 3.2.2) is pulled towards the
// mean speed of its K nearest Gaussians in 4D, distances taken after dividing
// x, y, z by the spatial and t by the temporal scene scale.
//
// KNN: a uniform grid over the bounding box of the scaled means (about two
// points per cell), a counting sort of the points into their cells, then one
// thread per point (in cell order, so a wavefront's queries share cells)
// searching shells of cells of growing Chebyshev radius around its own cell,
// keeping the K best (distance, index) pairs in registers.  The search stops
// once no unvisited cell can hold a point at or below the current K-th
// distance; that bound carries a margin for every float32 rounding of the cell
// assignment, so the result is the exact float32 K nearest neighbours: the
// squared distance ((d0^2 + d1^2) + d2^2) + d3^2 of the scaled coordinates
// u = x * fl(1 / scale), each operation rounded, ties by index, the point
// itself excluded.
//
// Loss: L = (1/N) sum_i |s_i - mean_{j in Omega_i} s_j|_1.  Its gradient with
// respect to s_i is (sign(d_i) - (1/K) sum_{m : i in Omega_m} sign(d_m)) / N,
// d_i = s_i - mean_j s_j; the second sum is gathered with integer atomics
// (exact, order-independent; the three components packed in one 64-bit word
// when n <= 2^20) and the result chained through s = V / W into Sigma_4 and on
// to the rotor and log-scales.
#include <hip/hip_runtime.h>

#include <math.h>

#include "r4d_internal.hpp"

namespace r4d {

namespace {

constexpr int kBlock = 256;
constexpr int kBoundBlocks = 1024;
// Target points per grid cell of the KNN (the grid has about n / this cells).
#ifndef R4D_KNN_CELL_POINTS
#define R4D_KNN_CELL_POINTS 2
#endif
constexpr uint32_t kCellPoints = R4D_KNN_CELL_POINTS;

struct Grid4 {
  float lo[4];    // lower corner of the box (scaled coordinates)
  float h;        // cell width
  float inv_h;    // fl(1 / h), the factor of the cell assignment
  float slack;    // bound on how far a point can sit outside its cell's box
  int32_t G[4];   // cells per dimension
  uint32_t cells;
};

__device__ __forceinline__ float4 scaled_point(const float* __restrict__ means, uint32_t n,
                                               uint32_t i, float4 inv) {
  return make_float4(means[i] * inv.x, means[size_t(n) + i] * inv.y,
                     means[2 * size_t(n) + i] * inv.z, means[3 * size_t(n) + i] * inv.w);
}

__device__ __forceinline__ float comp(float4 v, int d) {
  return d == 0 ? v.x : (d == 1 ? v.y : (d == 2 ? v.z : v.w));
}

// Cell coordinate of a scaled coordinate (the same expression everywhere).
__device__ __forceinline__ int cell_coord(float u, float lo, float inv_h, int G) {
  const int c = int(floorf((u - lo) * inv_h));
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

__device__ __forceinline__ uint32_t cell_id(const int c[4], const Grid4& g) {
  return uint32_t(c[0]) + uint32_t(g.G[0]) *
                              (uint32_t(c[1]) + uint32_t(g.G[1]) *
                                                    (uint32_t(c[2]) + uint32_t(g.G[2]) * uint32_t(c[3])));
}

__device__ __forceinline__ float dist2(float4 a, float4 b) {
#pragma clang fp contract(off)
  const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
  return ((d0 * d0 + d1 * d1) + d2 * d2) + d3 * d3;
}

// Per-workgroup minimum and maximum of the scaled coordinates.
__global__ __launch_bounds__(kBlock) void bounds_kernel(const float* __restrict__ means, uint32_t n,
                                                        float4 inv, float* __restrict__ partials) {
  __shared__ float s_v[kBlock / 64][8];
  float v[8] = {INFINITY, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const float4 u = scaled_point(means, n, i, inv);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      v[d] = fminf(v[d], comp(u, d));
      v[4 + d] = fmaxf(v[4 + d], comp(u, d));
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      v[d] = fminf(v[d], __shfl_xor(v[d], off, 64));
      v[4 + d] = fmaxf(v[4 + d], __shfl_xor(v[4 + d], off, 64));
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 8; ++c) s_v[wave][c] = v[c];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int c = threadIdx.x;
    float r = s_v[0][c];
    for (int w = 1; w < kBlock / 64; ++w) r = c < 4 ? fminf(r, s_v[w][c]) : fmaxf(r, s_v[w][c]);
    partials[blockIdx.x * 8 + c] = r;
  }
}

// One workgroup: the bounding box from the partials, then (thread 0) the cell
// width: the smallest h (to 64 bisection steps of its logarithm) with
// prod_d max(1, ceil(extent_d / h)) <= target cells.
__global__ __launch_bounds__(kBlock) void grid_setup_kernel(const float* __restrict__ partials,
                                                            uint32_t blocks, uint32_t target,
                                                            Grid4* __restrict__ grid) {
  __shared__ float s_v[kBlock / 64][8];
  __shared__ float s_box[8];
  float v[8] = {INFINITY, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (uint32_t b = threadIdx.x; b < blocks; b += kBlock)
#pragma unroll
    for (int c = 0; c < 8; ++c)
      v[c] = c < 4 ? fminf(v[c], partials[b * 8 + c]) : fmaxf(v[c], partials[b * 8 + c]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float o = __shfl_xor(v[c], off, 64);
      v[c] = c < 4 ? fminf(v[c], o) : fmaxf(v[c], o);
    }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int c = 0; c < 8; ++c) s_v[threadIdx.x >> 6][c] = v[c];
  __syncthreads();
  if (threadIdx.x < 8) {
    const int c = threadIdx.x;
    float r = s_v[0][c];
    for (int w = 1; w < kBlock / 64; ++w) r = c < 4 ? fminf(r, s_v[w][c]) : fmaxf(r, s_v[w][c]);
    s_box[c] = r;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double e[4], emax = 0.0;
  for (int d = 0; d < 4; ++d) {
    e[d] = double(s_box[4 + d]) - double(s_box[d]);
    emax = e[d] > emax ? e[d] : emax;
  }
  auto cells_for = [&](double h) {
    double p = 1.0;
    for (int d = 0; d < 4; ++d) {
      const double c = ceil(e[d] / h);
      p *= c > 1.0 ? c : 1.0;
    }
    return p;
  };
  double h = 1.0;
  if (emax > 0.0) {
    double hi = emax, lo = emax * 1e-7;  // cells_for(hi) == 1
    for (int it = 0; it < 64; ++it) {
      const double mid = sqrt(hi * lo);
      if (cells_for(mid) <= double(target))
        hi = mid;
      else
        lo = mid;
    }
    h = hi;
  }
  Grid4 g;
  // round the width up, so the cell count stays within the target
  float hf = float(h);
  if (double(hf) < h) hf = nextafterf(hf, INFINITY);
  uint32_t cells = 1;
  for (int d = 0; d < 4; ++d) {
    g.lo[d] = s_box[d];
    const double c = ceil(e[d] / double(hf));
    g.G[d] = c > 1.0 ? int(c) : 1;
    cells *= uint32_t(g.G[d]);
  }
  g.h = hf;
  g.inv_h = float(1.0 / double(hf));
  // the cell assignment rounds u - lo and its product with inv_h (relative
  // 2^-24 each) and inv_h itself: a point lies within a few 2^-24 (emax + h) of
  // its cell's box; 1e-6 is about 16 such roundings
  g.slack = float(1e-6 * (emax + h));
  g.cells = cells;
  *grid = g;
}

__global__ __launch_bounds__(kBlock) void cell_count_kernel(const float* __restrict__ means,
                                                            uint32_t n, float4 inv,
                                                            const Grid4* __restrict__ gridp,
                                                            uint32_t* __restrict__ counts,
                                                            uint32_t* __restrict__ cell_of,
                                                            uint32_t* __restrict__ rank) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const Grid4 g = *gridp;
  const float4 u = scaled_point(means, n, i, inv);
  int c[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) c[d] = cell_coord(comp(u, d), g.lo[d], g.inv_h, g.G[d]);
  const uint32_t id = cell_id(c, g);
  cell_of[i] = id;
  rank[i] = atomicAdd(&counts[id], 1u);
}

__global__ __launch_bounds__(kBlock) void cell_scatter_kernel(
    const float* __restrict__ means, uint32_t n, float4 inv, const uint32_t* __restrict__ starts,
    const uint32_t* __restrict__ cell_of, const uint32_t* __restrict__ rank,
    float4* __restrict__ su, uint32_t* __restrict__ sidx) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t pos = starts[cell_of[i]] + rank[i];
  su[pos] = scaled_point(means, n, i, inv);
  sidx[pos] = i;
}

// (d, j) ranks before (bd, bj)
__device__ __forceinline__ bool better(float d, uint32_t j, float bd, uint32_t bj) {
  return d < bd || (d == bd && j < bj);
}

// One thread per point, in cell order.  The K best candidates sit in the last
// K of KMAX register slots, sorted; the first KMAX - K slots hold -inf, which
// no candidate displaces.
template <int KMAX>
__global__ __launch_bounds__(kBlock) void knn_query_kernel(const float4* __restrict__ su,
                                                           const uint32_t* __restrict__ sidx,
                                                           const uint32_t* __restrict__ starts,
                                                           const Grid4* __restrict__ gridp,
                                                           uint32_t n, int k,
                                                           int32_t* __restrict__ out) {
  const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const Grid4 g = *gridp;
  const float4 q = su[p];
  const uint32_t qi = sidx[p];
  int c[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) c[d] = cell_coord(comp(q, d), g.lo[d], g.inv_h, g.G[d]);
  float bd[KMAX];
  uint32_t bi[KMAX];
#pragma unroll
  for (int s = 0; s < KMAX; ++s) {
    const bool dead = s < KMAX - k;
    bd[s] = dead ? -INFINITY : INFINITY;
    bi[s] = dead ? 0u : 0xffffffffu;
  }
  int rmax = 0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int a = c[d] > g.G[d] - 1 - c[d] ? c[d] : g.G[d] - 1 - c[d];
    rmax = a > rmax ? a : rmax;
  }
  // the points of sorted positions [b, e): cells that follow each other in x
  // are contiguous in the sorted order, so a run of cells is one range
  auto scan_range = [&](uint32_t b, uint32_t e) {
    for (uint32_t t = b; t < e; ++t) {
      const uint32_t j = sidx[t];
      const float dd = dist2(q, su[t]);
      if (j == qi || !better(dd, j, bd[KMAX - 1], bi[KMAX - 1])) continue;
#pragma unroll
      for (int s = KMAX - 1; s > 0; --s) {
        const bool up = better(dd, j, bd[s - 1], bi[s - 1]);
        const bool here = !up && better(dd, j, bd[s], bi[s]);
        bd[s] = up ? bd[s - 1] : (here ? dd : bd[s]);
        bi[s] = up ? bi[s - 1] : (here ? j : bi[s]);
      }
      if (better(dd, j, bd[0], bi[0])) {
        bd[0] = dd;
        bi[0] = j;
      }
    }
  };
  // gap2(d, a): the squared distance from q to the slab of cells with
  // coordinate a in dimension d (widened by the slack), in coordinates relative
  // to the box corner so that every rounding is relative to the box size; the
  // sum over the four dimensions bounds the distance to any point of a cell
  // from below (after a float32 rounding margin, applied in `pruned`)
  float qr[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) qr[d] = comp(q, d) - g.lo[d];
  auto gap2 = [&](int d, int a) {
    const float lo = float(a) * g.h;
    const float hi = float(a + 1) * g.h;
    float gap = fmaxf(lo - qr[d], qr[d] - hi) - g.slack;
    gap = gap > 0.f ? gap : 0.f;
    return gap * gap;
  };
  auto pruned = [&](float m) { return m * (1.0f - 1e-6f) > bd[KMAX - 1]; };
  for (int r = 0; r <= rmax; ++r) {
    if (r > 1 && bd[KMAX - 1] < INFINITY) {
      // shells 0 .. r - 1 are done: every unvisited point lies in a cell at
      // least r cells from q's in some coordinate, so more than (r - 1) h -
      // slack from q in that coordinate
      const float b = float(r - 1) * g.h * (1.0f - 1e-6f) - g.slack;
      if (b > 0.f && bd[KMAX - 1] < b * b * (1.0f - 1e-6f)) break;
    }
    // the cells at Chebyshev distance exactly r from c, clipped to the grid
    int lo[4], hi[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      lo[d] = c[d] - r > 0 ? c[d] - r : 0;
      hi[d] = c[d] + r < g.G[d] - 1 ? c[d] + r : g.G[d] - 1;
    }
    // the loop nest prunes whole slabs once their partial distance bound
    // exceeds the current k-th distance (the bound only grows inwards)
    auto visit = [&](int a[4], float m3) {
      if (pruned(m3 + gap2(0, a[0]))) return;
      const uint32_t id = cell_id(a, g);
      scan_range(starts[id], starts[id + 1]);
    };
    int a[4];
    for (a[3] = lo[3]; a[3] <= hi[3]; ++a[3]) {
      const float m3 = gap2(3, a[3]);
      if (pruned(m3)) continue;
      for (a[2] = lo[2]; a[2] <= hi[2]; ++a[2]) {
        const float m2 = m3 + gap2(2, a[2]);
        if (pruned(m2)) continue;
        for (a[1] = lo[1]; a[1] <= hi[1]; ++a[1]) {
          const float m1 = m2 + gap2(1, a[1]);
          if (pruned(m1)) continue;
          // with the other three strictly inside, only a0 = c0 - r and c0 + r
          const bool inner = r > 0 && abs(a[1] - c[1]) < r && abs(a[2] - c[2]) < r &&
                             abs(a[3] - c[3]) < r;
          if (inner) {
            a[0] = c[0] - r;
            if (a[0] >= 0) visit(a, m1);
            a[0] = c[0] + r;
            if (a[0] < g.G[0]) visit(a, m1);
          } else {
            // the x-run of cells lo[0] .. hi[0], trimmed at both ends to the
            // cells the bound does not prune (gap2 along x falls then rises)
            int x0 = lo[0], x1 = hi[0];
            while (x0 <= x1 && pruned(m1 + gap2(0, x0))) ++x0;
            while (x1 >= x0 && pruned(m1 + gap2(0, x1))) --x1;
            if (x0 <= x1) {
              a[0] = x0;
              const uint32_t id0 = cell_id(a, g);
              scan_range(starts[id0], starts[id0 + uint32_t(x1 - x0) + 1]);
            }
          }
        }
      }
    }
  }
  int32_t* o = out + size_t(qi) * size_t(k);
#pragma unroll
  for (int s = 0; s < KMAX; ++s)
    if (s >= KMAX - k) o[s - (KMAX - k)] = int32_t(bi[s]);
}

// ---- consistency loss

template <typename T>
struct alignas(sizeof(T) * 4) Speed {
  T x, y, z, pad;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void speed_kernel(GaussPtrs<T> g, Speed<T>* __restrict__ sp) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T ls[4], rot[8];
#pragma unroll
  for (int c = 0; c < 4; ++c) ls[c] = g.log_scales[c * (long)n + i];
#pragma unroll
  for (int c = 0; c < 8; ++c) rot[c] = g.rotors[c * (long)n + i];
  Fwd<T> f;
  cov4_fwd(ls, rot, f);
  const T iw = T(1) / f.W;
  sp[i] = Speed<T>{f.V[0] * iw, f.V[1] * iw, f.V[2] * iw, T(0)};
}

template <typename T>
__device__ __forceinline__ int sgn(T x) {
  return x > T(0) ? 1 : (x < T(0) ? -1 : 0);
}

// The three sign sums of a Gaussian packed in one 64-bit word, 21-bit two's
// complement fields at bits 0, 21 and 42: adding packed words adds the fields
// as long as no field's sum leaves [-2^20, 2^20), which holds when fewer than
// 2^20 Gaussians can name it as a neighbour (n <= 2^20).  One atomic per
// neighbour instead of three.
constexpr uint32_t kPackedSignsMaxN = 1u << 20;

__device__ __forceinline__ unsigned long long pack_signs(int g0, int g1, int g2) {
  return uint64_t(int64_t(g0)) + (uint64_t(int64_t(g1)) << 21) + (uint64_t(int64_t(g2)) << 42);
}

__device__ __forceinline__ int sext21(uint64_t v) {
  const int x = int(v & 0x1fffffu);
  return x >= (1 << 20) ? x - (1 << 21) : x;
}

__device__ __forceinline__ void unpack_signs(uint64_t w, int& g0, int& g1, int& g2) {
  g0 = sext21(w);
  w = (w - uint64_t(int64_t(g0))) >> 21;
  g1 = sext21(w);
  w = (w - uint64_t(int64_t(g1))) >> 21;
  g2 = sext21(w);
}

// Per Gaussian: d = s_i - mean of its neighbours' speeds; |d|_1 summed per
// workgroup into partials; sign(d) stored; sign(d) gathered onto every
// neighbour with integer atomics (one packed 64-bit atomic each when PACKED,
// else one 32-bit atomic per component).  Neighbour indices outside [0, n)
// are skipped.
template <typename T, bool PACKED>
__global__ __launch_bounds__(kBlock) void consistency_fwd_kernel(
    const Speed<T>* __restrict__ sp, const int32_t* __restrict__ nb, int k, uint32_t n,
    char4* __restrict__ sign_out, int32_t* __restrict__ gather, T* __restrict__ partials) {
  __shared__ T s_part[kBlock / 64];
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  T part = T(0);
  if (i < n) {
    T m0 = 0, m1 = 0, m2 = 0;
    const int32_t* row = nb + size_t(i) * size_t(k);
    for (int a = 0; a < k; ++a) {
      const uint32_t j = uint32_t(row[a]);
      if (j >= n) continue;
      const Speed<T> v = sp[j];
      m0 += v.x;
      m1 += v.y;
      m2 += v.z;
    }
    const T ik = T(1) / T(k);
    const Speed<T> s = sp[i];
    const T d0 = s.x - m0 * ik, d1 = s.y - m1 * ik, d2 = s.z - m2 * ik;
    part = fabs(d0) + fabs(d1) + fabs(d2);
    const int g0 = sgn(d0), g1 = sgn(d1), g2 = sgn(d2);
    sign_out[i] = make_char4(char(g0), char(g1), char(g2), 0);
    const unsigned long long pk = pack_signs(g0, g1, g2);
    for (int a = 0; a < k; ++a) {
      const uint32_t j = uint32_t(row[a]);
      if (j >= n) continue;
      int32_t* gj = gather + 4 * size_t(j);
      if (PACKED) {
        if (pk) atomicAdd(reinterpret_cast<unsigned long long*>(gj), pk);
      } else {
        if (g0) atomicAdd(gj, g0);
        if (g1) atomicAdd(gj + 1, g1);
        if (g2) atomicAdd(gj + 2, g2);
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

// *loss = (sum of partials) / n, in a fixed order (one workgroup).
template <typename T>
__global__ __launch_bounds__(kBlock) void loss_total_kernel(const T* __restrict__ partials,
                                                            uint32_t count, uint32_t n,
                                                            T* __restrict__ loss) {
  __shared__ T s_part[kBlock / 64];
  T part = T(0);
  for (uint32_t b = threadIdx.x; b < count; b += kBlock) part += partials[b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) *loss = ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) / T(n);
}

// dL/ds_i = (sign(d_i) - gather_i / K) / N, times `weight`, through s = V / W
// (dV = ds / W, dW = -(ds . s) / W) into Sigma_4, then to the log-scales and
// raw rotor; added to the outputs.
template <typename T, bool PACKED>
__global__ __launch_bounds__(kBlock) void consistency_bwd_kernel(
    GaussPtrs<T> g, const char4* __restrict__ signs, const int32_t* __restrict__ gather, int k,
    T scale, T* __restrict__ grot, T* __restrict__ gls) {
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const char4 sg = signs[i];
  int ga[3];
  if (PACKED) {
    unpack_signs(*reinterpret_cast<const unsigned long long*>(gather + 4 * size_t(i)), ga[0],
                 ga[1], ga[2]);
  } else {
    const int4 w = *reinterpret_cast<const int4*>(gather + 4 * size_t(i));
    ga[0] = w.x;
    ga[1] = w.y;
    ga[2] = w.z;
  }
  const T ik = T(1) / T(k);
  const T gs[3] = {scale * (T(sg.x) - T(ga[0]) * ik), scale * (T(sg.y) - T(ga[1]) * ik),
                   scale * (T(sg.z) - T(ga[2]) * ik)};
  if (gs[0] == T(0) && gs[1] == T(0) && gs[2] == T(0)) return;
  T ls[4], rot[8];
#pragma unroll
  for (int c = 0; c < 4; ++c) ls[c] = g.log_scales[c * (long)n + i];
#pragma unroll
  for (int c = 0; c < 8; ++c) rot[c] = g.rotors[c * (long)n + i];
  Fwd<T> f;
  cov4_fwd(ls, rot, f);
  const T iw = T(1) / f.W;
  const T s[3] = {f.V[0] * iw, f.V[1] * iw, f.V[2] * iw};
  T G4[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) G4[e] = T(0);
  // a unique off-diagonal entry V_c = Sigma_c3 = Sigma_3c: half its gradient
  // in each symmetric position
  G4[3] = G4[12] = T(0.5) * gs[0] * iw;
  G4[7] = G4[13] = T(0.5) * gs[1] * iw;
  G4[11] = G4[14] = T(0.5) * gs[2] * iw;
  G4[15] = -(gs[0] * s[0] + gs[1] * s[1] + gs[2] * s[2]) * iw;
  T gl[4] = {0, 0, 0, 0}, gr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  cov4_bwd(f, G4, gl, gr);
#pragma unroll
  for (int c = 0; c < 4; ++c) gls[c * (long)n + i] += gl[c];
#pragma unroll
  for (int c = 0; c < 8; ++c) grot[c * (long)n + i] += gr[c];
}

uint32_t knn_cells_cap(uint32_t n) { return n / kCellPoints > 1u ? n / kCellPoints : 1u; }

}  // namespace

// temp layout: bound partials | grid | counts/starts (cap + 1 each) | scan
// scratch | cell_of, rank (n each) | su (16 n) | sidx (4 n)
size_t knn4d_temp_bytes(uint32_t n) {
  const size_t cap = knn_cells_cap(n);
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  return a(kBoundBlocks * 8 * 4) + a(sizeof(Grid4)) + 2 * a((cap + 1) * 4) +
         a(scan_u32_temp_bytes(uint32_t(cap))) + 2 * a(size_t(n) * 4) + a(size_t(n) * 16) +
         a(size_t(n) * 4);
}

hipError_t launch_knn4d(const float* means, uint32_t n, int k, float inv_spatial,
                        float inv_temporal, int32_t* out, void* temp, hipStream_t stream) {
  if (n < 2 || k < 1 || k > 32 || uint32_t(k) >= n) return hipErrorInvalidValue;
  const uint32_t cap = knn_cells_cap(n);
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  uint8_t* p = static_cast<uint8_t*>(temp);
  float* partials = reinterpret_cast<float*>(p);
  p += a(kBoundBlocks * 8 * 4);
  Grid4* grid = reinterpret_cast<Grid4*>(p);
  p += a(sizeof(Grid4));
  uint32_t* counts = reinterpret_cast<uint32_t*>(p);
  p += a((size_t(cap) + 1) * 4);
  uint32_t* starts = reinterpret_cast<uint32_t*>(p);
  p += a((size_t(cap) + 1) * 4);
  void* scan_tmp = p;
  p += a(scan_u32_temp_bytes(cap));
  uint32_t* cell_of = reinterpret_cast<uint32_t*>(p);
  p += a(size_t(n) * 4);
  uint32_t* rank = reinterpret_cast<uint32_t*>(p);
  p += a(size_t(n) * 4);
  float4* su = reinterpret_cast<float4*>(p);
  p += a(size_t(n) * 16);
  uint32_t* sidx = reinterpret_cast<uint32_t*>(p);
  const float4 inv = make_float4(inv_spatial, inv_spatial, inv_spatial, inv_temporal);
  const uint32_t blocks = (n + kBlock - 1) / kBlock;
  const uint32_t bblocks = blocks < uint32_t(kBoundBlocks) ? blocks : uint32_t(kBoundBlocks);
  hipError_t e = fill_zero(counts, a((size_t(cap) + 1) * 4), stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bounds_kernel, dim3(bblocks), dim3(kBlock), 0, stream, means, n, inv, partials);
  hipLaunchKernelGGL(grid_setup_kernel, dim3(1), dim3(kBlock), 0, stream, partials, bblocks, cap,
                     grid);
  hipLaunchKernelGGL(cell_count_kernel, dim3(blocks), dim3(kBlock), 0, stream, means, n, inv, grid,
                     counts, cell_of, rank);
  if ((e = scan_u32(counts, cap, starts, scan_tmp, stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(cell_scatter_kernel, dim3(blocks), dim3(kBlock), 0, stream, means, n, inv,
                     starts, cell_of, rank, su, sidx);
  if (k <= 8)
    hipLaunchKernelGGL(knn_query_kernel<8>, dim3(blocks), dim3(kBlock), 0, stream, su, sidx,
                       starts, grid, n, k, out);
  else if (k <= 16)
    hipLaunchKernelGGL(knn_query_kernel<16>, dim3(blocks), dim3(kBlock), 0, stream, su, sidx,
                       starts, grid, n, k, out);
  else
    hipLaunchKernelGGL(knn_query_kernel<32>, dim3(blocks), dim3(kBlock), 0, stream, su, sidx,
                       starts, grid, n, k, out);
  return hipGetLastError();
}

// temp layout: speeds (4 T per Gaussian) | signs (4 B) | gather (16 B) |
// partials (one T per workgroup)
template <typename T>
size_t consistency_temp_bytes(uint32_t n) {
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t blocks = (size_t(n) + kBlock - 1) / kBlock;
  return a(size_t(n) * 4 * sizeof(T)) + a(size_t(n) * 4) + a(size_t(n) * 16) +
         a(blocks * sizeof(T));
}

template <typename T>
hipError_t launch_consistency(const GaussPtrs<T>& g, const int32_t* nb, int k, T weight, T* loss,
                              T* grad_rotors, T* grad_log_scales, void* temp,
                              hipStream_t stream) {
  const uint32_t n = uint32_t(g.n);
  if (g.n < 2 || k < 1 || uint32_t(k) >= n) return hipErrorInvalidValue;
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  const uint32_t blocks = (n + kBlock - 1) / kBlock;
  uint8_t* p = static_cast<uint8_t*>(temp);
  Speed<T>* sp = reinterpret_cast<Speed<T>*>(p);
  p += a(size_t(n) * 4 * sizeof(T));
  char4* signs = reinterpret_cast<char4*>(p);
  p += a(size_t(n) * 4);
  int32_t* gather = reinterpret_cast<int32_t*>(p);
  p += a(size_t(n) * 16);
  T* partials = reinterpret_cast<T*>(p);
  hipError_t e = fill_zero(gather, a(size_t(n) * 16), stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(speed_kernel<T>, dim3(blocks), dim3(kBlock), 0, stream, g, sp);
  const bool packed = n <= kPackedSignsMaxN;
  if (packed)
    hipLaunchKernelGGL((consistency_fwd_kernel<T, true>), dim3(blocks), dim3(kBlock), 0, stream,
                       sp, nb, k, n, signs, gather, partials);
  else
    hipLaunchKernelGGL((consistency_fwd_kernel<T, false>), dim3(blocks), dim3(kBlock), 0, stream,
                       sp, nb, k, n, signs, gather, partials);
  if (loss)
    hipLaunchKernelGGL(loss_total_kernel<T>, dim3(1), dim3(kBlock), 0, stream, partials, blocks, n,
                       loss);
  if (grad_rotors && grad_log_scales) {
    if (packed)
      hipLaunchKernelGGL((consistency_bwd_kernel<T, true>), dim3(blocks), dim3(kBlock), 0, stream,
                         g, signs, gather, k, weight / T(n), grad_rotors, grad_log_scales);
    else
      hipLaunchKernelGGL((consistency_bwd_kernel<T, false>), dim3(blocks), dim3(kBlock), 0,
                         stream, g, signs, gather, k, weight / T(n), grad_rotors,
                         grad_log_scales);
  }
  return hipGetLastError();
}

#define R4D_INST(T)                                                                          \
  template size_t consistency_temp_bytes<T>(uint32_t);                                       \
  template hipError_t launch_consistency<T>(const GaussPtrs<T>&, const int32_t*, int, T, T*, \
                                            T*, T*, void*, hipStream_t);
R4D_INST(float)
R4D_INST(double)
#undef R4D_INST

}  // namespace r4d
