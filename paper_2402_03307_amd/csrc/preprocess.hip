// Per-Gaussian preprocess kernels: one thread per Gaussian, SoA loads that are
// coalesced across a wavefront, SH coefficients read only for Gaussians that
// survive the time / near-plane culls.
//
// Forward writes the projected record consumed by the rasteriser, the tiles'
// bounding box, the tile count and the depth sort key.  Backward recomputes the
// forward intermediates from the parameters (nothing per Gaussian is stored
// between the passes except the 9 screen-space gradients) and chains them
// back to the parameters.
#include <hip/hip_runtime.h>

#include "r4d_internal.hpp"
#include "rowwalk.hpp"
#include "tileset.hpp"

namespace r4d {

namespace {

constexpr int kBlock = 256;

// qmax of a record: min(extent^2, 2 ln(o / alpha_min)), rounded up to T so that
// the stored bound never excludes a pixel the double value admits.  Negative
// (the Gaussian is never blended) when o < alpha_min.
template <typename T>
__device__ __forceinline__ T record_qmax(T o, const SettingsDev& st);

template <>
__device__ __forceinline__ double record_qmax<double>(double o, const SettingsDev& st) {
  if (!(o >= double(st.alpha_min))) return -1.0;
  const double Q = 2.0 * (log(o) - double(st.log_alpha_min));
  return Q < double(st.ext2) ? Q : double(st.ext2);
}

template <>
__device__ __forceinline__ float record_qmax<float>(float o, const SettingsDev& st) {
  const double Q = record_qmax<double>(double(o), st);
  float f = float(Q);
  if (double(f) < Q) f = __uint_as_float(__float_as_uint(f) + 1u);  // Q >= 0 here
  return f;
}

// Tile box and run constants of a record; false when no pixel can receive it.
template <typename T>
__device__ __forceinline__ bool record_box(const Rec<T>& rec, const ViewDev& v, int sh,
                                           TileBox& bx, SpanGeom& sg) {
  const double Q = double(rec.qmax);
  if (!(Q >= 0.0)) return false;
  const double mx = double(rec.mx), my = double(rec.my);
  const double a = double(rec.ca), b = double(rec.cb), c = double(rec.cc);
  if (!tile_box(mx, my, a, b, c, Q, v.W, v.H, sh, bx)) return false;
  sg = span_geom(mx, my, a, b, c, Q, v.W, v.H, sh, bx.x0, bx.x1);
  return true;
}

template <typename T, int DEG>
__global__ __launch_bounds__(kBlock) void preprocess_fwd_kernel(
    GaussPtrs<T> g, const ViewSlot* __restrict__ slots, SettingsDev st, uint32_t n_pad,
    Rec<T>* __restrict__ recs, Rect16* __restrict__ rects, uint32_t* __restrict__ tiles_touched,
    uint32_t* __restrict__ depth_keys, ulonglong2* __restrict__ block_totals) {
  __shared__ unsigned long long s_tot[2][kBlock / 64];
  __shared__ uint32_t s_cnt[kBlock];
  __shared__ int s_x0[kBlock], s_x1[kBlock], s_y0[kBlock], s_y1[kBlock];
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int vi = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const ViewDev v = slots[vi].v;
  const int sh = __builtin_ctz(unsigned(v.tile_size));
  const size_t row = size_t(vi) * size_t(n);
  TileBox bx = {0, 0, 0, 0};
  SpanGeom sg = {};
  sg.W = v.W;
  sg.H = v.H;
  sg.sh = sh;
  float depth = 0.0f;
  if (i < n) {
    T mu[4], ls[4], rot[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mu[c] = g.means[c * (long)n + i];
      ls[c] = g.log_scales[c * (long)n + i];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) rot[c] = g.rotors[c * (long)n + i];
    const T op = g.opacity[i];
    Fwd<T> f;
    gaussian_fwd<T>(mu, ls, rot, op, g.sh + i, (long)n, DEG, v, st, f);
    if (f.valid) {
      Rec<T> rec;
      rec.mx = f.mean2[0];
      rec.my = f.mean2[1];
      rec.ca = f.conic[0];
      rec.cb = f.conic[1];
      rec.cc = f.conic[2];
      rec.o = f.o_t;
      rec.depth = f.p[2];
      rec.qmax = record_qmax<T>(f.o_t, st);
      rec.r = f.rgb[0];
      rec.g = f.rgb[1];
      rec.b = f.rgb[2];
      rec.pad1 = T(0);
      if (record_box(rec, v, sh, bx, sg)) {
        recs[row + i] = rec;
        depth = float(f.p[2]);
      } else {
        bx = {0, 0, 0, 0};
      }
    }
  }
  // tile entries and the runs' bounding box: the rows of the wavefront's
  // Gaussians walked together, aggregated per Gaussian in LDS
  s_cnt[threadIdx.x] = 0u;
  s_x0[threadIdx.x] = 0x7fffffff;
  s_x1[threadIdx.x] = 0;
  s_y0[threadIdx.x] = 0x7fffffff;
  s_y1[threadIdx.x] = 0;
  __syncthreads();
  wave_rows(sg, bx.y0, bx.y1, lane, [&](bool ok, int o, int y, int x0, int x1) {
    if (ok && x0 < x1) {
      const int slot = wave * 64 + o;
      atomicAdd(&s_cnt[slot], uint32_t(x1 - x0));
      atomicMin(&s_x0[slot], x0);
      atomicMax(&s_x1[slot], x1);
      atomicMin(&s_y0[slot], y);
      atomicMax(&s_y1[slot], y + 1);
    }
  });
  __syncthreads();
  const uint32_t my_cnt = s_cnt[threadIdx.x];
  const bool vis = my_cnt > 0u;
  if (i < n) {
    Rect16 rc = {0, 0, 0, 0};
    if (vis) {
      rc.x0 = uint16_t(s_x0[threadIdx.x]);
      rc.x1 = uint16_t(s_x1[threadIdx.x]);
      rc.y0 = uint16_t(s_y0[threadIdx.x]);
      rc.y1 = uint16_t(s_y1[threadIdx.x]);
    }
    rects[row + i] = rc;
    tiles_touched[row + i] = my_cnt;
    depth_keys[size_t(vi) * n_pad + i] = vis ? __float_as_uint(depth) : 0xffffffffu;
  }
  // block totals of visible Gaussians and tile entries, written per block and
  // summed by totals_kernel (atomics on two addresses from every block would
  // serialise)
  unsigned long long c = my_cnt;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
  const unsigned long long m = __ballot(vis);
  if (lane == 0) {
    s_tot[0][wave] = __popcll(m);
    s_tot[1][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      a += s_tot[0][w];
      b += s_tot[1][w];
    }
    block_totals[size_t(vi) * gridDim.x + blockIdx.x] = make_ulonglong2(a, b);
  }
}

// totals[2v] = visible Gaussians of render v, totals[2v + 1] = its tile
// entries: the sum of the render's block totals (one workgroup per render).
__global__ __launch_bounds__(kBlock) void totals_kernel(const ulonglong2* __restrict__ block_totals,
                                                         uint32_t blocks,
                                                         unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long s_a[kBlock / 64], s_b[kBlock / 64];
  const uint32_t v = blockIdx.x;
  unsigned long long a = 0, b = 0;
  for (uint32_t i = threadIdx.x; i < blocks; i += kBlock) {
    const ulonglong2 t = block_totals[size_t(v) * blocks + i];
    a += t.x;
    b += t.y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_a[threadIdx.x >> 6] = a;
    s_b[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long ta = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      ta += s_a[w];
      tb += s_b[w];
    }
    totals[2 * v] = ta;
    totals[2 * v + 1] = tb;
  }
}

// Degree-specialised so that the SH loops unroll and the coefficient arrays
// live in registers.  Each thread owns one Gaussian and sums its gradients
// over the renders, recomputing the forward of each render it appears in.
// With one render the SH coefficients are loaded once into registers; with
// several they are re-read from memory (cached) in every render, which keeps
// the register count of the render loop at that of the single-render case.
template <typename T, int DEG, bool MULTI>
__global__ __launch_bounds__(kBlock) void preprocess_bwd_kernel(GaussPtrs<T> g,
                                                                const ViewSlot* __restrict__ slots,
                                                                int n_views, SettingsDev st,
                                                                const double* __restrict__ grad2d,
                                                                GradPtrs<T> out) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  T gmu[4] = {0, 0, 0, 0}, gls[4] = {0, 0, 0, 0}, grot[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gop = 0;
  T gsh[3 * K];
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) gsh[j] = T(0);
  const int nv = MULTI ? n_views : 1;
  for (int vi = 0; vi < nv; ++vi) {
    const double* g2v = grad2d + size_t(vi) * 9 * size_t(n);
    T g2[9];
    bool any = false;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      g2[c] = T(g2v[c * (long)n + i]);
      any |= g2[c] != T(0);
    }
    if (!any) continue;
    T mu[4], ls[4], rot[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mu[c] = g.means[c * (long)n + i];
      ls[c] = g.log_scales[c * (long)n + i];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) rot[c] = g.rotors[c * (long)n + i];
    const ViewDev v = slots[vi].v;
    Fwd<T> f;
    if (MULTI) {
      gaussian_fwd<T>(mu, ls, rot, g.opacity[i], g.sh + i, (long)n, DEG, v, st, f);
      gaussian_bwd<T>(f, g.sh + i, (long)n, DEG, v, g2, gmu, gls, grot, gop, gsh, 1L);
    } else {
      T shl[3 * K];
#pragma unroll
      for (int j = 0; j < 3 * K; ++j) shl[j] = g.sh[j * (long)n + i];
      gaussian_fwd<T>(mu, ls, rot, g.opacity[i], shl, 1, DEG, v, st, f);
      gaussian_bwd<T>(f, shl, 1, DEG, v, g2, gmu, gls, grot, gop, gsh, 1L);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    out.means[c * (long)n + i] = gmu[c];
    out.log_scales[c * (long)n + i] = gls[c];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) out.rotors[c * (long)n + i] = grot[c];
  out.opacity[i] = gop;
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) out.sh[j * (long)n + i] = gsh[j];
}

}  // namespace

#define R4D_DEG_DISPATCH(KERNEL, GRID, ...)                                              \
  switch (g.deg) {                                                                       \
    case 0: hipLaunchKernelGGL((KERNEL<T, 0>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 1: hipLaunchKernelGGL((KERNEL<T, 1>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 3: hipLaunchKernelGGL((KERNEL<T, 3>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                \
  }

template <typename T>
hipError_t launch_preprocess_fwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, uint32_t n_pad, Rec<T>* recs,
                                 Rect16* rects, uint32_t* tiles_touched, uint32_t* depth_keys,
                                 unsigned long long* totals, void* temp, hipStream_t stream) {
  if (g.n <= 0 || n_views <= 0) return hipSuccess;
  const uint32_t blocks = uint32_t((g.n + kBlock - 1) / kBlock);
  const dim3 grid(blocks, uint32_t(n_views));
  ulonglong2* block_totals = static_cast<ulonglong2*>(temp);
  R4D_DEG_DISPATCH(preprocess_fwd_kernel, grid, g, slots, st, n_pad, recs, rects, tiles_touched,
                   depth_keys, block_totals)
  hipLaunchKernelGGL(totals_kernel, dim3(uint32_t(n_views)), dim3(kBlock), 0, stream, block_totals,
                     blocks, totals);
  return hipGetLastError();
}

size_t preprocess_temp_bytes(uint32_t n, int n_views) {
  return size_t((n + kBlock - 1) / kBlock) * size_t(n_views) * sizeof(ulonglong2);
}

template <typename T>
hipError_t launch_preprocess_bwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, const double* grad2d,
                                 const GradPtrs<T>& out, hipStream_t stream) {
  if (g.n <= 0) return hipSuccess;
  const dim3 grid((g.n + kBlock - 1) / kBlock);
#define R4D_BWD_DISPATCH(MULTI)                                                              \
  switch (g.deg) {                                                                           \
    case 0: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 0, MULTI>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 1: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 1, MULTI>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 2: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 2, MULTI>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 3: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 3, MULTI>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    default: return hipErrorInvalidValue;                                                    \
  }
  if (n_views > 1) {
    R4D_BWD_DISPATCH(true)
  } else {
    R4D_BWD_DISPATCH(false)
  }
#undef R4D_BWD_DISPATCH
  return hipGetLastError();
}

#undef R4D_DEG_DISPATCH

#define R4D_INST(T)                                                                           \
  template hipError_t launch_preprocess_fwd<T>(const GaussPtrs<T>&, const ViewSlot*, int,      \
                                               const SettingsDev&, uint32_t, Rec<T>*, Rect16*, \
                                               uint32_t*, uint32_t*, unsigned long long*,      \
                                               void*, hipStream_t);                            \
  template hipError_t launch_preprocess_bwd<T>(const GaussPtrs<T>&, const ViewSlot*, int,      \
                                               const SettingsDev&, const double*,              \
                                               const GradPtrs<T>&, hipStream_t);
R4D_INST(float)
R4D_INST(double)
#undef R4D_INST

}  // namespace r4d
