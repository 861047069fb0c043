// Per-Gaussian preprocess kernels: one thread per Gaussian, SoA loads that are
// coalesced across a wavefront, SH coefficients read only for Gaussians that
// survive the time / near-plane culls.
//
// Forward writes the projected record consumed by the rasteriser, the tiles'
// bounding box, the tile count and the depth sort key (and, for a flow render,
// the Gaussian's 2D flow).  A static set (3D Gaussians: means, log-scales and
// quaternions with 3, 3 and 4 rows) skips the rotor, Sigma_4 and the slice.  Backward recomputes the forward intermediates from
// the parameters (nothing per Gaussian is stored between the passes except the
// 9, or with flow 11, screen-space gradients) and chains them back to the
// parameters.
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

// STATIC: a set of static 3D Gaussians (means [3][n], log-scales [3][n],
// quaternions [4][n] in the rotor slot) rendered with no slicing.
template <typename T, int DEG, bool STATIC>
__global__ __launch_bounds__(kBlock) void preprocess_fwd_kernel(
    GaussPtrs<T> g, const ViewSlot* __restrict__ slots, SettingsDev st, uint32_t n_pad,
    Rec<T>* __restrict__ recs, Vec2<T>* __restrict__ flows, Rect16* __restrict__ rects,
    uint32_t* __restrict__ tiles_touched, uint32_t* __restrict__ depth_keys,
    ulonglong2* __restrict__ block_totals, uint4* __restrict__ zero, uint64_t zero16,
    uint32_t n_views) {
  // per-Gaussian aggregates of the row walk, in kCopies copies picked by the
  // row's lane (consecutive rows of one Gaussian sit in consecutive lanes, so
  // its atomics spread over the copies instead of piling onto one address);
  // copies kStride words apart, so that one slot's copies fall in different banks
  constexpr int kCopies = 4, kStride = kBlock + 1;
  __shared__ unsigned long long s_tot[2][kBlock / 64];
  __shared__ uint32_t s_cnt[kCopies * kStride];
  __shared__ int s_x0[kCopies * kStride], s_x1[kCopies * kStride], s_y0[kCopies * kStride],
      s_y1[kCopies * kStride];
  const int n = g.n;
  // renders vary fastest over the workgroups, so that the workgroups of one
  // block of Gaussians run together and share its parameters in the caches
  const uint32_t vi = blockIdx.x % n_views, blk = blockIdx.x / n_views;
  const uint32_t nblk = gridDim.x / n_views;
  const int i = int(blk) * kBlock + int(threadIdx.x);
  // the run's counters and status words, cleared here for the later stages
  for (uint64_t z = uint64_t(blockIdx.x) * kBlock + threadIdx.x; z < zero16;
       z += uint64_t(gridDim.x) * kBlock)
    zero[z] = make_uint4(0u, 0u, 0u, 0u);
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
    const T op = g.opacity[i];
    Fwd<T> f;
    if (STATIC) {
      T mu[3], ls[3], q[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        mu[c] = g.means[c * (long)n + i];
        ls[c] = g.log_scales[c * (long)n + i];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = g.rotors[c * (long)n + i];
      gaussian_fwd_static<T>(mu, ls, q, op, g.sh + i, (long)n, DEG, v, st, f);
    } else {
      T mu[4], ls[4], rot[8];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        mu[c] = g.means[c * (long)n + i];
        ls[c] = g.log_scales[c * (long)n + i];
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) rot[c] = g.rotors[c * (long)n + i];
      gaussian_fwd<T>(mu, ls, rot, op, g.sh + i, (long)n, DEG, v, st, f);
    }
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
        if (flows) flows[row + i] = Vec2<T>{f.flow[0], f.flow[1]};
        depth = float(f.p[2]);
      } else {
        bx = {0, 0, 0, 0};
      }
    }
  }
  // tile entries and the runs' bounding box: the rows of the wavefront's
  // Gaussians walked together, aggregated per Gaussian in LDS
#pragma unroll
  for (int c = 0; c < kCopies; ++c) {
    const int q = c * kStride + int(threadIdx.x);
    s_cnt[q] = 0u;
    s_x0[q] = 0x7fffffff;
    s_x1[q] = 0;
    s_y0[q] = 0x7fffffff;
    s_y1[q] = 0;
  }
  __syncthreads();
  wave_rows(sg, bx.y0, bx.y1, lane, [&](bool ok, int o, int y, int x0, int x1) {
    if (ok && x0 < x1) {
      const int slot = (lane & (kCopies - 1)) * kStride + wave * 64 + o;
      atomicAdd(&s_cnt[slot], uint32_t(x1 - x0));
      atomicMin(&s_x0[slot], x0);
      atomicMax(&s_x1[slot], x1);
      atomicMin(&s_y0[slot], y);
      atomicMax(&s_y1[slot], y + 1);
    }
  });
  __syncthreads();
  uint32_t my_cnt = 0;
  int ax0 = 0x7fffffff, ax1 = 0, ay0 = 0x7fffffff, ay1 = 0;
#pragma unroll
  for (int c = 0; c < kCopies; ++c) {
    const int q = c * kStride + int(threadIdx.x);
    my_cnt += s_cnt[q];
    ax0 = min(ax0, s_x0[q]);
    ax1 = max(ax1, s_x1[q]);
    ay0 = min(ay0, s_y0[q]);
    ay1 = max(ay1, s_y1[q]);
  }
  const bool vis = my_cnt > 0u;
  if (i < n) {
    Rect16 rc = {0, 0, 0, 0};
    if (vis) {
      rc.x0 = uint16_t(ax0);
      rc.x1 = uint16_t(ax1);
      rc.y0 = uint16_t(ay0);
      rc.y1 = uint16_t(ay1);
    }
    rects[row + i] = rc;
    tiles_touched[row + i] = my_cnt;
    depth_keys[size_t(vi) * n_pad + i] = vis ? __float_as_uint(depth) : 0xffffffffu;
  }
  // block totals of visible Gaussians and tile entries, written per block and
  // summed by the compaction (atomics on two addresses from every block would
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
    block_totals[size_t(vi) * nblk + blk] = make_ulonglong2(a, b);
  }
}

// Exclusive scan of one value per thread over a workgroup of kBlock threads;
// *total receives the sum.
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x,
                                                              unsigned long long* s_w,
                                                              unsigned long long* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  unsigned long long before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    before += w < wave ? s_w[w] : 0ull;
    all += s_w[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// Compaction of the visible Gaussians' depth keys (index order kept), and the
// per-render totals.  Block b of render v adds up the block totals of the
// render's earlier blocks itself (a few loads per thread, no separate scan
// launch), writes its visible Gaussians from there on, and the render's last
// block writes totals[2v] = visible Gaussians, totals[2v + 1] = tile entries
// and dseg->len[v] = totals[2v].
__global__ __launch_bounds__(kBlock) void compact_keys_kernel(
    const uint32_t* __restrict__ depth_keys, uint32_t n, uint32_t n_pad,
    const ulonglong2* __restrict__ block_totals, unsigned long long* __restrict__ totals,
    SegTable* __restrict__ dseg, uint32_t* __restrict__ vis_keys,
    uint32_t* __restrict__ vis_index) {
  __shared__ uint32_t s_cnt[kBlock / 64];
  __shared__ unsigned long long s_sum[2][kBlock / 64];
  const uint32_t v = blockIdx.y, b = blockIdx.x, nb = gridDim.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool last = b + 1 == nb;
  const ulonglong2* bt = block_totals + size_t(v) * nb;
  unsigned long long before = 0, entries = 0;
  for (uint32_t j = threadIdx.x; j < (last ? nb : b); j += kBlock) {
    const ulonglong2 t = bt[j];
    before += j < b ? t.x : 0ull;
    entries += t.y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    before += __shfl_xor(before, off, 64);
    entries += __shfl_xor(entries, off, 64);
  }
  const uint32_t i = b * kBlock + threadIdx.x;
  const uint32_t key = i < n ? depth_keys[size_t(v) * n_pad + i] : 0xffffffffu;
  const bool vis = key != 0xffffffffu;
  const unsigned long long m = __ballot(vis);
  if (lane == 0) {
    s_cnt[wave] = uint32_t(__popcll(m));
    s_sum[0][wave] = before;
    s_sum[1][wave] = entries;
  }
  __syncthreads();
  unsigned long long start = 0, all_entries = 0;
  uint32_t mine = uint32_t(__popcll(m & ((1ull << lane) - 1ull))), in_block = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    start += s_sum[0][w];
    all_entries += s_sum[1][w];
    mine += w < wave ? s_cnt[w] : 0u;
    in_block += s_cnt[w];
  }
  if (vis) {
    vis_keys[size_t(v) * n_pad + start + mine] = key;
    vis_index[size_t(v) * n_pad + start + mine] = i;
  }
  if (last && threadIdx.x == 0) {
    totals[2 * v] = start + in_block;
    totals[2 * v + 1] = all_entries;
    dseg->len[v] = uint32_t(start + in_block);
  }
}

// Degree-specialised so that the SH loops unroll and the coefficient arrays
// live in registers.  Each thread owns one Gaussian and sums its gradients
// over the renders, recomputing the forward of each render it appears in.
// With one render the SH coefficients are loaded once into registers; with
// several they are re-read from memory (cached) in every render, which keeps
// the register count of the render loop at that of the single-render case.
template <typename T, int DEG, bool MULTI, bool FLOW, bool STATIC>
__global__ __launch_bounds__(kBlock) void preprocess_bwd_kernel(GaussPtrs<T> g,
                                                                const ViewSlot* __restrict__ slots,
                                                                int n_views, SettingsDev st,
                                                                const double* __restrict__ grad2d,
                                                                GradPtrs<T> out) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int NC = FLOW ? 11 : 9;
  const int n = g.n;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  // (a static Gaussian uses the first 3, 3 and 4 entries)
  T gmu[4] = {0, 0, 0, 0}, gls[4] = {0, 0, 0, 0}, grot[8] = {0, 0, 0, 0, 0, 0, 0, 0}, gop = 0;
  constexpr int RM = STATIC ? 3 : 4, RL = STATIC ? 3 : 4, RR = STATIC ? 4 : 8;
  T gsh[3 * K];
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) gsh[j] = T(0);
  const int nv = MULTI ? n_views : 1;
  for (int vi = 0; vi < nv; ++vi) {
    const double* g2v = grad2d + size_t(vi) * NC * size_t(n);
    T g2[NC];
    bool any = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      g2[c] = T(g2v[size_t(i) * NC + c]);
      any |= g2[c] != T(0);
    }
    if (!any) continue;
    T mu[4], ls[4], rot[8];
#pragma unroll
    for (int c = 0; c < RM; ++c) mu[c] = g.means[c * (long)n + i];
#pragma unroll
    for (int c = 0; c < RL; ++c) ls[c] = g.log_scales[c * (long)n + i];
#pragma unroll
    for (int c = 0; c < RR; ++c) rot[c] = g.rotors[c * (long)n + i];
    const ViewDev v = slots[vi].v;
    Fwd<T> f;
    auto fwd_bwd = [&](const T* shp, long stride) {
      if (STATIC) {
        gaussian_fwd_static<T>(mu, ls, rot, g.opacity[i], shp, stride, DEG, v, st, f);
        gaussian_bwd_static<T>(f, shp, stride, DEG, v, g2, gmu, gls, grot, gop, gsh, 1L);
      } else {
        gaussian_fwd<T>(mu, ls, rot, g.opacity[i], shp, stride, DEG, v, st, f);
        gaussian_bwd<T, T, FLOW>(f, shp, stride, DEG, v, g2, gmu, gls, grot, gop, gsh, 1L);
      }
    };
    if (MULTI) {
      fwd_bwd(g.sh + i, (long)n);
    } else {
      T shl[3 * K];
#pragma unroll
      for (int j = 0; j < 3 * K; ++j) shl[j] = g.sh[j * (long)n + i];
      fwd_bwd(shl, 1L);
    }
  }
#pragma unroll
  for (int c = 0; c < RM; ++c) out.means[c * (long)n + i] = gmu[c];
#pragma unroll
  for (int c = 0; c < RL; ++c) out.log_scales[c * (long)n + i] = gls[c];
#pragma unroll
  for (int c = 0; c < RR; ++c) out.rotors[c * (long)n + i] = grot[c];
  out.opacity[i] = gop;
#pragma unroll
  for (int j = 0; j < 3 * K; ++j) out.sh[j * (long)n + i] = gsh[j];
}

}  // namespace

#define R4D_DEG_DISPATCH(KERNEL, S, GRID, ...)                                           \
  switch (g.deg) {                                                                       \
    case 0: hipLaunchKernelGGL((KERNEL<T, 0, S>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 1: hipLaunchKernelGGL((KERNEL<T, 1, S>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2, S>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    case 3: hipLaunchKernelGGL((KERNEL<T, 3, S>), GRID, dim3(kBlock), 0, stream, __VA_ARGS__); break; \
    default: return hipErrorInvalidValue;                                                \
  }

template <typename T>
hipError_t launch_preprocess_fwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, uint32_t n_pad, Rec<T>* recs,
                                 Vec2<T>* flows, Rect16* rects, uint32_t* tiles_touched,
                                 uint32_t* depth_keys, unsigned long long* totals,
                                 uint32_t* vis_keys, uint32_t* vis_index, SegTable* dseg,
                                 void* temp, void* zero, size_t zero_bytes, bool static3d,
                                 hipStream_t stream) {
  if (g.n <= 0 || n_views <= 0) return hipSuccess;
  if ((zero_bytes & 15u) || (reinterpret_cast<uintptr_t>(zero) & 15u))
    return hipErrorInvalidValue;
  const uint32_t blocks = uint32_t((g.n + kBlock - 1) / kBlock);
  const dim3 grid(blocks, uint32_t(n_views));
  const dim3 grid_fwd(blocks * uint32_t(n_views));  // (render fastest)
  ulonglong2* block_totals = static_cast<ulonglong2*>(temp);
  uint4* z = static_cast<uint4*>(zero);
  const uint64_t z16 = zero_bytes / 16;
  if (static3d) {
    if (flows) return hipErrorInvalidValue;  // static Gaussians do not move
    R4D_DEG_DISPATCH(preprocess_fwd_kernel, true, grid_fwd, g, slots, st, n_pad, recs, flows,
                     rects, tiles_touched, depth_keys, block_totals, z, z16, uint32_t(n_views))
  } else {
    R4D_DEG_DISPATCH(preprocess_fwd_kernel, false, grid_fwd, g, slots, st, n_pad, recs, flows,
                     rects, tiles_touched, depth_keys, block_totals, z, z16, uint32_t(n_views))
  }
  hipLaunchKernelGGL(compact_keys_kernel, grid, dim3(kBlock), 0, stream, depth_keys, uint32_t(g.n),
                     n_pad, block_totals, totals, dseg, vis_keys, vis_index);
  return hipGetLastError();
}

size_t preprocess_temp_bytes(uint32_t n, int n_views) {
  const size_t blocks = size_t((n + kBlock - 1) / kBlock) * size_t(n_views);
  return blocks * sizeof(ulonglong2);
}

template <typename T>
hipError_t launch_preprocess_bwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, const double* grad2d, bool flow,
                                 bool static3d, const GradPtrs<T>& out, hipStream_t stream) {
  if (g.n <= 0) return hipSuccess;
  if (flow && static3d) return hipErrorInvalidValue;
  const dim3 grid((g.n + kBlock - 1) / kBlock);
#define R4D_BWD_DISPATCH(MULTI, FLOW, S)                                                     \
  switch (g.deg) {                                                                           \
    case 0: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 0, MULTI, FLOW, S>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 1: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 1, MULTI, FLOW, S>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 2: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 2, MULTI, FLOW, S>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    case 3: hipLaunchKernelGGL((preprocess_bwd_kernel<T, 3, MULTI, FLOW, S>), grid, dim3(kBlock), 0, stream, g, slots, n_views, st, grad2d, out); break; \
    default: return hipErrorInvalidValue;                                                    \
  }
  if (static3d) {
    if (n_views > 1) {
      R4D_BWD_DISPATCH(true, false, true)
    } else {
      R4D_BWD_DISPATCH(false, false, true)
    }
  } else if (flow) {
    if (n_views > 1) {
      R4D_BWD_DISPATCH(true, true, false)
    } else {
      R4D_BWD_DISPATCH(false, true, false)
    }
  } else if (n_views > 1) {
    R4D_BWD_DISPATCH(true, false, false)
  } else {
    R4D_BWD_DISPATCH(false, false, false)
  }
#undef R4D_BWD_DISPATCH
  return hipGetLastError();
}

#undef R4D_DEG_DISPATCH

#define R4D_INST(T)                                                                           \
  template hipError_t launch_preprocess_fwd<T>(const GaussPtrs<T>&, const ViewSlot*, int,      \
                                               const SettingsDev&, uint32_t, Rec<T>*, Vec2<T>*, \
                                               Rect16*, uint32_t*, uint32_t*,                  \
                                               unsigned long long*, uint32_t*, uint32_t*,      \
                                               SegTable*, void*, void*, size_t, bool,          \
                                               hipStream_t);                                   \
  template hipError_t launch_preprocess_bwd<T>(const GaussPtrs<T>&, const ViewSlot*, int,      \
                                               const SettingsDev&, const double*, bool, bool,  \
                                               const GradPtrs<T>&, hipStream_t);
R4D_INST(float)
R4D_INST(double)
#undef R4D_INST

}  // namespace r4d
