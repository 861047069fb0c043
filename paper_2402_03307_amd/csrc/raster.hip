// Tile rasteriser: front-to-back alpha compositing (paper Sec. 3.1, blending
// equation) and its reverse-mode derivative.
//
// One workgroup per tile, one pixel per lane.  The tile's list of Gaussian
// indices (sorted by depth) is walked in batches: every lane loads one projected
// record into LDS, then every lane reads the whole batch back (a broadcast read)
// and updates its pixel.  A workgroup stops as soon as every pixel of the tile
// has reached the transmittance floor.
//
// Per (pixel, Gaussian): d = mean2d - (x + .5, y + .5), q = d^T conic d; skip if
// q > extent^2; a = min(alpha_max, o exp(-q/2)); skip if a < alpha_min; stop if
// T (1 - a) < T_min; else C += rgb a T, T *= 1 - a.  Background added with the
// final T.  The forward stores, per pixel, the final T and the number of list
// entries up to the last blended one; the backward walks the list back to front
// from there, recovering T by division by (1 - a).
#include <hip/hip_runtime.h>

#include "r4d_internal.hpp"

namespace r4d {

namespace {

template <typename T> __device__ __forceinline__ T tfma(T a, T b, T c);
template <> __device__ __forceinline__ float tfma<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double tfma<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// exp(-q/2)
template <typename T> __device__ __forceinline__ T gauss_falloff(T q);
template <> __device__ __forceinline__ float gauss_falloff<float>(float q) {
  return __expf(-0.5f * q);
}
template <> __device__ __forceinline__ double gauss_falloff<double>(double q) {
  return exp(-0.5 * q);
}

// The one place where a (pixel, Gaussian) pair is evaluated; forward and backward
// call it with identical operands so that they take identical decisions.
template <typename T>
__device__ __forceinline__ bool eval_pair(const Rec<T>& r, T px, T py, T ext2, T amin, T amax,
                                          T& dx, T& dy, T& a_raw, T& alpha) {
  dx = r.mx - px;
  dy = r.my - py;
  const T q = tfma(r.ca * dx, dx, tfma(T(2) * r.cb * dx, dy, r.cc * dy * dy));
  if (!(q <= ext2)) return false;
  a_raw = r.o * gauss_falloff(q);
  alpha = a_raw < amax ? a_raw : amax;
  return alpha >= amin;
}

template <int TS>
struct TileCfg {
  static constexpr int kThreads = TS * TS;
  static constexpr int kBatch = kThreads < 256 ? kThreads : 256;
};

template <typename T, int TS>
__global__ __launch_bounds__(TS* TS) void raster_fwd_kernel(
    const Rec<T>* __restrict__ recs, const uint32_t* __restrict__ values,
    const uint2* __restrict__ ranges, ViewDev v, SettingsDev st, T* __restrict__ image,
    T* __restrict__ T_final, uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_eval) {
  constexpr int NT = TileCfg<TS>::kThreads;
  constexpr int NB = TileCfg<TS>::kBatch;
  __shared__ Rec<T> s_rec[NB];
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int x = tx * TS + int(threadIdx.x % TS);
  const int y = ty * TS + int(threadIdx.x / TS);
  const bool inside = x < v.W && y < v.H;
  const T px = T(x) + T(0.5), py = T(y) + T(0.5);
  const T ext2 = T(st.ext2), amin = T(st.alpha_min), amax = T(st.alpha_max), tmin = T(st.T_min);
  const uint2 rg = ranges[tile];
  T Tr = T(1), c0 = T(0), c1 = T(0), c2 = T(0);
  uint32_t last = 0, evals = 0;
  bool done = !inside;
  for (uint32_t base = rg.x; base < rg.y; base += NB) {
    if (__syncthreads_count(done) == NT) break;
    const uint32_t i = base + threadIdx.x;
    if (threadIdx.x < NB && i < rg.y) s_rec[threadIdx.x] = recs[values[i]];
    __syncthreads();
    if (!done) {
      const int nb = int(rg.y - base < uint32_t(NB) ? rg.y - base : uint32_t(NB));
      int j = 0;
      for (; j < nb; ++j) {
        const Rec<T> r = s_rec[j];
        T dx, dy, a_raw, alpha;
        if (!eval_pair(r, px, py, ext2, amin, amax, dx, dy, a_raw, alpha)) continue;
        const T Tn = Tr * (T(1) - alpha);
        if (Tn < tmin) {
          done = true;
          break;
        }
        const T w = alpha * Tr;
        c0 = tfma(r.r, w, c0);
        c1 = tfma(r.g, w, c1);
        c2 = tfma(r.b, w, c2);
        Tr = Tn;
        last = base - rg.x + uint32_t(j) + 1u;
      }
      evals += uint32_t(j < nb ? j + 1 : nb);
    }
  }
  if (inside) {
    const long hw = long(v.H) * v.W;
    const long pix = long(y) * v.W + x;
    image[pix] = tfma(Tr, T(v.bg[0]), c0);
    image[hw + pix] = tfma(Tr, T(v.bg[1]), c1);
    image[2 * hw + pix] = tfma(Tr, T(v.bg[2]), c2);
    T_final[pix] = Tr;
    n_contrib[pix] = last;
    if (n_eval) n_eval[pix] = evals;
  }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename T> __device__ __forceinline__ void atomic_add_nr(T* p, T v);
template <> __device__ __forceinline__ void atomic_add_nr<float>(float* p, float v) {
  __builtin_amdgcn_global_atomic_fadd_f32(p, v);
}
template <> __device__ __forceinline__ void atomic_add_nr<double>(double* p, double v) {
  atomicAdd(p, v);
}

template <typename T, int TS>
__global__ __launch_bounds__(TS* TS) void raster_bwd_kernel(
    const Rec<T>* __restrict__ recs, const uint32_t* __restrict__ values,
    const uint2* __restrict__ ranges, ViewDev v, SettingsDev st, const T* __restrict__ T_final,
    const uint32_t* __restrict__ n_contrib, const T* __restrict__ dL_dimage,
    T* __restrict__ grad2d, uint32_t n_gauss) {
  constexpr int NT = TileCfg<TS>::kThreads;
  constexpr int NB = TileCfg<TS>::kBatch;
  __shared__ Rec<T> s_rec[NB];
  __shared__ uint32_t s_idx[NB];
  __shared__ T s_grad[9][NB];
  __shared__ uint32_t s_max;
  const int tile = blockIdx.x;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int x = tx * TS + int(threadIdx.x % TS);
  const int y = ty * TS + int(threadIdx.x / TS);
  const bool inside = x < v.W && y < v.H;
  const T px = T(x) + T(0.5), py = T(y) + T(0.5);
  const T ext2 = T(st.ext2), amin = T(st.alpha_min), amax = T(st.alpha_max);
  const uint2 rg = ranges[tile];
  const long hw = long(v.H) * v.W;
  const long pix = long(y) * v.W + x;
  T Tcur = T(1), g0 = T(0), g1 = T(0), g2 = T(0);
  uint32_t ncon = 0;
  if (inside) {
    Tcur = T_final[pix];
    ncon = n_contrib[pix];
    g0 = dL_dimage[pix];
    g1 = dL_dimage[hw + pix];
    g2 = dL_dimage[2 * hw + pix];
  }
  // colour accumulated behind the current Gaussian (absolute, includes background)
  T acc0 = Tcur * T(v.bg[0]), acc1 = Tcur * T(v.bg[1]), acc2 = Tcur * T(v.bg[2]);
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  if (ncon) atomicMax(&s_max, ncon);
  __syncthreads();
  const uint32_t maxn = s_max;
  const int lane = threadIdx.x & 63;
  for (uint32_t bend = maxn; bend > 0;) {
    const uint32_t bstart = bend > uint32_t(NB) ? bend - NB : 0u;
    const int nb = int(bend - bstart);
    if (threadIdx.x < NB) {
      if (int(threadIdx.x) < nb) {
        const uint32_t idx = values[rg.x + bstart + threadIdx.x];
        s_idx[threadIdx.x] = idx;
        s_rec[threadIdx.x] = recs[idx];
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) s_grad[c][threadIdx.x] = T(0);
    }
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const Rec<T> r = s_rec[j];
      T dx = 0, dy = 0, a_raw = 0, alpha = 0;
      bool use = inside && (bstart + uint32_t(j) < ncon) &&
                 eval_pair(r, px, py, ext2, amin, amax, dx, dy, a_raw, alpha);
      T gm_x = 0, gm_y = 0, gca = 0, gcb = 0, gcc = 0, go = 0, gr = 0, gg = 0, gb = 0;
      if (use) {
        const T om = T(1) - alpha;
        const T Ti = Tcur / om;
        const T w = alpha * Ti;
        gr = w * g0;
        gg = w * g1;
        gb = w * g2;
        const T inv_om = T(1) / om;
        const T dL_da = g0 * (Ti * r.r - acc0 * inv_om) + g1 * (Ti * r.g - acc1 * inv_om) +
                        g2 * (Ti * r.b - acc2 * inv_om);
        acc0 = tfma(r.r, w, acc0);
        acc1 = tfma(r.g, w, acc1);
        acc2 = tfma(r.b, w, acc2);
        Tcur = Ti;
        if (a_raw < amax) {
          // a = o exp(-q/2): da/do = exp(-q/2), da/dq = -a/2
          go = dL_da * (a_raw / r.o);
          const T gq = T(-0.5) * dL_da * a_raw;
          gca = gq * dx * dx;
          gcb = gq * T(2) * dx * dy;
          gcc = gq * dy * dy;
          gm_x = gq * T(2) * (r.ca * dx + r.cb * dy);
          gm_y = gq * T(2) * (r.cb * dx + r.cc * dy);
        }
      }
      if (__ballot(use)) {
        gm_x = wave_sum(gm_x);
        gm_y = wave_sum(gm_y);
        gca = wave_sum(gca);
        gcb = wave_sum(gcb);
        gcc = wave_sum(gcc);
        go = wave_sum(go);
        gr = wave_sum(gr);
        gg = wave_sum(gg);
        gb = wave_sum(gb);
        if (lane == 0) {
          if (NT == 64) {
            s_grad[0][j] += gm_x;
            s_grad[1][j] += gm_y;
            s_grad[2][j] += gca;
            s_grad[3][j] += gcb;
            s_grad[4][j] += gcc;
            s_grad[5][j] += go;
            s_grad[6][j] += gr;
            s_grad[7][j] += gg;
            s_grad[8][j] += gb;
          } else {
            atomicAdd(&s_grad[0][j], gm_x);
            atomicAdd(&s_grad[1][j], gm_y);
            atomicAdd(&s_grad[2][j], gca);
            atomicAdd(&s_grad[3][j], gcb);
            atomicAdd(&s_grad[4][j], gcc);
            atomicAdd(&s_grad[5][j], go);
            atomicAdd(&s_grad[6][j], gr);
            atomicAdd(&s_grad[7][j], gg);
            atomicAdd(&s_grad[8][j], gb);
          }
        }
      }
    }
    __syncthreads();
    // one global atomic per (tile, Gaussian, component)
    for (int e = threadIdx.x; e < 9 * nb; e += NT) {
      const int c = e / nb, j = e % nb;
      const T val = s_grad[c][j];
      if (val != T(0)) atomic_add_nr(&grad2d[long(c) * n_gauss + s_idx[j]], val);
    }
    __syncthreads();
    bend = bstart;
  }
}

__global__ __launch_bounds__(256) void l1_grad_kernel(const float* __restrict__ image,
                                                      const float* __restrict__ target,
                                                      int64_t count, float inv_count,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ loss) {
  __shared__ float s_part[4];
  const int64_t stride = int64_t(gridDim.x) * 256;
  float part = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += stride) {
    const float d = image[i] - target[i];
    grad[i] = d > 0.f ? inv_count : (d < 0.f ? -inv_count : 0.f);
    part += fabsf(d);
  }
  if (loss) {
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0)
      atomic_add_nr(loss, (s_part[0] + s_part[1] + s_part[2] + s_part[3]) * inv_count);
  }
}

template <typename T, int TS>
hipError_t raster_fwd_ts(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                         const ViewDev& v, const SettingsDev& st, T* image, T* T_final,
                         uint32_t* n_contrib, uint32_t* n_eval, hipStream_t stream) {
  const int tiles = v.tiles_x * v.tiles_y;
  hipLaunchKernelGGL((raster_fwd_kernel<T, TS>), dim3(tiles), dim3(TS * TS), 0, stream, recs,
                     values, ranges, v, st, image, T_final, n_contrib, n_eval);
  return hipGetLastError();
}

template <typename T, int TS>
hipError_t raster_bwd_ts(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                         const ViewDev& v, const SettingsDev& st, const T* T_final,
                         const uint32_t* n_contrib, const T* dL_dimage, T* grad2d,
                         uint32_t n_gaussians, hipStream_t stream) {
  const int tiles = v.tiles_x * v.tiles_y;
  hipLaunchKernelGGL((raster_bwd_kernel<T, TS>), dim3(tiles), dim3(TS * TS), 0, stream, recs,
                     values, ranges, v, st, T_final, n_contrib, dL_dimage, grad2d, n_gaussians);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_raster_fwd(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                             const ViewDev& v, const SettingsDev& st, T* image, T* T_final,
                             uint32_t* n_contrib, uint32_t* n_eval, hipStream_t stream) {
  switch (v.tile_size) {
    case 8:
      return raster_fwd_ts<T, 8>(recs, values, ranges, v, st, image, T_final, n_contrib, n_eval,
                                 stream);
    case 16:
      return raster_fwd_ts<T, 16>(recs, values, ranges, v, st, image, T_final, n_contrib, n_eval,
                                  stream);
    case 32:
      return raster_fwd_ts<T, 32>(recs, values, ranges, v, st, image, T_final, n_contrib, n_eval,
                                  stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_raster_bwd(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                             const ViewDev& v, const SettingsDev& st, const T* T_final,
                             const uint32_t* n_contrib, const T* dL_dimage, T* grad2d,
                             uint32_t n_gaussians, hipStream_t stream) {
  switch (v.tile_size) {
    case 8:
      return raster_bwd_ts<T, 8>(recs, values, ranges, v, st, T_final, n_contrib, dL_dimage,
                                 grad2d, n_gaussians, stream);
    case 16:
      return raster_bwd_ts<T, 16>(recs, values, ranges, v, st, T_final, n_contrib, dL_dimage,
                                  grad2d, n_gaussians, stream);
    case 32:
      return raster_bwd_ts<T, 32>(recs, values, ranges, v, st, T_final, n_contrib, dL_dimage,
                                  grad2d, n_gaussians, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, float* grad,
                          float* loss, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (loss) {
    hipError_t e = hipMemsetAsync(loss, 0, sizeof(float), stream);
    if (e != hipSuccess) return e;
  }
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(l1_grad_kernel, dim3(blocks), dim3(256), 0, stream, image, target, count,
                     1.0f / float(count), grad, loss);
  return hipGetLastError();
}

template hipError_t launch_raster_fwd<float>(const Rec<float>*, const uint32_t*, const uint2*,
                                             const ViewDev&, const SettingsDev&, float*, float*,
                                             uint32_t*, uint32_t*, hipStream_t);
template hipError_t launch_raster_fwd<double>(const Rec<double>*, const uint32_t*, const uint2*,
                                              const ViewDev&, const SettingsDev&, double*,
                                              double*, uint32_t*, uint32_t*, hipStream_t);
template hipError_t launch_raster_bwd<float>(const Rec<float>*, const uint32_t*, const uint2*,
                                             const ViewDev&, const SettingsDev&, const float*,
                                             const uint32_t*, const float*, float*, uint32_t,
                                             hipStream_t);
template hipError_t launch_raster_bwd<double>(const Rec<double>*, const uint32_t*, const uint2*,
                                              const ViewDev&, const SettingsDev&, const double*,
                                              const uint32_t*, const double*, double*, uint32_t,
                                              hipStream_t);

}  // namespace r4d
