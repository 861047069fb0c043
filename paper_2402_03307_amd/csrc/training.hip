// The optimisation step around the render: the entropy loss on the opacities
// (Sec. 3.3 "Entropy Loss"), one fused Adam update of every parameter group,
// and the opacity reset.  The paper follows 3D Gaussian Splatting for the
// optimiser (Sec. 4, "Implementation Details"): per-group learning rates, the
// position rate decayed exponentially, the opacity optimised as a logit.
//
// Adam is elementwise and HBM-bound (28 bytes per element in float32: the
// parameter, gradient and two moments read, the parameter and moments
// written); one launch covers all five groups, each thread walking the
// concatenated element range, so no group needs a launch of its own.
#include <hip/hip_runtime.h>

#include <math.h>

#include "r4d_internal.hpp"

namespace r4d {

namespace {

constexpr int kBlock = 256;

// One element's update (shared by the scalar and the 4-wide kernels).
__device__ __forceinline__ void adam_one(float& p, float g, float& mo, float& vo, float& l,
                                         bool is_logit, float lr, float bc1, float bc2,
                                         const AdamConfig& c) {
  if (is_logit) {  // opacity: the update acts on the logit
    const float o = 1.0f / (1.0f + expf(-l));
    g *= o * (1.0f - o);
  }
  const float mm = c.beta1 * mo + (1.0f - c.beta1) * g;
  const float vv = c.beta2 * vo + (1.0f - c.beta2) * g * g;
  mo = mm;
  vo = vv;
  const float upd = lr * (mm / bc1) / (sqrtf(vv / bc2) + c.eps);
  if (is_logit) {
    l -= upd;
    p = 1.0f / (1.0f + expf(-l));
  } else {
    p -= upd;
  }
}

// VEC = 4: four consecutive elements per thread with 16-byte accesses (valid
// when n is a multiple of 4 and every array is 16-byte aligned, so that the
// four fall in one group and one row); VEC = 1 otherwise.
template <int VEC>
__global__ __launch_bounds__(kBlock) void adam_kernel(AdamGroups G, float* __restrict__ logit,
                                                      float* __restrict__ m,
                                                      float* __restrict__ v,
                                                      const int32_t* __restrict__ step,
                                                      AdamConfig c) {
  const int32_t t0 = *step;  // steps already taken
  const float t = float(t0) + 1.0f;
  const float bc1 = 1.0f - powf(c.beta1, t);
  const float bc2 = 1.0f - powf(c.beta2, t);
  float u = c.lr_means_steps > 0 ? float(t0) / float(c.lr_means_steps) : 1.0f;
  u = u < 1.0f ? u : 1.0f;
  const float lr_means = expf((1.0f - u) * logf(c.lr_means_init) + u * logf(c.lr_means_final));
  const float lrs[4] = {lr_means, c.lr_log_scales, c.lr_rotors, c.lr_opacity};
  const uint64_t total = G.off[5] / VEC;
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += stride) {
    const uint64_t e = i * VEC;
    int k = 0;
#pragma unroll
    for (int q = 1; q < 5; ++q) k += e >= G.off[q] ? 1 : 0;
    const uint64_t local = e - G.off[k];
    // rows 0..2 of the SH array: degree 0
    const float lr = k == 4 ? (local < 3ull * G.n ? c.lr_sh_dc : c.lr_sh_rest) : lrs[k];
    const bool is_logit = k == 3;
    if (VEC == 4) {
      float4 p = *reinterpret_cast<const float4*>(G.p[k] + local);
      const float4 g = *reinterpret_cast<const float4*>(G.g[k] + local);
      float4 mo = *reinterpret_cast<const float4*>(m + e);
      float4 vo = *reinterpret_cast<const float4*>(v + e);
      float4 l = is_logit ? *reinterpret_cast<const float4*>(logit + local)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
      adam_one(p.x, g.x, mo.x, vo.x, l.x, is_logit, lr, bc1, bc2, c);
      adam_one(p.y, g.y, mo.y, vo.y, l.y, is_logit, lr, bc1, bc2, c);
      adam_one(p.z, g.z, mo.z, vo.z, l.z, is_logit, lr, bc1, bc2, c);
      adam_one(p.w, g.w, mo.w, vo.w, l.w, is_logit, lr, bc1, bc2, c);
      *reinterpret_cast<float4*>(G.p[k] + local) = p;
      *reinterpret_cast<float4*>(m + e) = mo;
      *reinterpret_cast<float4*>(v + e) = vo;
      if (is_logit) *reinterpret_cast<float4*>(logit + local) = l;
    } else {
      float p = G.p[k][local], mo = m[e], vo = v[e];
      float l = is_logit ? logit[local] : 0.f;
      adam_one(p, G.g[k][local], mo, vo, l, is_logit, lr, bc1, bc2, c);
      G.p[k][local] = p;
      m[e] = mo;
      v[e] = vo;
      if (is_logit) logit[local] = l;
    }
  }
}

__global__ void step_increment_kernel(int32_t* __restrict__ step) { *step += 1; }

// o <- min(o, cap) through the logit; the opacity moments [off, off + n) cleared.
__global__ __launch_bounds__(kBlock) void opacity_reset_kernel(uint32_t n, float cap,
                                                               float cap_logit,
                                                               float* __restrict__ logit,
                                                               float* __restrict__ opacity,
                                                               float* __restrict__ m_op,
                                                               float* __restrict__ v_op) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float l = logit[i];
  const float o = 1.0f / (1.0f + expf(-l));
  if (o > cap) {
    logit[i] = cap_logit;
    opacity[i] = cap;
  }
  m_op[i] = 0.f;
  v_op[i] = 0.f;
}

// Optimiser state of a fresh parameter set: the opacity logit
// ln(o / (1 - o)) of the activated opacity (o clamped to [1e-7, 1 - 1e-7], in
// float64), both Adam moments zero over every element, the step count zero.
__global__ __launch_bounds__(kBlock) void state_init_kernel(uint32_t n, uint64_t total,
                                                            const float* __restrict__ opacity,
                                                            float* __restrict__ logit,
                                                            float* __restrict__ m,
                                                            float* __restrict__ v,
                                                            int32_t* __restrict__ step) {
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < total; i += stride) {
    m[i] = 0.f;
    v[i] = 0.f;
    if (i < n) {
      const double o = fmin(fmax(double(opacity[i]), 1e-7), 1.0 - 1e-7);
      logit[i] = float(log(o) - log1p(-o));
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *step = 0;
}

// Per workgroup: sum of -o ln o into partials; grad += weight * d/do of the
// mean, -(ln o + 1) / n.
__global__ __launch_bounds__(kBlock) void entropy_kernel(const float* __restrict__ opacity,
                                                         uint32_t n, float gscale,
                                                         float* __restrict__ grad,
                                                         float* __restrict__ partials) {
  __shared__ float s_part[kBlock / 64];
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  float part = 0.f;
  if (i < n) {
    const float o = opacity[i];
    const float lo = logf(o);
    part = -o * lo;
    if (grad) grad[i] += gscale * (-(lo + 1.0f));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

__global__ __launch_bounds__(kBlock) void mean_of_partials_kernel(const float* __restrict__ partials,
                                                                  uint32_t count, uint32_t n,
                                                                  float* __restrict__ loss) {
  __shared__ float s_part[kBlock / 64];
  float part = 0.f;
  for (uint32_t b = threadIdx.x; b < count; b += kBlock) part += partials[b];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) *loss = ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) / float(n);
}

}  // namespace

hipError_t launch_adam(const AdamGroups& groups, float* logit, float* m, float* v, int32_t* step,
                       const AdamConfig& cfg, hipStream_t stream) {
  const uint64_t total = groups.off[5];
  if (total == 0) return hipSuccess;
  auto aligned = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  bool vec = groups.n % 4 == 0 && aligned(logit) && aligned(m) && aligned(v);
  for (int q = 0; q < 5; ++q) vec = vec && aligned(groups.p[q]) && aligned(groups.g[q]);
  uint64_t blocks = (total / (vec ? 4 : 1) + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;  // grid-stride beyond: 2M threads cover HBM latency
  if (vec)
    hipLaunchKernelGGL(adam_kernel<4>, dim3(uint32_t(blocks)), dim3(kBlock), 0, stream, groups,
                       logit, m, v, step, cfg);
  else
    hipLaunchKernelGGL(adam_kernel<1>, dim3(uint32_t(blocks)), dim3(kBlock), 0, stream, groups,
                       logit, m, v, step, cfg);
  hipLaunchKernelGGL(step_increment_kernel, dim3(1), dim3(1), 0, stream, step);
  return hipGetLastError();
}

hipError_t launch_opacity_reset(uint32_t n, float cap, float* logit, float* opacity, float* m_op,
                                float* v_op, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const float cap_logit = float(log(double(cap)) - log1p(-double(cap)));
  hipLaunchKernelGGL(opacity_reset_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     stream, n, cap, cap_logit, logit, opacity, m_op, v_op);
  return hipGetLastError();
}

hipError_t launch_state_init(uint32_t n, uint64_t total, const float* opacity, float* logit,
                             float* m, float* v, int32_t* step, hipStream_t stream) {
  uint64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(state_init_kernel, dim3(uint32_t(blocks)), dim3(kBlock), 0, stream, n, total,
                     opacity, logit, m, v, step);
  return hipGetLastError();
}

size_t entropy_temp_bytes(uint32_t n) { return ((size_t(n) + kBlock - 1) / kBlock) * 4 + 256; }

hipError_t launch_entropy(const float* opacity, uint32_t n, float weight, float* loss, float* grad,
                          void* temp, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t blocks = (n + kBlock - 1) / kBlock;
  float* partials = static_cast<float*>(temp);
  hipLaunchKernelGGL(entropy_kernel, dim3(blocks), dim3(kBlock), 0, stream, opacity, n,
                     weight / float(n), grad, partials);
  if (loss)
    hipLaunchKernelGGL(mean_of_partials_kernel, dim3(1), dim3(kBlock), 0, stream, partials, blocks,
                       n, loss);
  return hipGetLastError();
}

}  // namespace r4d

// ---- density control (3D Gaussian Splatting's, applied to 4D Gaussians)

namespace r4d {

namespace {

// Per Gaussian, over the renders where it is listed in some tile: the norm of
// the projected-mean gradient in normalised device coordinates (pixel
// gradient times (W/2, H/2)) added to accum, and the count of such renders.
__global__ __launch_bounds__(kBlock) void densify_stats_kernel(
    const double* __restrict__ grad2d, int nc, const uint32_t* __restrict__ dkeys, uint32_t n_pad,
    const ViewSlot* __restrict__ slots, int n_views, uint32_t n, float* __restrict__ accum,
    int32_t* __restrict__ count) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  int32_t c = 0;
  for (int v = 0; v < n_views; ++v) {
    if (dkeys[size_t(v) * n_pad + i] == 0xffffffffu) continue;
    const double* g = grad2d + size_t(v) * size_t(nc) * n;
    const double gx = g[size_t(i) * nc] * (0.5 * double(slots[v].v.W));
    const double gy = g[size_t(i) * nc + 1] * (0.5 * double(slots[v].v.H));
    a += sqrt(gx * gx + gy * gy);
    c += 1;
  }
  if (c) {
    accum[i] += float(a);
    count[i] += c;
  }
}

struct DensifyDev {
  float grad_threshold, size_log, min_opacity, big_log, shrink;
  int has_big;
};

__device__ __forceinline__ bool survives(float o, float max_log_scale, const DensifyDev& c) {
  return !(o < c.min_opacity) && !(c.has_big && max_log_scale > c.big_log);
}

// Per Gaussian: how many copies it keeps (0 / 1), clones (0 / 1) and children
// (0 / 2) contribute to the new set.
__global__ __launch_bounds__(kBlock) void densify_classify_kernel(
    const float* __restrict__ log_scales, const float* __restrict__ opacity,
    const float* __restrict__ accum, const int32_t* __restrict__ count, uint32_t n, DensifyDev c,
    uint32_t* __restrict__ n_keep, uint32_t* __restrict__ n_clone, uint32_t* __restrict__ n_child) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t cnt = count[i];
  const float avg = cnt > 0 ? accum[i] / float(cnt) : 0.f;
  const bool selected = cnt > 0 && avg >= c.grad_threshold;
  const float l0 = log_scales[i], l1 = log_scales[size_t(n) + i], l2 = log_scales[2 * size_t(n) + i];
  const float mls = fmaxf(fmaxf(l0, l1), l2);
  const bool small = mls <= c.size_log;
  const bool split = selected && !small;
  const float o = opacity[i];
  const bool ok = survives(o, mls, c);
  const float cm = fmaxf(fmaxf(l0 - c.shrink, l1 - c.shrink), l2 - c.shrink);
  n_keep[i] = (!split && ok) ? 1u : 0u;
  n_clone[i] = (selected && small && ok) ? 1u : 0u;
  n_child[i] = (split && survives(o, cm, c)) ? 2u : 0u;
}

struct DensifyIO {
  // parameter groups in / out (means, log_scales, rotors, opacity, sh)
  const float* pin[5];
  float* pout[5];
  uint32_t rows[5];
  const float* logit_in;
  float* logit_out;
  const float* m_in;
  const float* v_in;
  float* m_out;
  float* v_out;
  uint32_t n_in, n_out;
};

__global__ __launch_bounds__(kBlock) void densify_scatter_kernel(
    DensifyIO io, const uint32_t* __restrict__ off_keep, const uint32_t* __restrict__ off_clone,
    const uint32_t* __restrict__ off_child, uint32_t total_keep, uint32_t total_clone,
    const float* __restrict__ normals, DensifyDev c) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= io.n_in) return;
  const uint32_t nk = off_keep[i + 1] - off_keep[i];
  const uint32_t nc = off_clone[i + 1] - off_clone[i];
  const uint32_t nh = off_child[i + 1] - off_child[i];
  if (!(nk | nc | nh)) return;
  const size_t ni = io.n_in, no = io.n_out;
  // destinations: the kept copy (moments carried), the clone, the children
  const uint32_t dk = off_keep[i];
  const uint32_t dc = total_keep + off_clone[i];
  const uint32_t dh = total_keep + total_clone + off_child[i];
  size_t base_in = 0, base_out = 0;  // group's first element in the moment arrays
  for (int q = 0; q < 5; ++q) {
    for (uint32_t r = 0; r < io.rows[q]; ++r) {
      const float x = io.pin[q][r * ni + i];
      if (nk) {
        io.pout[q][r * no + dk] = x;
        io.m_out[base_out + r * no + dk] = io.m_in[base_in + r * ni + i];
        io.v_out[base_out + r * no + dk] = io.v_in[base_in + r * ni + i];
      }
      if (nc) {
        io.pout[q][r * no + dc] = x;
        io.m_out[base_out + r * no + dc] = 0.f;
        io.v_out[base_out + r * no + dc] = 0.f;
      }
      if (nh) {
        for (uint32_t h = 0; h < 2; ++h) {
          float y = x;
          if (q == 1) y = x - c.shrink;  // log-scales of a child
          io.pout[q][r * no + dh + h] = y;  // means are overwritten below
          io.m_out[base_out + r * no + dh + h] = 0.f;
          io.v_out[base_out + r * no + dh + h] = 0.f;
        }
      }
    }
    base_in += size_t(io.rows[q]) * ni;
    base_out += size_t(io.rows[q]) * no;
  }
  const float lg = io.logit_in[i];
  if (nk) io.logit_out[dk] = lg;
  if (nc) io.logit_out[dc] = lg;
  if (nh) {
    io.logit_out[dh] = lg;
    io.logit_out[dh + 1] = lg;
    // children at mu + R diag(s) z_h, R the normalised rotor's rotation and s
    // the parent's scales
    float ls[4], rot[8];
    for (int k = 0; k < 4; ++k) ls[k] = io.pin[1][k * ni + i];
    for (int k = 0; k < 8; ++k) rot[k] = io.pin[2][k * ni + i];
    Fwd<float> f;
    cov4_fwd(ls, rot, f);
    for (uint32_t h = 0; h < 2; ++h) {
      float sz[4];
      for (int k = 0; k < 4; ++k)
        sz[k] = expf(ls[k]) * normals[size_t(k) * 2 * ni + 2 * size_t(i) + h];
      for (int row = 0; row < 4; ++row) {
        float acc = io.pin[0][row * ni + i];
        for (int k = 0; k < 4; ++k) acc += f.R[4 * row + k] * sz[k];
        io.pout[0][row * no + dh + h] = acc;
      }
    }
  }
}

}  // namespace

hipError_t launch_densify_stats(const double* grad2d, int nc, const uint32_t* dkeys,
                                uint32_t n_pad, const ViewSlot* slots, int n_views, uint32_t n,
                                float* accum, int32_t* count, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(densify_stats_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     stream, grad2d, nc, dkeys, n_pad, slots, n_views, n, accum, count);
  return hipGetLastError();
}

size_t densify_temp_bytes(uint32_t n) {
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  return 6 * a((size_t(n) + 1) * 4) + 3 * a(scan_u32_temp_bytes(n)) + 256;
}

hipError_t densify_count(const DensifyArgs& d, void* temp, uint32_t* totals_host,
                         hipStream_t stream) {
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  const uint32_t n = d.n_in;
  uint8_t* p = static_cast<uint8_t*>(temp);
  uint32_t* cnt[3];
  uint32_t* off[3];
  void* scr[3];
  for (int q = 0; q < 3; ++q) {
    cnt[q] = reinterpret_cast<uint32_t*>(p);
    p += a((size_t(n) + 1) * 4);
    off[q] = reinterpret_cast<uint32_t*>(p);
    p += a((size_t(n) + 1) * 4);
    scr[q] = p;
    p += a(scan_u32_temp_bytes(n));
  }
  const DensifyDev c{d.grad_threshold, d.size_log, d.min_opacity, d.big_log, d.shrink, d.has_big};
  hipLaunchKernelGGL(densify_classify_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     stream, d.log_scales, d.opacity, d.accum, d.count, n, c, cnt[0], cnt[1],
                     cnt[2]);
  for (int q = 0; q < 3; ++q) {
    const hipError_t e = scan_u32(cnt[q], n, off[q], scr[q], stream);
    if (e != hipSuccess) return e;
  }
  for (int q = 0; q < 3; ++q) {
    const hipError_t e = hipMemcpyAsync(totals_host + q, off[q] + n, 4, hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t densify_scatter(const DensifyArgs& d, const void* temp, uint32_t total_keep,
                           uint32_t total_clone, uint32_t n_out, hipStream_t stream) {
  auto a = [](size_t b) { return (b + 255) & ~size_t(255); };
  const uint32_t n = d.n_in;
  const uint8_t* p = static_cast<const uint8_t*>(temp);
  const uint32_t* off[3];
  for (int q = 0; q < 3; ++q) {
    p += a((size_t(n) + 1) * 4);
    off[q] = reinterpret_cast<const uint32_t*>(p);
    p += a((size_t(n) + 1) * 4);
    p += a(scan_u32_temp_bytes(n));
  }
  DensifyIO io{};
  for (int q = 0; q < 5; ++q) {
    io.pin[q] = d.pin[q];
    io.pout[q] = d.pout[q];
    io.rows[q] = d.rows[q];
  }
  io.logit_in = d.logit_in;
  io.logit_out = d.logit_out;
  io.m_in = d.m_in;
  io.v_in = d.v_in;
  io.m_out = d.m_out;
  io.v_out = d.v_out;
  io.n_in = n;
  io.n_out = n_out;
  const DensifyDev c{d.grad_threshold, d.size_log, d.min_opacity, d.big_log, d.shrink, d.has_big};
  hipLaunchKernelGGL(densify_scatter_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     stream, io, off[0], off[1], off[2], total_keep, total_clone, d.normals, c);
  return hipGetLastError();
}

}  // namespace r4d
