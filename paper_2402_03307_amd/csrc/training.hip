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
  const uint64_t total = G.off[5];
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t e = uint64_t(blockIdx.x) * kBlock + threadIdx.x; e < total; e += stride) {
    int k = 0;
#pragma unroll
    for (int q = 1; q < 5; ++q) k += e >= G.off[q] ? 1 : 0;
    const uint64_t local = e - G.off[k];
    float g = G.g[k][local];
    float lr;
    if (k == 4) {
      lr = local < 3ull * G.n ? c.lr_sh_dc : c.lr_sh_rest;  // rows 0..2: degree 0
    } else {
      lr = lrs[k];
    }
    float l = 0.f;
    if (k == 3) {  // opacity: the update acts on the logit
      l = logit[local];
      const float o = 1.0f / (1.0f + expf(-l));
      g *= o * (1.0f - o);
    }
    const float mm = c.beta1 * m[e] + (1.0f - c.beta1) * g;
    const float vv = c.beta2 * v[e] + (1.0f - c.beta2) * g * g;
    m[e] = mm;
    v[e] = vv;
    const float upd = lr * (mm / bc1) / (sqrtf(vv / bc2) + c.eps);
    if (k == 3) {
      l -= upd;
      logit[local] = l;
      G.p[3][local] = 1.0f / (1.0f + expf(-l));
    } else {
      G.p[k][local] -= upd;
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
  uint64_t blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;  // grid-stride beyond: 2M threads cover HBM latency
  hipLaunchKernelGGL(adam_kernel, dim3(uint32_t(blocks)), dim3(kBlock), 0, stream, groups, logit,
                     m, v, step, cfg);
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
