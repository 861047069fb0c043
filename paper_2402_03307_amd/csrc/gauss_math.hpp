// Per-Gaussian math of the 4D-rotor render path, forward and backward.
//
// Written for T = float (the product path) and T = double (finite-difference
// checks).  Everything here is __host__ __device__ and allocation-free.
//
// Forward, per Gaussian and render (view, time t):
//   rotor normalisation (App. A "4D Rotor Normalization"): one step along the
//     gradient of eps = p s - b01 b23 + b02 b13 - b03 b12 with the root of
//     eps (1 + delta^2) + l^2 delta = 0 that vanishes with eps, evaluated as
//     delta = -2 eps / (l^2 + sqrt(l^4 - 4 eps^2)), then division by the norm;
//   rotor -> 4x4 rotation (App. A "4D Rotor to Rotation Matrix", 16 quadratic
//     forms);
//   Sigma_4 = R diag(s^2) R^T, s = exp(log s) (Sec. 3.2.1);
//   temporal slice (Sec. 3.2.2 Eq. center-motion, App. A Schur-complement form):
//     mu(t) = mu_xyz + (t - mu_t) V / W, Sigma_3D = U - V V^T / W,
//     opacity decay exp(-(t - mu_t)^2 / (2 W)), dropped when (t-mu_t)^2/W > tau;
//   view transform, near-plane drop, EWA projection Sigma_2D = J Wv Sigma Wv^T J^T
//     + dilation I (Sec. 3.1), conic = Sigma_2D^-1;
//   SH colour rgb = max(0, sum Y_lm(d) c_lm + 0.5), d the unit direction from the
//     camera centre to mu(t) (Sec. 3.1);
//   2D flow: the sliced mean moves with speed V / W (Sec. 3.2.2); its projection
//     is the time derivative of the pinhole mean, in pixels per unit of t.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define R4D_HD __host__ __device__ __forceinline__

namespace r4d {

// View constants as the kernels see them.
struct ViewDev {
  float M[9];       // world-to-camera rotation, row-major
  float tw[3];      // world-to-camera translation
  float cam[3];     // camera centre in world space = -M^T tw
  float fx, fy, cx, cy;
  float limx, limy; // guard-band limits on x/z and y/z
  float t;
  float bg[3];
  int32_t W, H;
  int32_t tiles_x, tiles_y, tile_size;
};

struct SettingsDev {
  float near_plane, time_cull, ext2, alpha_min, alpha_max, T_min, dilation;
  float log_alpha_min;   // ln(alpha_min)
};

// Per-Gaussian projected record, 12 scalars: (mx, my, ca, cb), (cc, o, depth, qmax),
// (r, g, b, 0).  q(d) = ca dx^2 + 2 cb dx dy + cc dy^2 with d = mean2d - pixel;
// qmax = min(extent^2, 2 ln(o / alpha_min)) rounded up to T, the largest q at
// which the Gaussian can still be blended (the bound the tile lists follow).
template <typename T>
struct alignas(sizeof(T) * 4) Rec {
  T mx, my, ca, cb;
  T cc, o, depth, qmax;
  T r, g, b, pad1;
};

// A pair of scalars stored together (a Gaussian's 2D flow, a pixel's flow state).
template <typename T>
struct alignas(sizeof(T) * 2) Vec2 {
  T x, y;
};

template <typename T> R4D_HD T r4d_sqrt(T x);
template <> R4D_HD float r4d_sqrt<float>(float x) { return sqrtf(x); }
template <> R4D_HD double r4d_sqrt<double>(double x) { return sqrt(x); }
template <typename T> R4D_HD T r4d_exp(T x);
template <> R4D_HD float r4d_exp<float>(float x) { return expf(x); }
template <> R4D_HD double r4d_exp<double>(double x) { return exp(x); }
template <typename T> R4D_HD T r4d_log(T x);
template <> R4D_HD float r4d_log<float>(float x) { return logf(x); }
template <> R4D_HD double r4d_log<double>(double x) { return log(x); }

template <typename T> R4D_HD T tmax(T a, T b) { return a > b ? a : b; }
template <typename T> R4D_HD T tmin(T a, T b) { return a < b ? a : b; }

// Intermediates of the per-Gaussian forward that the backward reuses.
template <typename T>
struct Fwd {
  // rotor normalisation
  T r[8], g[8];
  T eps, l2, sq, den, delta;
  T r1[8], inv_n1, rn[8];
  bool degenerate;
  // rotation, covariance
  T R[16];
  T s2[4];
  T U[6];            // xx, xy, xz, yy, yz, zz
  T V[3], W;
  // slice
  T dt, invW, lam_dt2, decay;
  T vel[3], mu3[3], S3[6];
  T o_t;
  // projection
  T p[3];
  T ipz, txz, tyz;   // 1/z, clamped x/z, clamped y/z
  bool clx, cly;
  T Tm[6];           // J Wv, row-major 2x3
  T A, B, C;         // Sigma_2D entries (with dilation)
  T det;
  T conic[3];
  T mean2[2];
  // colour
  T dir[3], inv_nd, d[3];
  T raw[3], rgb[3];
  // camera-space speed of the sliced mean and its projection
  T vc[3], flow[2];
  bool valid;
};

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3, l-major, m = -l..l, in the sign
// convention of the 3DGS renderer lineage.  Normalisation constants:
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the usual associated-Legendre
// polynomial factors, folded into one number per function.
namespace sh {
constexpr double Y00 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double K1 = 0.4886025119029199;     // sqrt(3/(4 pi))
constexpr double K2a = 1.0925484305920792;    // sqrt(15/(4 pi))
constexpr double K2b = 0.31539156525252005;   // sqrt(5/(16 pi))
constexpr double K2c = 0.5462742152960396;    // sqrt(15/(16 pi))
constexpr double K3a = 0.5900435899266435;    // sqrt(35/(32 pi))
constexpr double K3b = 2.890611442640554;     // sqrt(105/(4 pi))
constexpr double K3c = 0.4570457994644658;    // sqrt(21/(32 pi))
constexpr double K3d = 0.3731763325901154;    // sqrt(7/(16 pi))
constexpr double K3e = 1.445305721320277;     // sqrt(105/(16 pi))
}  // namespace sh

template <typename T>
R4D_HD void sh_eval(int deg, T x, T y, T z, T* Y) {
  Y[0] = T(sh::Y00);
  if (deg < 1) return;
  Y[1] = -T(sh::K1) * y;
  Y[2] = T(sh::K1) * z;
  Y[3] = -T(sh::K1) * x;
  if (deg < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[4] = T(sh::K2a) * x * y;
  Y[5] = -T(sh::K2a) * y * z;
  Y[6] = T(sh::K2b) * (2 * zz - xx - yy);
  Y[7] = -T(sh::K2a) * x * z;
  Y[8] = T(sh::K2c) * (xx - yy);
  if (deg < 3) return;
  Y[9] = -T(sh::K3a) * y * (3 * xx - yy);
  Y[10] = T(sh::K3b) * x * y * z;
  Y[11] = -T(sh::K3c) * y * (4 * zz - xx - yy);
  Y[12] = T(sh::K3d) * z * (2 * zz - 3 * xx - 3 * yy);
  Y[13] = -T(sh::K3c) * x * (4 * zz - xx - yy);
  Y[14] = T(sh::K3e) * z * (xx - yy);
  Y[15] = -T(sh::K3a) * x * (xx - 3 * yy);
}

// Given gY[k] = dL/dY_k, accumulate dL/d(x, y, z) of the polynomial basis.
template <typename T>
R4D_HD void sh_grad(int deg, T x, T y, T z, const T* gY, T& gx, T& gy, T& gz) {
  gx = gy = gz = T(0);
  if (deg < 1) return;
  gy += -T(sh::K1) * gY[1];
  gz += T(sh::K1) * gY[2];
  gx += -T(sh::K1) * gY[3];
  if (deg < 2) return;
  const T xx = x * x, yy = y * y, zz = z * z;
  // Y4 = a xy
  gx += T(sh::K2a) * y * gY[4];
  gy += T(sh::K2a) * x * gY[4];
  // Y5 = -a yz
  gy += -T(sh::K2a) * z * gY[5];
  gz += -T(sh::K2a) * y * gY[5];
  // Y6 = b (2zz - xx - yy)
  gx += -2 * T(sh::K2b) * x * gY[6];
  gy += -2 * T(sh::K2b) * y * gY[6];
  gz += 4 * T(sh::K2b) * z * gY[6];
  // Y7 = -a xz
  gx += -T(sh::K2a) * z * gY[7];
  gz += -T(sh::K2a) * x * gY[7];
  // Y8 = c (xx - yy)
  gx += 2 * T(sh::K2c) * x * gY[8];
  gy += -2 * T(sh::K2c) * y * gY[8];
  if (deg < 3) return;
  // Y9 = -a (3 xx y - y^3)
  gx += -6 * T(sh::K3a) * x * y * gY[9];
  gy += -3 * T(sh::K3a) * (xx - yy) * gY[9];
  // Y10 = b xyz
  gx += T(sh::K3b) * y * z * gY[10];
  gy += T(sh::K3b) * x * z * gY[10];
  gz += T(sh::K3b) * x * y * gY[10];
  // Y11 = -c (4 y zz - xx y - y^3)
  gx += 2 * T(sh::K3c) * x * y * gY[11];
  gy += -T(sh::K3c) * (4 * zz - xx - 3 * yy) * gY[11];
  gz += -8 * T(sh::K3c) * y * z * gY[11];
  // Y12 = d (2 z^3 - 3 xx z - 3 yy z)
  gx += -6 * T(sh::K3d) * x * z * gY[12];
  gy += -6 * T(sh::K3d) * y * z * gY[12];
  gz += T(sh::K3d) * (6 * zz - 3 * xx - 3 * yy) * gY[12];
  // Y13 = -c (4 x zz - x^3 - x yy)
  gx += -T(sh::K3c) * (4 * zz - 3 * xx - yy) * gY[13];
  gy += 2 * T(sh::K3c) * x * y * gY[13];
  gz += -8 * T(sh::K3c) * x * z * gY[13];
  // Y14 = e z (xx - yy)
  gx += 2 * T(sh::K3e) * x * z * gY[14];
  gy += -2 * T(sh::K3e) * y * z * gY[14];
  gz += T(sh::K3e) * (xx - yy) * gY[14];
  // Y15 = -a (x^3 - 3 x yy)
  gx += -3 * T(sh::K3a) * (xx - yy) * gY[15];
  gy += 6 * T(sh::K3a) * x * y * gY[15];
}

// ---------------------------------------------------------------------------
// Rotor normalisation and rotor -> matrix.  Storage order:
// 0 s, 1 b01, 2 b02, 3 b12, 4 b03, 5 b13, 6 b23, 7 p.

template <typename T>
R4D_HD void rotor_fwd(Fwd<T>& f) {
  const T* r = f.r;
  const T s = r[0], b01 = r[1], b02 = r[2], b12 = r[3], b03 = r[4], b13 = r[5], b23 = r[6],
          p = r[7];
  f.eps = p * s - b01 * b23 + b02 * b13 - b03 * b12;
  // grad eps: the involution pairing s<->p, b01<->b23, b02<->b13, b03<->b12
  f.g[0] = p;
  f.g[1] = -b23;
  f.g[2] = b13;
  f.g[3] = -b03;
  f.g[4] = -b12;
  f.g[5] = b02;
  f.g[6] = -b01;
  f.g[7] = s;
  T l2 = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) l2 += r[i] * r[i];
  f.l2 = l2;
  const T disc = tmax(l2 * l2 - 4 * f.eps * f.eps, T(0));
  f.sq = r4d_sqrt(disc);
  f.den = l2 + f.sq;
  f.delta = f.den > T(0) ? -2 * f.eps / f.den : T(0);
  T n2 = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    f.r1[i] = r[i] + f.delta * f.g[i];
    n2 += f.r1[i] * f.r1[i];
  }
  f.degenerate = !(l2 >= T(1e-12)) || !(n2 >= T(1e-12));
  if (f.degenerate) {
    f.inv_n1 = T(0);
#pragma unroll
    for (int i = 0; i < 8; ++i) f.rn[i] = T(0);
    f.rn[0] = T(1);
  } else {
    f.inv_n1 = T(1) / r4d_sqrt(n2);
#pragma unroll
    for (int i = 0; i < 8; ++i) f.rn[i] = f.r1[i] * f.inv_n1;
  }
  const T* q = f.rn;
  const T S = q[0], a01 = q[1], a02 = q[2], a12 = q[3], a03 = q[4], a13 = q[5], a23 = q[6],
          P = q[7];
  const T S2 = S * S, P2 = P * P, x01 = a01 * a01, x02 = a02 * a02, x12 = a12 * a12,
          x03 = a03 * a03, x13 = a13 * a13, x23 = a23 * a23;
  T* R = f.R;
  R[0] = -x01 - x02 - x03 + x12 + x13 + x23 - P2 + S2;
  R[1] = 2 * (a01 * S - a02 * a12 - a03 * a13 + a23 * P);
  R[2] = 2 * (a01 * a12 + a02 * S - a03 * a23 - a13 * P);
  R[3] = 2 * (a01 * a13 + a02 * a23 + a03 * S + a12 * P);
  R[4] = 2 * (-a01 * S - a02 * a12 - a03 * a13 - a23 * P);
  R[5] = -x01 + x02 + x03 - x12 - x13 + x23 - P2 + S2;
  R[6] = 2 * (-a01 * a02 + a03 * P + a12 * S - a13 * a23);
  R[7] = 2 * (-a01 * a03 - a02 * P + a12 * a23 + a13 * S);
  R[8] = 2 * (a01 * a12 - a02 * S - a03 * a23 + a13 * P);
  R[9] = 2 * (-a01 * a02 - a03 * P - a12 * S - a13 * a23);
  R[10] = x01 - x02 + x03 - x12 + x13 - x23 - P2 + S2;
  R[11] = 2 * (a01 * P - a02 * a03 - a12 * a13 + a23 * S);
  R[12] = 2 * (a01 * a13 + a02 * a23 - a03 * S - a12 * P);
  R[13] = 2 * (-a01 * a03 + a02 * P + a12 * a23 - a13 * S);
  R[14] = 2 * (-a01 * P - a02 * a03 - a12 * a13 - a23 * S);
  R[15] = x01 + x02 - x03 + x12 - x13 - x23 - P2 + S2;
}

// dL/dR (16, row-major) -> dL/d(normalised rotor) -> dL/d(raw rotor), added to gr.
template <typename T>
R4D_HD void rotor_bwd(const Fwd<T>& f, const T* G, T* gr) {
  if (f.degenerate) return;
  const T* q = f.rn;
  const T S = q[0], a01 = q[1], a02 = q[2], a12 = q[3], a03 = q[4], a13 = q[5], a23 = q[6],
          P = q[7];
  T gS = 0, g01 = 0, g02 = 0, g12 = 0, g03 = 0, g13 = 0, g23 = 0, gP = 0;
  // diagonal entries: R_kk = sum_m sign_km c_m^2
  {
    const T d0 = G[0], d1 = G[5], d2 = G[10], d3 = G[15];
    gS += 2 * S * (d0 + d1 + d2 + d3);
    gP += -2 * P * (d0 + d1 + d2 + d3);
    g01 += 2 * a01 * (-d0 - d1 + d2 + d3);
    g02 += 2 * a02 * (-d0 + d1 - d2 + d3);
    g12 += 2 * a12 * (d0 - d1 - d2 + d3);
    g03 += 2 * a03 * (-d0 + d1 + d2 - d3);
    g13 += 2 * a13 * (d0 - d1 + d2 - d3);
    g23 += 2 * a23 * (d0 + d1 - d2 - d3);
  }
  // off-diagonal entries: each 2 * (sum of signed bilinear terms)
#define R4D_BL(Gv, sgn, X, gX, Y, gY) \
  do {                                \
    gX += (sgn)*2 * (Y) * (Gv);       \
    gY += (sgn)*2 * (X) * (Gv);       \
  } while (0)
  // R01 = 2(b01 s - b02 b12 - b03 b13 + b23 p)
  R4D_BL(G[1], 1, a01, g01, S, gS);
  R4D_BL(G[1], -1, a02, g02, a12, g12);
  R4D_BL(G[1], -1, a03, g03, a13, g13);
  R4D_BL(G[1], 1, a23, g23, P, gP);
  // R02 = 2(b01 b12 + b02 s - b03 b23 - b13 p)
  R4D_BL(G[2], 1, a01, g01, a12, g12);
  R4D_BL(G[2], 1, a02, g02, S, gS);
  R4D_BL(G[2], -1, a03, g03, a23, g23);
  R4D_BL(G[2], -1, a13, g13, P, gP);
  // R03 = 2(b01 b13 + b02 b23 + b03 s + b12 p)
  R4D_BL(G[3], 1, a01, g01, a13, g13);
  R4D_BL(G[3], 1, a02, g02, a23, g23);
  R4D_BL(G[3], 1, a03, g03, S, gS);
  R4D_BL(G[3], 1, a12, g12, P, gP);
  // R10 = 2(-b01 s - b02 b12 - b03 b13 - b23 p)
  R4D_BL(G[4], -1, a01, g01, S, gS);
  R4D_BL(G[4], -1, a02, g02, a12, g12);
  R4D_BL(G[4], -1, a03, g03, a13, g13);
  R4D_BL(G[4], -1, a23, g23, P, gP);
  // R12 = 2(-b01 b02 + b03 p + b12 s - b13 b23)
  R4D_BL(G[6], -1, a01, g01, a02, g02);
  R4D_BL(G[6], 1, a03, g03, P, gP);
  R4D_BL(G[6], 1, a12, g12, S, gS);
  R4D_BL(G[6], -1, a13, g13, a23, g23);
  // R13 = 2(-b01 b03 - b02 p + b12 b23 + b13 s)
  R4D_BL(G[7], -1, a01, g01, a03, g03);
  R4D_BL(G[7], -1, a02, g02, P, gP);
  R4D_BL(G[7], 1, a12, g12, a23, g23);
  R4D_BL(G[7], 1, a13, g13, S, gS);
  // R20 = 2(b01 b12 - b02 s - b03 b23 + b13 p)
  R4D_BL(G[8], 1, a01, g01, a12, g12);
  R4D_BL(G[8], -1, a02, g02, S, gS);
  R4D_BL(G[8], -1, a03, g03, a23, g23);
  R4D_BL(G[8], 1, a13, g13, P, gP);
  // R21 = 2(-b01 b02 - b03 p - b12 s - b13 b23)
  R4D_BL(G[9], -1, a01, g01, a02, g02);
  R4D_BL(G[9], -1, a03, g03, P, gP);
  R4D_BL(G[9], -1, a12, g12, S, gS);
  R4D_BL(G[9], -1, a13, g13, a23, g23);
  // R23 = 2(b01 p - b02 b03 - b12 b13 + b23 s)
  R4D_BL(G[11], 1, a01, g01, P, gP);
  R4D_BL(G[11], -1, a02, g02, a03, g03);
  R4D_BL(G[11], -1, a12, g12, a13, g13);
  R4D_BL(G[11], 1, a23, g23, S, gS);
  // R30 = 2(b01 b13 + b02 b23 - b03 s - b12 p)
  R4D_BL(G[12], 1, a01, g01, a13, g13);
  R4D_BL(G[12], 1, a02, g02, a23, g23);
  R4D_BL(G[12], -1, a03, g03, S, gS);
  R4D_BL(G[12], -1, a12, g12, P, gP);
  // R31 = 2(-b01 b03 + b02 p + b12 b23 - b13 s)
  R4D_BL(G[13], -1, a01, g01, a03, g03);
  R4D_BL(G[13], 1, a02, g02, P, gP);
  R4D_BL(G[13], 1, a12, g12, a23, g23);
  R4D_BL(G[13], -1, a13, g13, S, gS);
  // R32 = 2(-b01 p - b02 b03 - b12 b13 - b23 s)
  R4D_BL(G[14], -1, a01, g01, P, gP);
  R4D_BL(G[14], -1, a02, g02, a03, g03);
  R4D_BL(G[14], -1, a12, g12, a13, g13);
  R4D_BL(G[14], -1, a23, g23, S, gS);
#undef R4D_BL
  const T gn[8] = {gS, g01, g02, g12, g03, g13, g23, gP};
  // rn = r1 / |r1|
  T dot = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) dot += f.rn[i] * gn[i];
  T g1[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) g1[i] = (gn[i] - f.rn[i] * dot) * f.inv_n1;
  // r1 = r + delta(r) grad_eps(r); grad_eps is linear and symmetric (an involution
  // with signs), so its transpose maps g1 the same way.
  T gdelta = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) gdelta += g1[i] * f.g[i];
  T Pg1[8];
  Pg1[0] = g1[7];
  Pg1[1] = -g1[6];
  Pg1[2] = g1[5];
  Pg1[3] = -g1[4];
  Pg1[4] = -g1[3];
  Pg1[5] = g1[2];
  Pg1[6] = -g1[1];
  Pg1[7] = g1[0];
  // delta = -2 eps / den, den = l2 + sqrt(l2^2 - 4 eps^2)
  T ddelta_deps = 0, ddelta_dl2 = 0;
  if (f.den > T(0)) {
    const T inv_den = T(1) / f.den;
    T dden_deps = 0, dden_dl2 = 1;
    if (f.sq > T(0)) {
      dden_deps = -4 * f.eps / f.sq;
      dden_dl2 = 1 + f.l2 / f.sq;
    }
    ddelta_deps = -2 * inv_den + 2 * f.eps * inv_den * inv_den * dden_deps;
    ddelta_dl2 = 2 * f.eps * inv_den * inv_den * dden_dl2;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
    gr[i] += g1[i] + f.delta * Pg1[i] + gdelta * (ddelta_deps * f.g[i] + ddelta_dl2 * 2 * f.r[i]);
}

// ---------------------------------------------------------------------------
// Sigma_4 = R diag(s^2) R^T of one Gaussian from its raw rotor and log-scales
// (Sec. 3.2.1): fills the rotor, rotation, s^2, U, V and W fields of f.
template <typename T>
R4D_HD void cov4_fwd(const T ls[4], const T rot[8], Fwd<T>& f) {
#pragma unroll
  for (int i = 0; i < 8; ++i) f.r[i] = rot[i];
  rotor_fwd(f);
#pragma unroll
  for (int k = 0; k < 4; ++k) f.s2[k] = r4d_exp(2 * ls[k]);
  const T* R = f.R;
  // Sigma_ij = sum_k R_ik R_jk s_k^2
  auto sig = [&](int i, int j) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += R[4 * i + k] * R[4 * j + k] * f.s2[k];
    return acc;
  };
  f.U[0] = sig(0, 0);
  f.U[1] = sig(0, 1);
  f.U[2] = sig(0, 2);
  f.U[3] = sig(1, 1);
  f.U[4] = sig(1, 2);
  f.U[5] = sig(2, 2);
  f.V[0] = sig(0, 3);
  f.V[1] = sig(1, 3);
  f.V[2] = sig(2, 3);
  f.W = sig(3, 3);
}

// Given G4, the full symmetric gradient of L with respect to Sigma_4, adds
// dL/d(log-scales) and dL/d(raw rotor).
template <typename T>
R4D_HD void cov4_bwd(const Fwd<T>& f, const T G4[16], T gls[4], T grot[8]) {
  const T* R = f.R;
  // G4 R
  T GR[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      GR[4 * i + k] = G4[4 * i] * R[k] + G4[4 * i + 1] * R[4 + k] + G4[4 * i + 2] * R[8 + k] +
                      G4[4 * i + 3] * R[12 + k];
  // dL/dR_ik = 2 (G4 R)_ik s2_k ; dL/ds2_k = (R^T G4 R)_kk
  T gR[16];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) gR[4 * i + k] = 2 * GR[4 * i + k] * f.s2[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T gs2 = R[k] * GR[k] + R[4 + k] * GR[4 + k] + R[8 + k] * GR[8 + k] + R[12 + k] * GR[12 + k];
    gls[k] += gs2 * 2 * f.s2[k];
  }
  rotor_bwd(f, gR, grot);
}

// ---------------------------------------------------------------------------
// Projection and colour of a 3D Gaussian (f.mu3, f.S3, f.vel, f.o_t set): view
// transform, near-plane drop, EWA projection, conic, 2D flow, SH colour
// (Sec. 3.1).  Sets f.valid when the Gaussian survives.
template <typename T, typename ShT>
R4D_HD void project_fwd(const ShT* shp, long sh_stride, int deg, const ViewDev& v,
                        const SettingsDev& st, Fwd<T>& f) {
  // view transform
  const T* mu = f.mu3;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    f.p[i] = T(v.M[3 * i]) * mu[0] + T(v.M[3 * i + 1]) * mu[1] + T(v.M[3 * i + 2]) * mu[2] +
             T(v.tw[i]);
  if (!(f.p[2] > T(st.near_plane))) return;
  f.ipz = T(1) / f.p[2];
  const T rx = f.p[0] * f.ipz, ry = f.p[1] * f.ipz;
  const T lx = T(v.limx), ly = T(v.limy);
  f.clx = rx < -lx || rx > lx;
  f.cly = ry < -ly || ry > ly;
  f.txz = tmin(lx, tmax(-lx, rx));
  f.tyz = tmin(ly, tmax(-ly, ry));
  const T fx = T(v.fx), fy = T(v.fy);
  const T J00 = fx * f.ipz, J02 = -fx * f.txz * f.ipz;
  const T J11 = fy * f.ipz, J12 = -fy * f.tyz * f.ipz;
  // Tm = J Wv
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    f.Tm[c] = J00 * T(v.M[c]) + J02 * T(v.M[6 + c]);
    f.Tm[3 + c] = J11 * T(v.M[3 + c]) + J12 * T(v.M[6 + c]);
  }
  // Sigma_2D = Tm S3 Tm^T + dilation I
  const T* S = f.S3;
  const T* a = f.Tm;
  const T* b = f.Tm + 3;
  const T Sa0 = S[0] * a[0] + S[1] * a[1] + S[2] * a[2];
  const T Sa1 = S[1] * a[0] + S[3] * a[1] + S[4] * a[2];
  const T Sa2 = S[2] * a[0] + S[4] * a[1] + S[5] * a[2];
  const T Sb0 = S[0] * b[0] + S[1] * b[1] + S[2] * b[2];
  const T Sb1 = S[1] * b[0] + S[3] * b[1] + S[4] * b[2];
  const T Sb2 = S[2] * b[0] + S[4] * b[1] + S[5] * b[2];
  f.A = a[0] * Sa0 + a[1] * Sa1 + a[2] * Sa2 + T(st.dilation);
  f.B = a[0] * Sb0 + a[1] * Sb1 + a[2] * Sb2;
  f.C = b[0] * Sb0 + b[1] * Sb1 + b[2] * Sb2 + T(st.dilation);
  f.det = f.A * f.C - f.B * f.B;
  if (!(f.det > T(0))) return;
  const T idet = T(1) / f.det;
  f.conic[0] = f.C * idet;
  f.conic[1] = -f.B * idet;
  f.conic[2] = f.A * idet;
  f.mean2[0] = fx * f.p[0] * f.ipz + T(v.cx);
  f.mean2[1] = fy * f.p[1] * f.ipz + T(v.cy);
  // flow: d/dt of (fx x / z, fy y / z) with d p / dt = Wv vel
#pragma unroll
  for (int i = 0; i < 3; ++i)
    f.vc[i] = T(v.M[3 * i]) * f.vel[0] + T(v.M[3 * i + 1]) * f.vel[1] +
              T(v.M[3 * i + 2]) * f.vel[2];
  f.flow[0] = fx * f.ipz * (f.vc[0] - f.p[0] * f.ipz * f.vc[2]);
  f.flow[1] = fy * f.ipz * (f.vc[1] - f.p[1] * f.ipz * f.vc[2]);
  // colour
#pragma unroll
  for (int i = 0; i < 3; ++i) f.dir[i] = mu[i] - T(v.cam[i]);
  f.inv_nd = T(1) / r4d_sqrt(f.dir[0] * f.dir[0] + f.dir[1] * f.dir[1] + f.dir[2] * f.dir[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) f.d[i] = f.dir[i] * f.inv_nd;
  T Y[16];
  sh_eval(deg, f.d[0], f.d[1], f.d[2], Y);
  const int k = (deg + 1) * (deg + 1);
#pragma unroll
  for (int c = 0; c < 3; ++c) f.raw[c] = T(0.5);
  for (int j = 0; j < k; ++j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) f.raw[c] += Y[j] * T(shp[(3 * j + c) * sh_stride]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) f.rgb[c] = tmax(f.raw[c], T(0));
  f.valid = true;
}

// ---------------------------------------------------------------------------
// Full per-Gaussian forward.  `sh` points at coefficient 0 of this Gaussian's
// [3k] SH column (stride n between rows).

template <typename T, typename ShT>
R4D_HD void gaussian_fwd(const T mu4[4], const T ls[4], const T rot[8], T opacity, const ShT* shp,
                         long sh_stride, int deg, const ViewDev& v, const SettingsDev& st,
                         Fwd<T>& f) {
  f.valid = false;
  cov4_fwd(ls, rot, f);
  // temporal slice
  f.dt = T(v.t) - mu4[3];
  f.invW = T(1) / f.W;
  f.lam_dt2 = f.dt * f.dt * f.invW;
  if (!(f.lam_dt2 <= T(st.time_cull))) return;
  f.decay = r4d_exp(T(-0.5) * f.lam_dt2);
  f.o_t = opacity * f.decay;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    f.vel[i] = f.V[i] * f.invW;
    f.mu3[i] = mu4[i] + f.dt * f.vel[i];
  }
  f.S3[0] = f.U[0] - f.V[0] * f.vel[0];
  f.S3[1] = f.U[1] - f.V[0] * f.vel[1];
  f.S3[2] = f.U[2] - f.V[0] * f.vel[2];
  f.S3[3] = f.U[3] - f.V[1] * f.vel[1];
  f.S3[4] = f.U[4] - f.V[1] * f.vel[2];
  f.S3[5] = f.U[5] - f.V[2] * f.vel[2];
  project_fwd(shp, sh_stride, deg, v, st, f);
}

// Static 3D Gaussian (the paper's 3D/4D unification, Sec. 3.2.1: a rotor with
// no temporal part acts as a quaternion and the Gaussian does not move, so its
// slice at every time is the 3D Gaussian itself, with no opacity decay).
// q = (w, x, y, z), normalised here; R3 the usual quaternion rotation, equal to
// the rotor rotation of (s, b01, b02, b12) = (w, -z, y, -x);
// Sigma_3D = R3 diag(s^2) R3^T.  R3 is kept in f.R[0..8] (row-major), the
// normalised quaternion in f.rn[0..3].
template <typename T>
R4D_HD void quat_fwd(const T q[4], Fwd<T>& f) {
  const T n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  f.degenerate = !(n2 >= T(1e-12));
  f.inv_n1 = f.degenerate ? T(0) : T(1) / r4d_sqrt(n2);
#pragma unroll
  for (int i = 0; i < 4; ++i) f.rn[i] = f.degenerate ? (i == 0 ? T(1) : T(0)) : q[i] * f.inv_n1;
  const T w = f.rn[0], x = f.rn[1], y = f.rn[2], z = f.rn[3];
  T* R = f.R;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

template <typename T, typename ShT>
R4D_HD void gaussian_fwd_static(const T mu[3], const T ls[3], const T q[4], T opacity,
                                const ShT* shp, long sh_stride, int deg, const ViewDev& v,
                                const SettingsDev& st, Fwd<T>& f) {
  f.valid = false;
  quat_fwd(q, f);
#pragma unroll
  for (int k = 0; k < 3; ++k) f.s2[k] = r4d_exp(2 * ls[k]);
  const T* R = f.R;
  auto sig = [&](int i, int j) {
    return R[3 * i] * R[3 * j] * f.s2[0] + R[3 * i + 1] * R[3 * j + 1] * f.s2[1] +
           R[3 * i + 2] * R[3 * j + 2] * f.s2[2];
  };
  f.S3[0] = sig(0, 0);
  f.S3[1] = sig(0, 1);
  f.S3[2] = sig(0, 2);
  f.S3[3] = sig(1, 1);
  f.S3[4] = sig(1, 2);
  f.S3[5] = sig(2, 2);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    f.mu3[i] = mu[i];
    f.vel[i] = T(0);
  }
  f.decay = T(1);
  f.o_t = opacity;
  project_fwd(shp, sh_stride, deg, v, st, f);
}

// Gradients of one Gaussian.  In: dL/d(mean2 x, y), the gradient H of L with
// respect to the symmetric 2x2 matrix Sigma_2D (entries (0,0), (0,1) = (1,0),
// (1,1); a change dS of the matrix changes L by sum_ij H_ij dS_ij), dL/d(o_t),
// dL/d(rgb), and with FLOW dL/d(flow x, y) in g2[9], g2[10].  Out (added):
// mu4[4], ls[4], rot[8], opacity, and the SH column via gsh (stride gsh_stride).
//
// The rasteriser hands over the Sigma_2D gradient rather than the conic one: for
// a long thin footprint the conic gradient is dominated by a component along the
// major axis that Sigma_2D = conic^-1 almost ignores, so forming -Q G Q from it
// in single precision cancels badly; the rasteriser instead sums the well-scaled
// per-pixel terms (Q d)(Q d)^T directly.
//
// project_bwd is the part shared by 4D and static Gaussians: it leaves
// dL/d(mu3), the symmetric full-matrix gradient dL/d(Sigma_3D) (6 unique
// entries), dL/d(vel) of the flow (FLOW) and dL/d(o_t), and adds the SH
// gradient.
template <typename T, typename ShT, bool FLOW>
R4D_HD void project_bwd(const Fwd<T>& f, const ShT* shp, long sh_stride, int deg,
                        const ViewDev& v, const T* g2, T gmu3[3], T gS3[6], T gvel[3], T& go_t,
                        T* gsh, long gsh_stride) {
  const T gm_x = g2[0], gm_y = g2[1];
  const T H00 = g2[2], H01 = g2[3], H11 = g2[4];
  go_t = g2[5];
  const T grgb[3] = {g2[6], g2[7], g2[8]};
#pragma unroll
  for (int i = 0; i < 3; ++i) gmu3[i] = gvel[i] = T(0);
  // ---- SH colour
  {
    T graw[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) graw[c] = f.raw[c] >= T(0) ? grgb[c] : T(0);
    T Y[16];
    sh_eval(deg, f.d[0], f.d[1], f.d[2], Y);
    const int k = (deg + 1) * (deg + 1);
    T gY[16];
    for (int j = 0; j < k; ++j) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gsh[(3 * j + c) * gsh_stride] += Y[j] * graw[c];
        acc += T(shp[(3 * j + c) * sh_stride]) * graw[c];
      }
      gY[j] = acc;
    }
    T gdx, gdy, gdz;
    sh_grad(deg, f.d[0], f.d[1], f.d[2], gY, gdx, gdy, gdz);
    const T dot = gdx * f.d[0] + gdy * f.d[1] + gdz * f.d[2];
    gmu3[0] += (gdx - f.d[0] * dot) * f.inv_nd;
    gmu3[1] += (gdy - f.d[1] * dot) * f.inv_nd;
    gmu3[2] += (gdz - f.d[2] * dot) * f.inv_nd;
  }
  // Sigma_2D = Tm S3 Tm^T: dL/dS3 = Tm^T H Tm ; dL/dTm = 2 H Tm S3
  const T* a = f.Tm;
  const T* b = f.Tm + 3;
  // (Tm^T H Tm)_ij = a_i (H00 a_j + H01 b_j) + b_i (H01 a_j + H11 b_j)
  {
    T ha[3], hb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ha[j] = H00 * a[j] + H01 * b[j];
      hb[j] = H01 * a[j] + H11 * b[j];
    }
    gS3[0] = a[0] * ha[0] + b[0] * hb[0];
    gS3[1] = a[0] * ha[1] + b[0] * hb[1];
    gS3[2] = a[0] * ha[2] + b[0] * hb[2];
    gS3[3] = a[1] * ha[1] + b[1] * hb[1];
    gS3[4] = a[1] * ha[2] + b[1] * hb[2];
    gS3[5] = a[2] * ha[2] + b[2] * hb[2];
  }
  T gTm[6];
  {
    const T* S = f.S3;
    const T Sa[3] = {S[0] * a[0] + S[1] * a[1] + S[2] * a[2], S[1] * a[0] + S[3] * a[1] + S[4] * a[2],
                     S[2] * a[0] + S[4] * a[1] + S[5] * a[2]};
    const T Sb[3] = {S[0] * b[0] + S[1] * b[1] + S[2] * b[2], S[1] * b[0] + S[3] * b[1] + S[4] * b[2],
                     S[2] * b[0] + S[4] * b[1] + S[5] * b[2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      gTm[j] = 2 * (H00 * Sa[j] + H01 * Sb[j]);
      gTm[3 + j] = 2 * (H01 * Sa[j] + H11 * Sb[j]);
    }
  }
  // Tm = J Wv: dL/dJ = dL/dTm Wv^T (only J00, J02, J11, J12 are non-zero entries)
  T gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gJ00 += gTm[c] * T(v.M[c]);
    gJ02 += gTm[c] * T(v.M[6 + c]);
    gJ11 += gTm[3 + c] * T(v.M[3 + c]);
    gJ12 += gTm[3 + c] * T(v.M[6 + c]);
  }
  const T fx = T(v.fx), fy = T(v.fy);
  const T ipz = f.ipz, ipz2 = ipz * ipz;
  T gp[3] = {0, 0, 0};
  // J00 = fx/z, J11 = fy/z
  gp[2] += -(gJ00 * fx + gJ11 * fy) * ipz2;
  // J02 = -fx x/z^2 (unclamped) or -fx L/z (x/z clamped to L)
  if (!f.clx) {
    gp[0] += -gJ02 * fx * ipz2;
    gp[2] += gJ02 * 2 * fx * f.p[0] * ipz2 * ipz;
  } else {
    gp[2] += gJ02 * fx * f.txz * ipz2;
  }
  if (!f.cly) {
    gp[1] += -gJ12 * fy * ipz2;
    gp[2] += gJ12 * 2 * fy * f.p[1] * ipz2 * ipz;
  } else {
    gp[2] += gJ12 * fy * f.tyz * ipz2;
  }
  // mean2 = (fx x/z + cx, fy y/z + cy)
  gp[0] += gm_x * fx * ipz;
  gp[1] += gm_y * fy * ipz;
  gp[2] += -(gm_x * fx * f.p[0] + gm_y * fy * f.p[1]) * ipz2;
  // flow = (fx (vx/z - x vz/z^2), fy (vy/z - y vz/z^2)), vc = Wv vel
  if (FLOW) {
    const T hx = g2[9] * fx, hy = g2[10] * fy;
    const T ipz3 = ipz2 * ipz;
    const T gvc0 = hx * ipz, gvc1 = hy * ipz;
    const T gvc2 = -(hx * f.p[0] + hy * f.p[1]) * ipz2;
    gp[0] += -hx * f.vc[2] * ipz2;
    gp[1] += -hy * f.vc[2] * ipz2;
    gp[2] += hx * (2 * f.p[0] * f.vc[2] * ipz3 - f.vc[0] * ipz2) +
             hy * (2 * f.p[1] * f.vc[2] * ipz3 - f.vc[1] * ipz2);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      gvel[c] = T(v.M[c]) * gvc0 + T(v.M[3 + c]) * gvc1 + T(v.M[6 + c]) * gvc2;
  }
  // p = Wv mu3 + tw
#pragma unroll
  for (int c = 0; c < 3; ++c)
    gmu3[c] += T(v.M[c]) * gp[0] + T(v.M[3 + c]) * gp[1] + T(v.M[6 + c]) * gp[2];
}

template <typename T, typename ShT, bool FLOW = false>
R4D_HD void gaussian_bwd(const Fwd<T>& f, const ShT* shp, long sh_stride, int deg,
                         const ViewDev& v, const T* g2, T gmu4[4], T gls[4], T grot[8],
                         T& gop, T* gsh, long gsh_stride) {
  if (!f.valid) return;
  T gmu3[3], gS3[6], gvel[3], go_t;
  project_bwd<T, ShT, FLOW>(f, shp, sh_stride, deg, v, g2, gmu3, gS3, gvel, go_t, gsh,
                            gsh_stride);
  // ---- temporal slice
  // mu3 = mu_xyz + dt vel, vel = V/W (also the flow's speed) ; S3 = U - V V^T / W ;
  // o_t = o exp(-dt^2/(2W))
  T gV[3], gW = 0, gdt = 0;
  {
    // gS3 holds the symmetric full-matrix gradient Tm^T H Tm (entry (i,j) and
    // (j,i) equal; a unique off-diagonal scalar has twice that gradient).
    const T Gs[9] = {gS3[0], gS3[1], gS3[2],
                     gS3[1], gS3[3], gS3[4],
                     gS3[2], gS3[4], gS3[5]};
    T GV[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      GV[i] = Gs[3 * i] * f.V[0] + Gs[3 * i + 1] * f.V[1] + Gs[3 * i + 2] * f.V[2];
    const T VGV = f.V[0] * GV[0] + f.V[1] * GV[1] + f.V[2] * GV[2];
    // dL/dvel = dt dL/dmu3 + (flow part)
    T gv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) gv[i] = f.dt * gmu3[i] + gvel[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) gV[i] = -2 * GV[i] * f.invW + gv[i] * f.invW;
    const T vdot = f.vel[0] * gmu3[0] + f.vel[1] * gmu3[1] + f.vel[2] * gmu3[2];
    const T vgv = f.vel[0] * gv[0] + f.vel[1] * gv[1] + f.vel[2] * gv[2];
    gW += VGV * f.invW * f.invW - vgv * f.invW;
    gW += go_t * f.o_t * T(0.5) * f.dt * f.dt * f.invW * f.invW;
    gdt += vdot - go_t * f.o_t * f.dt * f.invW;
  }
  gmu4[0] += gmu3[0];
  gmu4[1] += gmu3[1];
  gmu4[2] += gmu3[2];
  gmu4[3] += -gdt;
  gop += go_t * f.decay;
  // ---- Sigma_4 = R diag(s2) R^T ; full symmetric gradient G4
  T G4[16];
  G4[0] = gS3[0];
  G4[1] = G4[4] = gS3[1];
  G4[2] = G4[8] = gS3[2];
  G4[5] = gS3[3];
  G4[6] = G4[9] = gS3[4];
  G4[10] = gS3[5];
  G4[3] = G4[12] = T(0.5) * gV[0];
  G4[7] = G4[13] = T(0.5) * gV[1];
  G4[11] = G4[14] = T(0.5) * gV[2];
  G4[15] = gW;
  // the U block of Sigma_4 enters Sigma_3D directly: dL/dU = dL/dS3 (already in G4)
  cov4_bwd(f, G4, gls, grot);
}

// dL/dR3 (9, row-major) of the normalised quaternion's rotation -> dL/d(raw
// quaternion), added to gq.
template <typename T>
R4D_HD void quat_bwd(const Fwd<T>& f, const T G[9], T gq[4]) {
  if (f.degenerate) return;
  const T w = f.rn[0], x = f.rn[1], y = f.rn[2], z = f.rn[3];
  // derivatives of the nine entries written out per component
  const T gw = 2 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  const T gx = 2 * (y * G[1] + z * G[2] + y * G[3] - 2 * x * G[4] - w * G[5] + z * G[6] +
                    w * G[7] - 2 * x * G[8]);
  const T gy = 2 * (-2 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] +
                    z * G[7] - 2 * y * G[8]);
  const T gz = 2 * (-2 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2 * z * G[4] + y * G[5] +
                    x * G[6] + y * G[7]);
  // q_hat = q / |q|
  const T dot = w * gw + x * gx + y * gy + z * gz;
  gq[0] += (gw - w * dot) * f.inv_n1;
  gq[1] += (gx - x * dot) * f.inv_n1;
  gq[2] += (gy - y * dot) * f.inv_n1;
  gq[3] += (gz - z * dot) * f.inv_n1;
}

// Gradients of a static 3D Gaussian (see gaussian_fwd_static): g2 as for
// gaussian_bwd (no flow); out (added): mu[3], ls[3], q[4], opacity, SH column.
template <typename T, typename ShT>
R4D_HD void gaussian_bwd_static(const Fwd<T>& f, const ShT* shp, long sh_stride, int deg,
                                const ViewDev& v, const T* g2, T gmu[3], T gls[3], T gq[4],
                                T& gop, T* gsh, long gsh_stride) {
  if (!f.valid) return;
  T gmu3[3], gS3[6], gvel[3], go_t;
  project_bwd<T, ShT, false>(f, shp, sh_stride, deg, v, g2, gmu3, gS3, gvel, go_t, gsh,
                             gsh_stride);
#pragma unroll
  for (int i = 0; i < 3; ++i) gmu[i] += gmu3[i];
  gop += go_t;
  // Sigma_3D = R3 diag(s2) R3^T with the full symmetric gradient G
  const T G[9] = {gS3[0], gS3[1], gS3[2], gS3[1], gS3[3], gS3[4], gS3[2], gS3[4], gS3[5]};
  const T* R = f.R;
  T GR[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      GR[3 * i + k] = G[3 * i] * R[k] + G[3 * i + 1] * R[3 + k] + G[3 * i + 2] * R[6 + k];
  T gR[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) gR[3 * i + k] = 2 * GR[3 * i + k] * f.s2[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T gs2 = R[k] * GR[k] + R[3 + k] * GR[3 + k] + R[6 + k] * GR[6 + k];
    gls[k] += gs2 * 2 * f.s2[k];
  }
  quat_bwd(f, gR, gq);
}

}  // namespace r4d
