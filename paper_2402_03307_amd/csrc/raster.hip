// Tile rasteriser: front-to-back alpha compositing (paper Sec. 3.1, blending
// equation) and its reverse-mode derivative.
//
// One workgroup per tile.  The tile's list of Gaussian indices (sorted by depth)
// is walked in batches: every lane loads one projected record into LDS, then
// every lane reads the whole batch back (a broadcast read) and updates its
// pixels.  A workgroup stops as soon as every pixel of the tile has reached the
// transmittance floor.
//
// Per (pixel, Gaussian): d = mean2d - (x + .5, y + .5), q = d^T conic d; skip if
// q > extent^2; a = min(alpha_max, o exp(-q/2)); skip if a < alpha_min; stop if
// T (1 - a) < T_min; else C += rgb a T, T *= 1 - a.  Background added with the
// final T.  The forward stores, per pixel, the final T and the number of list
// entries up to the last blended one; the backward walks the list back to front
// from there, recovering T by division by (1 - a).
//
// A flow render composites each Gaussian's 2D flow with the same weights as two
// more channels (background 0): the rendered optical flow of the speed field
// (Sec. 3.2.2), which the backward differentiates like a colour.
#include <hip/hip_runtime.h>

#include "front.hpp"
#include "r4d_internal.hpp"
#include "rowwalk.hpp"

namespace r4d {

namespace {

template <typename T> __device__ __forceinline__ T tfma(T a, T b, T c);
template <> __device__ __forceinline__ float tfma<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double tfma<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// exp2
template <typename T> __device__ __forceinline__ T texp2(T x);
template <> __device__ __forceinline__ float texp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double texp2<double>(double x) { return exp2(x); }

// -log2(e) / 2: exp(-q/2) = exp2(kHalfLog2e * q)
constexpr double kHalfLog2e = -0.72134752044448170368;

// A record as the rasteriser keeps it in LDS: the conic is pre-multiplied by
// k = -log2(e)/2 so that the Gaussian falloff is one exp2 of a quadratic form.
template <typename T>
struct Staged {
  T mx, my, A, B;
  T C, o, r, g;
  T b, e_thr, fu, fv;  // fu, fv: the 2D flow (flow renders; 0 otherwise)
};

template <typename T> __device__ __forceinline__ T tlog2(T x);
template <> __device__ __forceinline__ float tlog2<float>(float x) { return __log2f(x); }
template <> __device__ __forceinline__ double tlog2<double>(double x) { return log2(x); }

// e_thr: the smallest e (= k q, see eval_pair) at which the pair passes both
// the extent test (q <= extent^2, e >= k extent^2) and the alpha test
// (o exp2(e) >= alpha_min, e >= log2(alpha_min / o)).
template <typename T>
__device__ __forceinline__ Staged<T> stage(const Rec<T>& r, T e_min, T amin) {
  const T k = T(kHalfLog2e);
  const T e_alpha = tlog2(amin / r.o);
  return Staged<T>{r.mx, r.my, k * r.ca, k * r.cb, k * r.cc, r.o, r.r, r.g, r.b,
                   e_alpha > e_min ? e_alpha : e_min, T(0), T(0)};
}

// The one place where a (pixel, Gaussian) pair is evaluated; forward and backward
// call it with identical operands so that they take identical decisions.
// With d = mean2d - pixel centre: u = k Q d (the offset whitened by the conic Q),
// e = d . u = k q, G = exp2(e) = exp(-q/2), a_raw = o G, alpha = min(alpha_max,
// a_raw).  Evaluated without branches: the result says whether the pair passes
// the extent and alpha tests (e >= e_thr).  The backward builds its
// screen-space gradients from u.
template <typename T>
__device__ __forceinline__ bool eval_pair(const Staged<T>& r, T px, T py, T amax, T& ux, T& uy,
                                          T& G, T& a_raw, T& alpha) {
  const T dx = r.mx - px;
  const T dy = r.my - py;
  ux = tfma(r.B, dy, r.A * dx);
  uy = tfma(r.B, dx, r.C * dy);
  const T e = tfma(dx, ux, dy * uy);
  G = texp2(e);
  a_raw = r.o * G;
  alpha = fmin(a_raw, amax);
  return e >= r.e_thr;
}

// 1/x: the hardware reciprocal in float (about 1 ulp), exact division in double.
template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sums over each row of 16 lanes with DPP lane moves (no LDS traffic): pairs
// (quad_perm 1,0,3,2), quads (quad_perm 2,3,0,1), half rows (row_half_mirror),
// rows (row_mirror); afterwards every lane of a row holds its row's sums.  The
// N reductions advance step by step, so that the DPP moves of one value fill
// the hazard slots of the others.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false);
  return x + __int_as_float(moved);
}

template <int N>
__device__ __forceinline__ void row_sums(float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add<0xb1, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add<0x4e, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add<0x141, 0xf>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add<0x140, 0xf>(v[i]);
}

// x plus the value the lane move CTRL brings, all rows written (a lane with no
// source adds 0), so that the move folds into the addition.
template <int CTRL>
__device__ __forceinline__ float dpp_add_all(float x) {
  const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true);
  return x + __int_as_float(moved);
}

// Sums over the whole wavefront, valid in row 3 (lanes 48..63) only: the row
// sums r0..r3, then row_bcast:15 (lane 47 -> row 3, lane 15 -> row 1), which
// leaves r2 + r3 in row 3 and r0 + r1 in lane 31, then row_bcast:31 (lane 31
// -> row 3).  The other rows end up with partial sums that nothing reads.
template <int N>
__device__ __forceinline__ void wave_sums(float (&v)[N]) {
  row_sums(v);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add_all<0x142>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = dpp_add_all<0x143>(v[i]);
}
template <int N>
__device__ __forceinline__ void wave_sums(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
}

// gfx950 lane swaps.  permlane32_swap(x, y) exchanges the upper 32 lanes of x
// with the lower 32 lanes of y, so the sum of the two results holds x folded
// in half (lane l: x[l] + x[l + 32]) in lanes 0..31 and y folded in lanes
// 32..63.  permlane16_swap does the same with the odd 16-lane rows of x and the
// even rows of y: the sum holds rows (x0 + x1, y0 + y1, x2 + x3, y2 + y3).
__device__ __forceinline__ float fold32(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float fold16(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wavefront sums of the NC per-Gaussian components, stored to s_slot[c] (added,
// when several wavefronts share a tile).  Float: components are
// folded four at a time, fold16(fold32(a, b), fold32(c, d)), which leaves a,
// c, b, d partial sums in rows 0..3, and the row sums finish them; a ninth
// component alone takes the row sums and two row broadcasts (total in row 3).
// Lane 16 r stores row r's totals.
template <int NC, int NT>
__device__ __forceinline__ void store_wave_sums(float (&sv)[NC], float* s_slot, int lane) {
  static_assert(NC == 9 || NC == 11, "component groups of 4 + 1 or 4 + 3");
  float q[3];  // two groups of 4, then the rest
  q[0] = fold16(fold32(sv[0], sv[1]), fold32(sv[2], sv[3]));
  q[1] = fold16(fold32(sv[4], sv[5]), fold32(sv[6], sv[7]));
  if constexpr (NC == 9)
    q[2] = sv[8];
  else
    q[2] = fold16(fold32(sv[8], sv[9]), fold32(sv[10], 0.0f));
  row_sums(q);
  if constexpr (NC == 9) {
    q[2] = dpp_add_all<0x142>(q[2]);
    q[2] = dpp_add_all<0x143>(q[2]);
  }
  if ((lane & 15) == 0) {
    const int r = lane >> 4;
    const int c = ((r & 1) << 1) | (r >> 1);  // row r holds component 4 g + c of group g
    if (NT == 64) {
      s_slot[c] = q[0];
      s_slot[4 + c] = q[1];
      if (NC == 9 && r == 3) s_slot[8] = q[2];
      if (NC == 11 && c < 3) s_slot[8 + c] = q[2];
    } else {
      atomicAdd(&s_slot[c], q[0]);
      atomicAdd(&s_slot[4 + c], q[1]);
      if (NC == 9 && r == 3) atomicAdd(&s_slot[8], q[2]);
      if (NC == 11 && c < 3) atomicAdd(&s_slot[8 + c], q[2]);
    }
  }
}
template <int NC, int NT>
__device__ __forceinline__ void store_wave_sums(double (&sv)[NC], double* s_slot, int lane) {
  wave_sums(sv);
  if (lane == 63) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (NT == 64)
        s_slot[c] = sv[c];
      else
        atomicAdd(&s_slot[c], sv[c]);
    }
  }
}

template <typename T> __device__ __forceinline__ void atomic_add_nr(T* p, T v);
template <> __device__ __forceinline__ void atomic_add_nr<double>(double* p, double v) {
  atomicAdd(p, v);
}

// A workgroup covers one TS x TS tile with TS*TS/PPT lanes (a multiple of 64); lane t handles
// column t % TS of rows t / TS + k * (TS / PPT), k < PPT.  More pixels per lane
// amortise the LDS record reads (and, in the backward, the wavefront reductions).
template <int TS, int PPT>
struct TileCfg {
  static constexpr int kThreads = TS * TS / PPT;
  static constexpr int kRowStep = TS / PPT;
  // records staged in LDS per batch: small batches waste few loads on a tile
  // that saturates early in its list (measured faster than 128 or 256 on the
  // 500k / 1352x1014 render)
  static constexpr int kBatch = 64;
  // whole wavefronts only: the backward's reductions work on whole wavefronts
  static_assert(kThreads % 64 == 0, "a tile must map onto whole wavefronts");
};

// Collection of a tile's rest entries (front.hpp): the Gaussians at depth
// positions [r0, n_vis) of render vi whose row run in tile row ty covers
// column tx, in depth order, into a range of the render's rest area.  A pass
// over the depth-ordered tile boxes, kRestItems positions per thread per step
// (loaded together, the next step's while this one is finished): the
// positions whose box holds the tile are placed by a workgroup scan into a
// candidate list in LDS (in depth order), whose entries the threads then test
// one each against the row run, so that the dependent loads (index, record)
// of all candidates are in flight together; the hits are placed by a second
// scan and kept in LDS (kRestHits entries), so that after one reservation
// they are written out.  A list longer than that is found again in a second
// pass that writes it directly.  Returns [start, end) ([0, 0) for none).
// s_red: NT / 64 + 1 words of LDS; s_buf: kRestHits + NT * kRestItems words.
constexpr uint32_t kRestHits = 4096;
constexpr int kRestItems = 16;

template <typename T, int NT>
__device__ uint2 collect_rest(const FrontCollect& fc, uint32_t vi, uint32_t front16,
                              const Rec<T>* __restrict__ recs, const ViewDev& v, int tx, int ty,
                              uint32_t* __restrict__ values, uint32_t* s_red, uint32_t* s_buf) {
  constexpr int kItems = kRestItems;
  constexpr uint32_t kStep = uint32_t(NT) * kItems;
  uint32_t* s_hits = s_buf;
  uint32_t* s_cand = s_buf + kRestHits;
  const uint32_t nvis = uint32_t(fc.totals[2 * vi]);
  const uint32_t r0 = front_cut(nvis, front16);
  const size_t row = size_t(vi) * fc.n_pad;
  const Rect16* __restrict__ sr = fc.srect + row;
  const uint32_t* __restrict__ ord = fc.order + row;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // workgroup exclusive scan of one count per thread; *all: the sum
  auto scan = [&](uint32_t c, uint32_t* all) -> uint32_t {
    uint32_t inc = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) s_red[wave] = inc;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      const uint32_t t = s_red[w];
      before += w < wave ? t : 0u;
      sum += t;
    }
    __syncthreads();
    *all = sum;
    return before + inc - c;
  };
  auto covers = [&](const Rect16& r) {
    return tx >= int(r.x0) && tx < int(r.x1) && ty >= int(r.y0) && ty < int(r.y1);
  };
  // one pass over the positions; out(p, gi) receives hit number p
  auto pass = [&](auto&& out) -> uint32_t {
    uint32_t total = 0;
    Rect16 rr[kItems];
    auto load = [&](uint32_t k0) {
      const uint32_t kt = k0 + uint32_t(threadIdx.x) * kItems;
#pragma unroll
      for (int i = 0; i < kItems; ++i)
        rr[i] = kt + i < nvis ? sr[kt + i] : Rect16{0, 0, 0, 0};
    };
    load(r0);
#pragma unroll 1
    for (uint32_t k0 = r0; k0 < nvis; k0 += kStep) {
      const uint32_t kt = k0 + uint32_t(threadIdx.x) * kItems;
      uint32_t bm = 0;
#pragma unroll
      for (int i = 0; i < kItems; ++i) bm |= covers(rr[i]) ? 1u << i : 0u;
      if (k0 + kStep < nvis) load(k0 + kStep);
      uint32_t nc;
      uint32_t c = scan(uint32_t(__popc(bm)), &nc);
#pragma unroll
      for (int i = 0; i < kItems; ++i)
        if ((bm >> i) & 1u) s_cand[c++] = kt + uint32_t(i);
      __syncthreads();
      // (the scans' barriers keep the next step's writes of s_cand behind these reads)
#pragma unroll 1
      for (uint32_t b = 0; b < nc; b += NT) {
        const uint32_t ci = b + threadIdx.x;
        bool hit = false;
        uint32_t gi = 0;
        if (ci < nc) {
          const uint32_t k = s_cand[ci];
          gi = ord[k];
          int x0, x1;
          row_span(geom_of(recs[gi], sr[k], v), ty, x0, x1);
          hit = tx >= x0 && tx < x1;
        }
        uint32_t nh;
        const uint32_t p = total + scan(hit ? 1u : 0u, &nh);
        if (hit) out(p, gi);
        total += nh;
      }
    }
    return total;
  };
  const uint32_t total = pass([&](uint32_t p, uint32_t gi) {
    if (p < kRestHits) s_hits[p] = gi;
  });
  if (total == 0u) return make_uint2(0u, 0u);
  if (threadIdx.x == 0) {
    const uint32_t take = (total + kSegment - 1) / kSegment * kSegment;
    uint32_t a = fc.table->app_base[vi] + atomicAdd(&fc.table->cursor[vi], take);
    if (uint64_t(a) + total > uint64_t(fc.table->app_end[vi])) {
      atomicOr(fc.overflow, 1u);
      a = 0xffffffffu;
    } else {
      atomicAdd(&fc.table->rest_tiles[vi], 1u);
    }
    s_red[NT / 64] = a;
  }
  __syncthreads();
  const uint32_t a = s_red[NT / 64];
  if (a == 0xffffffffu) return make_uint2(0u, 0u);
  if (total <= kRestHits)
    for (uint32_t j = threadIdx.x; j < total; j += NT) values[a + j] = s_hits[j];
  else
    pass([&](uint32_t p, uint32_t gi) { values[a + p] = gi; });
  // the workgroup reads these entries next
  __threadfence_block();
  __syncthreads();
  return make_uint2(a, a + total);
}

// Forward.  A pixel that has stopped keeps its final transmittance in Tf and
// continues with T = 0, which makes every later contribution zero and every later
// transmittance test fail, so no per-pixel "done" flag is carried through the
// loop.  COUNT counts, per pixel, the entries evaluated and the entries
// blended, stored as a pair in n_eval (measurement builds only).  cut: the
// tile holds a front list (front.hpp).  If its pixels outlast it, the main
// pass (REST false) queues the tile and leaves it; the rest pass (REST true)
// renders a queued tile from the start, collecting the rest of its list when
// the front list runs out.
template <typename T, int TS, int PPT, bool COUNT, bool FLOW, bool REST>
__device__ __forceinline__ void raster_fwd_tile(
    Staged<T>* s_rec, uint32_t* s_walk, uint32_t* s_red, uint32_t* s_hits,
    const Rec<T>* __restrict__ recs,
    const Vec2<T>* __restrict__ flows, uint32_t* __restrict__ values, const uint2 rg, bool cut,
    const FrontCollect& fc, uint32_t vi, uint32_t front16, uint32_t tile_end, int tile,
    uint32_t gtile, const ViewDev& v, const SettingsDev& st, T* __restrict__ image,
    T* __restrict__ flow_image, T* __restrict__ T_final, uint32_t* __restrict__ n_contrib,
    uint32_t* __restrict__ n_eval, Ck<T>* __restrict__ ck, Vec2<T>* __restrict__ ckf,
    T* __restrict__ img_copy, T* __restrict__ flow_copy, uint32_t* __restrict__ walk,
    uint2* __restrict__ rest_out) {
  using Cfg = TileCfg<TS, PPT>;
  constexpr int NT = Cfg::kThreads;
  constexpr int NB = Cfg::kBatch;
  static_assert(kSegment % NB == 0, "segment boundaries must fall on batch boundaries");
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int x = tx * TS + int(threadIdx.x % TS);
  const int y0 = ty * TS + int(threadIdx.x / TS);
  const T px = T(x) + T(0.5);
  const T e_min = T(kHalfLog2e) * T(st.ext2);
  const T amin = T(st.alpha_min), amax = T(st.alpha_max), tmin = T(st.T_min);
  T py[PPT], Tr[PPT], c0[PPT], c1[PPT], c2[PPT], c3[PPT], c4[PPT];
  uint32_t last[PPT], evals[PPT], blends[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int y = y0 + k * Cfg::kRowStep;
    py[k] = T(y) + T(0.5);
    // pixels outside the image start finished
    Tr[k] = (x < v.W && y < v.H) ? T(1) : T(0);
    c0[k] = c1[k] = c2[k] = c3[k] = c4[k] = T(0);
    last[k] = evals[k] = blends[k] = 0u;
  }
  if (threadIdx.x == 0) *s_walk = 0u;
  // list positions [0, len): the front (or whole) list, then the rest once collected
  uint2 rest = make_uint2(0u, 0u);
  uint32_t len = rg.y - rg.x;
  bool pending = cut;
  for (uint32_t jbase = 0;; jbase += NB) {
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PPT; ++k) lane_done &= !(Tr[k] > T(0));
    if (__syncthreads_count(lane_done) == NT) break;
    if (pending && jbase + NB >= len) {
      // the front list ends in this batch (or at its end) with pixels still
      // running
      if (!REST) {
        if (threadIdx.x == 0) fc.queue[atomicAdd(&fc.table->queued, 1u)] = gtile;
        return;
      }
      // collect the rest before the batch, so that the boundary state below is
      // saved wherever the list goes on
      rest = collect_rest<T, NT>(fc, vi, front16, recs, v, tile % v.tiles_x, tile / v.tiles_x,
                                 values, s_red, s_hits);
      len += rest.y - rest.x;
      pending = false;
      if (threadIdx.x == 0 && rest.y > rest.x) rest_out[gtile] = rest;
    }
    if (jbase >= len) break;
    const uint32_t i = jbase + threadIdx.x;
    if (threadIdx.x < NB && i < len) {
      const uint32_t idx = values[list_pos(rg, rest, i)];
      Staged<T> sr = stage(recs[idx], e_min, amin);
      if (FLOW) {
        const Vec2<T> fl = flows[idx];
        sr.fu = fl.x;
        sr.fv = fl.y;
      }
      s_rec[threadIdx.x] = sr;
    }
    __syncthreads();
    const int nb = int(len - jbase < uint32_t(NB) ? len - jbase : uint32_t(NB));
    if (__ballot(!lane_done)) {
#pragma unroll 2
      for (int j = 0; j < nb; ++j) {
        const Staged<T> r = s_rec[j];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          T ux, uy, G, a_raw, alpha;
          const bool pass = eval_pair(r, px, py[k], amax, ux, uy, G, a_raw, alpha);
          const T wa = alpha * Tr[k];            // the weight, if blended
          const T Tn = tfma(-alpha, Tr[k], Tr[k]);  // T (1 - alpha)
          if (COUNT) evals[k] += Tr[k] > T(0) ? 1u : 0u;
          const bool blend = pass & (Tn >= tmin);
          if (COUNT) blends[k] += blend ? 1u : 0u;
          // The first Gaussian that would take T below T_min stops the pixel,
          // which keeps its final transmittance negated from then on (a
          // finished pixel has Tr <= 0, so nothing blends or stops it again):
          // a pair that passes but does not blend stops a running pixel.
          const bool run = pass & (Tr[k] > T(0));
          const T w = blend ? wa : T(0);
          c0[k] = tfma(r.r, w, c0[k]);
          c1[k] = tfma(r.g, w, c1[k]);
          c2[k] = tfma(r.b, w, c2[k]);
          if (FLOW) {
            c3[k] = tfma(r.fu, w, c3[k]);
            c4[k] = tfma(r.fv, w, c4[k]);
          }
          Tr[k] = blend ? Tn : (run ? -Tr[k] : Tr[k]);
          last[k] = blend ? jbase + uint32_t(j) + 1u : last[k];
        }
      }
    }
    // state after the first m segments of the list, for the backward's
    // independent segment walks (only where the list goes on)
    const uint32_t done_n = jbase + uint32_t(NB);
    if (done_n % kSegment == 0u && done_n < len) {
      const size_t slot =
          size_t(boundary_slot(rg, rest, gtile, tile_end, done_n / kSegment)) * (TS * TS);
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int pt = (int(threadIdx.x / TS) + k * Cfg::kRowStep) * TS + int(threadIdx.x % TS);
        ck[slot + pt] = Ck<T>{Tr[k], c0[k], c1[k], c2[k]};
        if (FLOW) ckf[slot + pt] = Vec2<T>{c3[k], c4[k]};
      }
    }
  }
  const long hw = long(v.H) * v.W;
  uint32_t lane_walk = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int y = y0 + k * Cfg::kRowStep;
    if (x < v.W && y < v.H) {
      const long pix = long(y) * v.W + x;
      const T Tfin = Tr[k] > T(0) ? Tr[k] : -Tr[k];
      const T o0 = tfma(Tfin, T(v.bg[0]), c0[k]);
      const T o1 = tfma(Tfin, T(v.bg[1]), c1[k]);
      const T o2 = tfma(Tfin, T(v.bg[2]), c2[k]);
      image[pix] = o0;
      image[hw + pix] = o1;
      image[2 * hw + pix] = o2;
      img_copy[pix] = o0;
      img_copy[hw + pix] = o1;
      img_copy[2 * hw + pix] = o2;
      if (FLOW) {
        flow_image[pix] = c3[k];
        flow_image[hw + pix] = c4[k];
        flow_copy[pix] = c3[k];
        flow_copy[hw + pix] = c4[k];
      }
      T_final[pix] = Tfin;
      n_contrib[pix] = last[k];
      if (COUNT) {
        n_eval[2 * pix] = evals[k];
        n_eval[2 * pix + 1] = blends[k];
      }
      lane_walk = last[k] > lane_walk ? last[k] : lane_walk;
    }
  }
  // the tile's backward walk: up to its furthest last contributor
  if (lane_walk) atomicMax(s_walk, lane_walk);
  __syncthreads();
  if (threadIdx.x == 0) walk[gtile] = *s_walk;
}

// Screen-space gradient components per Gaussian: 9, and 2 more (flow) for a
// flow render.
template <bool FLOW>
constexpr int kComps = FLOW ? 11 : 9;

template <typename T, int TS, int PPT, bool FLOW>
struct BwdShared {
  Staged<T> rec[TileCfg<TS, PPT>::kBatch];
  uint32_t idx[TileCfg<TS, PPT>::kBatch];
  // per batch slot and component
  T grad[TileCfg<TS, PPT>::kBatch][kComps<FLOW>];
  uint32_t max;
};

template <typename T, int TS, int PPT, bool FLOW>
__device__ __forceinline__ void raster_bwd_tile(
    BwdShared<T, TS, PPT, FLOW>& sh, const Rec<T>* __restrict__ recs,
    const Vec2<T>* __restrict__ flows, const uint32_t* __restrict__ values, const uint2 rg,
    const uint2 rest, uint32_t tile_end, int tile, uint32_t gtile, uint32_t seg, uint32_t walk,
    const ViewDev& v,
    const SettingsDev& st, const T* __restrict__ T_final, const uint32_t* __restrict__ n_contrib,
    const T* __restrict__ img_copy, const T* __restrict__ flow_copy,
    const Ck<T>* __restrict__ ck, const Vec2<T>* __restrict__ ckf,
    const T* __restrict__ dL_dimage, const T* __restrict__ dL_dflow, double* __restrict__ grad2d) {
  using Cfg = TileCfg<TS, PPT>;
  constexpr int NT = Cfg::kThreads;
  constexpr int NB = Cfg::kBatch;
  constexpr int NC = kComps<FLOW>;
  Staged<T>* s_rec = sh.rec;
  uint32_t* s_idx = sh.idx;
  T(*s_grad)[NC] = sh.grad;
  uint32_t& s_max = sh.max;
  const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
  const int x = tx * TS + int(threadIdx.x % TS);
  const int y0 = ty * TS + int(threadIdx.x / TS);
  const T px = T(x) + T(0.5);
  const T e_min = T(kHalfLog2e) * T(st.ext2);
  const T amin = T(st.alpha_min), amax = T(st.alpha_max);
  const long hw = long(v.H) * v.W;
  // this walk covers list positions [lo, hi) (segment `seg`, back to front)
  const uint32_t lo = seg * kSegment;
  const uint32_t seg_end = lo + kSegment;
  const uint32_t hi = walk < seg_end ? walk : seg_end;
  const size_t cslot = size_t(boundary_slot(rg, rest, gtile, tile_end, seg + 1)) * (TS * TS);
  // Per pixel: the upstream gradients g (colour, then flow) and gacc = g . (colour
  // accumulated behind the current Gaussian, background included).  Only that
  // dot product enters dL/da, and g is fixed per pixel, so one running sum
  // gacc += w (g . c) stands for the per-channel accumulators.
  T py[PPT], Tcur[PPT], g0[PPT], g1[PPT], g2[PPT], gacc[PPT];
  T g3[PPT], g4[PPT];  // flow channels
  uint32_t ncon[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int y = y0 + k * Cfg::kRowStep;
    py[k] = T(y) + T(0.5);
    Tcur[k] = T(1);
    g0[k] = g1[k] = g2[k] = g3[k] = g4[k] = T(0);
    ncon[k] = 0u;
    gacc[k] = T(0);
    if (x < v.W && y < v.H) {
      const long pix = long(y) * v.W + x;
      ncon[k] = n_contrib[pix];
      g0[k] = dL_dimage[pix];
      g1[k] = dL_dimage[hw + pix];
      g2[k] = dL_dimage[2 * hw + pix];
      if (FLOW) {
        g3[k] = dL_dflow[pix];
        g4[k] = dL_dflow[hw + pix];
      }
      if (ncon[k] > seg_end) {
        // the pixel goes on past this segment: start from the forward's state
        // at the segment's end; colour behind = final colour - colour in front
        const int pt = (int(threadIdx.x / TS) + k * Cfg::kRowStep) * TS + int(threadIdx.x % TS);
        const Ck<T> c = ck[cslot + pt];
        Tcur[k] = c.t;
        gacc[k] = tfma(g0[k], img_copy[pix] - c.r,
                       tfma(g1[k], img_copy[hw + pix] - c.g, g2[k] * (img_copy[2 * hw + pix] - c.b)));
        if (FLOW) {
          const Vec2<T> cf = ckf[cslot + pt];
          gacc[k] = tfma(g3[k], flow_copy[pix] - cf.x, tfma(g4[k], flow_copy[hw + pix] - cf.y, gacc[k]));
        }
      } else {
        // behind the last contributor: the background seen through T_final
        // (the flow's background is 0)
        Tcur[k] = T_final[pix];
        gacc[k] = Tcur[k] * tfma(g0[k], T(v.bg[0]), tfma(g1[k], T(v.bg[1]), g2[k] * T(v.bg[2])));
      }
    }
  }
  (void)s_max;
  const int lane = threadIdx.x & 63;
  for (uint32_t bend = hi; bend > lo;) {
    const uint32_t bstart = bend > lo + uint32_t(NB) ? bend - NB : lo;
    const int nb = int(bend - bstart);
    if (threadIdx.x < NB) {
      if (int(threadIdx.x) < nb) {
        const uint32_t idx = values[list_pos(rg, rest, bstart + threadIdx.x)];
        s_idx[threadIdx.x] = idx;
        Staged<T> sr = stage(recs[idx], e_min, amin);
        if (FLOW) {
          const Vec2<T> fl = flows[idx];
          sr.fu = fl.x;
          sr.fv = fl.y;
        }
        s_rec[threadIdx.x] = sr;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) s_grad[threadIdx.x][c] = T(0);
    }
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const Staged<T> r = s_rec[j];
      // pass 1: which of this lane's pixels blended the Gaussian
      T ux[PPT], uy[PPT], G[PPT], a_raw[PPT], alpha[PPT];
      bool use[PPT], band[PPT];
      bool any = false;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const bool pass = eval_pair(r, px, py[k], amax, ux[k], uy[k], G[k], a_raw[k], alpha[k]);
        const bool in_front = bstart + uint32_t(j) < ncon[k];
        use[k] = pass & in_front;
        // some pixel of the wavefront's band k blended it (the two masks are
        // taken apart, so that each is the comparison's own lane mask)
        band[k] = (__builtin_amdgcn_ballot_w64(pass) & __builtin_amdgcn_ballot_w64(in_front)) != 0ull;
        any |= band[k];
      }
      if (!any) continue;  // no pixel of the wavefront blended it
      // pass 2: per-pixel derivatives, summed over the lane's pixels as
      // s0..s4 = sum g (ux, uy, ux^2, ux uy, uy^2) with g = a dL/da (the
      // screen-space mean and Sigma_2D gradients are linear in these), s5 = sum
      // dL/da exp(-q/2), s6..s8 = sum a T dL/dC (s9, s10 the same for the flow)
      T sv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) sv[c] = T(0);
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        // (a band where no pixel blended it leaves every sum and state unchanged)
        if (!band[k]) continue;
        const T inv_om = fast_rcp(T(1) - alpha[k]);
        const T Ti = Tcur[k] * inv_om;  // transmittance in front of this Gaussian
        const T w = use[k] ? alpha[k] * Ti : T(0);
        // dC/da = T c - (colour behind) / (1 - a), dotted with g
        T gc = tfma(g0[k], r.r, tfma(g1[k], r.g, g2[k] * r.b));
        if (FLOW) gc = tfma(g3[k], r.fu, tfma(g4[k], r.fv, gc));
        // no gradient through the alpha clamp
        const T dL_da =
            (use[k] & (a_raw[k] < amax)) ? inv_om * (Tcur[k] * gc - gacc[k]) : T(0);
        gacc[k] = tfma(gc, w, gacc[k]);
        Tcur[k] = use[k] ? Ti : Tcur[k];
        const T ga = dL_da * a_raw[k];
        const T gx = ga * ux[k], gy = ga * uy[k];
        sv[0] += gx;
        sv[1] += gy;
        sv[2] = tfma(gx, ux[k], sv[2]);
        sv[3] = tfma(gx, uy[k], sv[3]);
        sv[4] = tfma(gy, uy[k], sv[4]);
        sv[5] = tfma(dL_da, G[k], sv[5]);
        sv[6] = tfma(w, g0[k], sv[6]);
        sv[7] = tfma(w, g1[k], sv[7]);
        sv[8] = tfma(w, g2[k], sv[8]);
        if (FLOW) {
          sv[9] = tfma(w, g3[k], sv[9]);
          sv[10] = tfma(w, g4[k], sv[10]);
        }
      }
      // sums over the wavefront, kept in LDS (the components' scale factors
      // are applied when the batch is flushed); with several wavefronts per
      // tile the sums of all of them add up
      store_wave_sums<NC, NT>(sv, s_grad[j], lane);
    }
    __syncthreads();
    // One global atomic per (tile, Gaussian, component); the sum over tiles is
    // kept in double because its terms have mixed signs and can cancel.
    // With u = Q d (the staged value is k u): a = o exp(-q/2) gives dL/dq =
    // -g / 2 per pixel, dq/dmean2d = 2 u, and, since dq = -u^T dSigma_2D u for
    // Sigma_2D = Q^-1, dL/dSigma_2D = sum g u u^T / 2; so the components are
    // d/d mean2d = -s0,1 / k, d/d Sigma_2D (0,0), (0,1) = (1,0), (1,1) =
    // s2,3,4 / (2 k^2), d/d opacity_t = s5, d/d rgb = s6,7,8 (d/d flow = s9,10).
    // grad2d is Gaussian-major, so the lanes of one instruction cover a few
    // Gaussians' components in a few cache lines rather than one line each.
    for (int e = threadIdx.x; e < NC * nb; e += NT) {
      const int j = e / NC, c = e % NC;
      const T scale = c < 2 ? T(-1.0 / kHalfLog2e)
                            : (c < 5 ? T(0.5 / (kHalfLog2e * kHalfLog2e)) : T(1));
      const T val = s_grad[j][c] * scale;
      if (val != T(0)) atomic_add_nr(&grad2d[size_t(s_idx[j]) * NC + c], double(val));
    }
    __syncthreads();
    bend = bstart;
  }
}

// Render holding global tile g: the last slot whose first tile is <= g.
__device__ __forceinline__ int slot_of_tile(const ViewSlot* __restrict__ slots, int n_views,
                                            uint32_t g) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (slots[mid].tile_base <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Persistent launches: each workgroup starts on tile blockIdx.x and then takes
// further tiles (of any render) from a counter until none is left, so renders
// of uneven size share one launch and a workgroup that drew short lists simply
// takes more tiles.  (The first tile comes from the launch itself: a counter
// taken by every workgroup at once would serialise the start.)
template <typename T, int TS, int PPT, bool COUNT, bool FLOW>
__global__ __launch_bounds__(TS* TS / PPT) void raster_fwd_kernel(
    const Rec<T>* __restrict__ recs, const Vec2<T>* __restrict__ flows, uint32_t n,
    uint32_t* __restrict__ values, const uint2* __restrict__ ranges, FrontCollect fc,
    const ViewSlot* __restrict__ slots, int n_views, uint32_t total_tiles, SettingsDev st,
    T* __restrict__ image, T* __restrict__ flow_image, T* __restrict__ T_final,
    uint32_t* __restrict__ n_contrib, uint32_t* __restrict__ n_eval, RasterSaved<T> sv,
    uint32_t* __restrict__ tickets) {
  constexpr int NT = TS * TS / PPT;
  __shared__ Staged<T> s_rec[TileCfg<TS, PPT>::kBatch];
  __shared__ uint32_t s_ticket, s_walk;
  for (uint32_t g = blockIdx.x; g < total_tiles;) {
    const int vi = slot_of_tile(slots, n_views, g);
    const ViewSlot& sl = slots[vi];
    const ViewDev v = sl.v;
    const size_t pb = size_t(sl.pix_base);
    const int tile = int(g - sl.tile_base);
    const uint32_t front16 = sl.front16;
    // a front list: the render has a depth cut and the tile is not kept whole
    bool cut = false;
    if (fc.keep && front16) {
      const uint32_t nvis = uint32_t(fc.totals[2 * vi]);
      if (front_cut(nvis, front16) < nvis)
        cut = !tile_kept(fc.keep + sl.keep_base + size_t(tile / v.tiles_x) * keep_words(v.tiles_x),
                         tile % v.tiles_x);
    }
    const uint32_t tile_end = sl.tile_base + uint32_t(v.tiles_x) * uint32_t(v.tiles_y);
    raster_fwd_tile<T, TS, PPT, COUNT, FLOW, false>(
        s_rec, &s_walk, nullptr, nullptr, recs + size_t(vi) * n,
        FLOW ? flows + size_t(vi) * n : nullptr,
        values, ranges[g], cut, fc, uint32_t(vi), front16, tile_end, tile, g, v, st,
        image + 3 * pb, FLOW ? flow_image + 2 * pb : nullptr, T_final + pb, n_contrib + pb,
        COUNT ? n_eval + 2 * pb : nullptr, sv.ck, sv.ckf, sv.img + 3 * pb,
        FLOW ? sv.flow + 2 * pb : nullptr, sv.walk, sv.rest);
    if (threadIdx.x == 0) s_ticket = gridDim.x + atomicAdd(tickets, 1u);
    __syncthreads();
    g = s_ticket;
    __syncthreads();
  }
}

// The rest pass of the front lists (front.hpp): the tiles the main pass
// queued (their pixels outlasted their front lists), each rendered again from
// the start with its rest collected, by a persistent grid of kRestGroups
// workgroups; with nothing queued every workgroup returns at once.
template <typename T, int TS, int PPT, bool COUNT, bool FLOW>
__global__ __launch_bounds__(TS* TS / PPT) void raster_rest_kernel(
    const Rec<T>* __restrict__ recs, const Vec2<T>* __restrict__ flows, uint32_t n,
    uint32_t* __restrict__ values, const uint2* __restrict__ ranges, FrontCollect fc,
    const ViewSlot* __restrict__ slots, int n_views, SettingsDev st, T* __restrict__ image,
    T* __restrict__ flow_image, T* __restrict__ T_final, uint32_t* __restrict__ n_contrib,
    uint32_t* __restrict__ n_eval, RasterSaved<T> sv) {
  constexpr int NT = TS * TS / PPT;
  __shared__ Staged<T> s_rec[TileCfg<TS, PPT>::kBatch];
  __shared__ uint32_t s_walk;
  __shared__ uint32_t s_red[NT / 64 + 1];
  __shared__ uint32_t s_hits[kRestHits + NT * kRestItems];
  const uint32_t count = fc.table->queued;
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t g = fc.queue[it];
    const int vi = slot_of_tile(slots, n_views, g);
    const ViewSlot& sl = slots[vi];
    const ViewDev v = sl.v;
    const size_t pb = size_t(sl.pix_base);
    const uint32_t tile_end = sl.tile_base + uint32_t(v.tiles_x) * uint32_t(v.tiles_y);
    raster_fwd_tile<T, TS, PPT, COUNT, FLOW, true>(
        s_rec, &s_walk, s_red, s_hits, recs + size_t(vi) * n,
        FLOW ? flows + size_t(vi) * n : nullptr,
        values, ranges[g], true, fc, uint32_t(vi), sl.front16, tile_end, int(g - sl.tile_base), g,
        v, st, image + 3 * pb, FLOW ? flow_image + 2 * pb : nullptr, T_final + pb,
        n_contrib + pb, COUNT ? n_eval + 2 * pb : nullptr, sv.ck, sv.ckf, sv.img + 3 * pb,
        FLOW ? sv.flow + 2 * pb : nullptr, sv.walk, sv.rest);
    __syncthreads();
  }
}

// Workgroups of the rest pass: enough for the queued tiles of a render to run
// at once (four per CU fit in LDS), since each is one of the longest walks.
constexpr uint32_t kRestGroups = 1024;

// Length classes of the tiles' last segments (seg_queue_kernel) and where the
// queue lengths sit in the backward's ticket words.
constexpr uint32_t kLenBuckets = 8;
constexpr int kQueueCounts = 8;

// Backward work items are (tile, segment) pairs, so the segments of one long
// list run in parallel; they are taken from the queues of seg_queue_kernel in
// queue order (q_count: the nine queue lengths).
template <typename T, int TS, int PPT, bool FLOW>
__global__ __launch_bounds__(TS* TS / PPT) void raster_bwd_kernel(
    const Rec<T>* __restrict__ recs, const Vec2<T>* __restrict__ flows, uint32_t n,
    const uint32_t* __restrict__ values, const uint2* __restrict__ ranges,
    const ViewSlot* __restrict__ slots, int n_views, SettingsDev st,
    const T* __restrict__ T_final, const uint32_t* __restrict__ n_contrib, RasterSaved<T> sv,
    const uint2* __restrict__ q_full, const uint2* __restrict__ q_last, uint32_t total_tiles,
    const T* __restrict__ dL_dimage, const T* __restrict__ dL_dflow,
    double* __restrict__ grad2d, uint32_t* __restrict__ tickets) {
  __shared__ BwdShared<T, TS, PPT, FLOW> sh;
  __shared__ uint32_t s_ticket;
  uint32_t qn[1 + kLenBuckets], total = 0;
#pragma unroll
  for (uint32_t k = 0; k <= kLenBuckets; ++k) {
    qn[k] = tickets[kQueueCounts + k];
    total += qn[k];
  }
  for (uint32_t it = blockIdx.x; it < total;) {
    uint2 item;
    if (it < qn[0]) {
      item = q_full[it];
    } else {
      // queue 1 + k holding position r (it < total, so k stays below kLenBuckets)
      uint32_t r = it - qn[0], k = 0;
#pragma unroll
      for (uint32_t b = 0; b + 1 < kLenBuckets; ++b) {
        if (k == b && r >= qn[1 + b]) {
          r -= qn[1 + b];
          k = b + 1;
        }
      }
      item = q_last[size_t(k) * total_tiles + r];
    }
    const uint32_t g = item.x;
    const uint32_t seg = item.y;
    const int vi = slot_of_tile(slots, n_views, g);
    const ViewSlot& sl = slots[vi];
    const ViewDev v = sl.v;
    const size_t pb = size_t(sl.pix_base);
    raster_bwd_tile<T, TS, PPT, FLOW>(
        sh, recs + size_t(vi) * n, FLOW ? flows + size_t(vi) * n : nullptr, values, ranges[g],
        sv.rest[g], sl.tile_base + uint32_t(v.tiles_x) * uint32_t(v.tiles_y),
        int(g - sl.tile_base), g, seg, sv.walk[g], v, st, T_final + pb, n_contrib + pb,
        sv.img + 3 * pb, FLOW ? sv.flow + 2 * pb : nullptr, sv.ck, sv.ckf, dL_dimage + 3 * pb,
        FLOW ? dL_dflow + 2 * pb : nullptr, grad2d + size_t(vi) * kComps<FLOW> * n);
    if (threadIdx.x == 0) s_ticket = gridDim.x + atomicAdd(tickets, 1u);
    __syncthreads();
    it = s_ticket;
    __syncthreads();
  }
}

// Work items of the backward: the 256-entry segments of every tile's list up
// to its furthest last contributor, as (tile, segment) pairs in nine queues:
// queue 0 holds every segment but a tile's last (all full, kSegment entries),
// queue 1 + b the tiles' last segments of length class b (longer first).  The
// backward takes queue 0, then queues 1..8, so the short items fill the end of
// its launch; the order within a queue does not matter.  One thread per tile;
// a wavefront reserves its places with one atomic per queue.  q_count: 9
// counters, zeroed by the caller; q_full: capacity >= the segments in all;
// q_last: kLenBuckets arrays of total_tiles pairs.

__device__ __forceinline__ uint32_t len_bucket(uint32_t len) {
  const uint32_t b = (kSegment - len) * kLenBuckets / kSegment;
  return b < kLenBuckets ? b : kLenBuckets - 1;
}

__global__ __launch_bounds__(256) void seg_queue_kernel(const uint32_t* __restrict__ walk,
                                                        uint32_t total_tiles,
                                                        uint32_t* __restrict__ q_count,
                                                        uint2* __restrict__ q_full,
                                                        uint2* __restrict__ q_last) {
  const int lane = threadIdx.x & 63;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  const uint32_t w = t < total_tiles ? walk[t] : 0u;
  const uint32_t cnt = (w + kSegment - 1) / kSegment;
  const uint32_t f = cnt > 0u ? cnt - 1u : 0u;
  // full segments: a wavefront scan of the counts
  const uint32_t incl = wave_incl_scan_u32(f, lane);
  const uint32_t excl = incl - f;
  const uint32_t total_w = __shfl(incl, 63, 64);
  // last segments by length class: a ballot per class, this lane's class mask
  const uint32_t cls = cnt > 0u ? len_bucket(w - f * kSegment) : kLenBuckets;
  const unsigned long long lt = (1ull << lane) - 1ull;
  unsigned long long mine = 0ull;
  uint32_t n_cls = 0;  // lane k < kLenBuckets: the wavefront's tiles of class k
#pragma unroll
  for (uint32_t k = 0; k < kLenBuckets; ++k) {
    const unsigned long long m = __ballot(cls == k);
    if (cls == k) mine = m;
    if (uint32_t(lane) == k) n_cls = uint32_t(__popcll(m));
  }
  // every reservation of the wavefront in one atomic instruction: lanes
  // 0 .. kLenBuckets-1 for the classes, lane 63 for the full segments
  uint32_t* q = nullptr;
  uint32_t amount = 0;
  if (uint32_t(lane) < kLenBuckets) {
    q = &q_count[1 + lane];
    amount = n_cls;
  } else if (lane == 63) {
    q = &q_count[0];
    amount = total_w;
  }
  uint32_t got = 0;
  if (amount) got = atomicAdd(q, amount);
  const uint32_t base = __shfl(got, 63, 64);
  const uint32_t cb = __shfl(got, int(cls < kLenBuckets ? cls : 0u), 64);
  // full segments: the wavefront writes its segments 64 at a time, each lane
  // finding the tile of its segment by a binary search over the tiles' first
  // positions
  for (uint32_t c = 0; c < total_w; c += 64) {
    const uint32_t i = c + uint32_t(lane);
    const int o = wave_upper_lane(excl, i);
    const uint32_t tile = __shfl(t, o, 64);
    const uint32_t seg = i - __shfl(excl, o, 64);
    if (i < total_w) q_full[base + i] = make_uint2(tile, seg);
  }
  if (cls < kLenBuckets)
    q_last[size_t(cls) * total_tiles + cb + uint32_t(__popcll(mine & lt))] = make_uint2(t, f);
}

int compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cus;
}

// Wavefronts per compute unit of the backward's persistent launch.
constexpr uint32_t kBwdWavesPerCu = 24;

// Workgroups resident on the whole chip at once (occupancy x compute units);
// a persistent launch needs no more.
template <typename K>
uint32_t resident_groups(K kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1 || cus < 1) {
    (void)hipGetLastError();
    return 2048u;
  }
  return uint32_t(per_cu) * uint32_t(cus);
}

// Per-view L1 gradient: blockIdx.y = view.  Each workgroup writes its share
// of the view's mean absolute difference to partials[v * gridDim.x + b].
// (Adding the shares in the last workgroup to finish instead of a second
// launch needs a device-scope release per workgroup, which writes back the
// L2 with the gradient in it: measured 38 us against 14 + 5.)
__global__ __launch_bounds__(256) void l1_grad_views_kernel(const float* __restrict__ image,
                                                            const float* __restrict__ target,
                                                            L1Views lv, float* __restrict__ grad,
                                                            float* __restrict__ partials) {
  __shared__ float s_part[4];
  const int v = blockIdx.y;
  const int64_t b0 = lv.base[v], cnt = lv.count[v];
  const float inv = 1.0f / float(cnt);
  const int64_t stride = int64_t(gridDim.x) * 256;
  auto one = [&](float d) { return d > 0.f ? inv : (d < 0.f ? -inv : 0.f); };
  float part = 0.f;
  int64_t done = 0;
  const float* im = image + b0;
  const float* tg = target + b0;
  float* gr = grad + b0;
  if (((reinterpret_cast<uintptr_t>(im) | reinterpret_cast<uintptr_t>(tg) |
        reinterpret_cast<uintptr_t>(gr)) & 15u) == 0) {
    // 16-byte accesses (four values per thread and step), the rest below
    const int64_t n4 = cnt / 4;
    const float4* im4 = reinterpret_cast<const float4*>(im);
    const float4* tg4 = reinterpret_cast<const float4*>(tg);
    float4* gr4 = reinterpret_cast<float4*>(gr);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n4; i += stride) {
      const float4 a = im4[i], t = tg4[i];
      const float4 d = make_float4(a.x - t.x, a.y - t.y, a.z - t.z, a.w - t.w);
      gr4[i] = make_float4(one(d.x), one(d.y), one(d.z), one(d.w));
      part += (fabsf(d.x) + fabsf(d.y)) + (fabsf(d.z) + fabsf(d.w));
    }
    done = n4 * 4;
  }
  for (int64_t i = done + int64_t(blockIdx.x) * 256 + threadIdx.x; i < cnt; i += stride) {
    const float d = im[i] - tg[i];
    gr[i] = one(d);
    part += fabsf(d);
  }
  if (partials) {
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0)
      partials[size_t(v) * gridDim.x + blockIdx.x] =
          (s_part[0] + s_part[1] + s_part[2] + s_part[3]) * inv;
  }
}

// *loss = sum of partials[0..count) (one workgroup).
__global__ __launch_bounds__(256) void sum_partials_kernel(const float* __restrict__ partials,
                                                           uint32_t count, float* __restrict__ loss) {
  __shared__ float s_part[4];
  float part = 0.f;
  for (uint32_t i = threadIdx.x; i < count; i += 256) part += partials[i];
  part = wave_sum(part);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (s_part[0] + s_part[1]) + (s_part[2] + s_part[3]);
}

template <typename T, int TS, int PPT>
hipError_t raster_fwd_cfg(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                          uint32_t* values, const uint2* ranges, const FrontCollect& fc,
                          const ViewSlot* slots,
                          int n_views, uint32_t total_tiles, const SettingsDev& st, T* image,
                          T* flow_image, T* T_final, uint32_t* n_contrib, uint32_t* n_eval,
                          const RasterSaved<T>& sv, uint32_t* tickets, hipStream_t stream) {
  constexpr int NT = TS * TS / PPT;
  if (flows && (n_eval || !flow_image || !sv.ckf || !sv.flow)) return hipErrorInvalidValue;
  static const uint32_t cap_count =
      resident_groups(raster_fwd_kernel<T, TS, PPT, true, false>, NT);
  static const uint32_t cap_plain =
      resident_groups(raster_fwd_kernel<T, TS, PPT, false, false>, NT);
  static const uint32_t cap_flow = resident_groups(raster_fwd_kernel<T, TS, PPT, false, true>, NT);
  const uint32_t cap = flows ? cap_flow : (n_eval ? cap_count : cap_plain);
  const uint32_t grid = total_tiles < cap ? total_tiles : cap;
  if (grid == 0) return hipSuccess;
  if (flows)
    hipLaunchKernelGGL((raster_fwd_kernel<T, TS, PPT, false, true>), dim3(grid), dim3(NT), 0,
                       stream, recs, flows, n, values, ranges, fc, slots, n_views, total_tiles,
                       st, image, flow_image, T_final, n_contrib, n_eval, sv, tickets);
  else if (n_eval)
    hipLaunchKernelGGL((raster_fwd_kernel<T, TS, PPT, true, false>), dim3(grid), dim3(NT), 0,
                       stream, recs, flows, n, values, ranges, fc, slots, n_views, total_tiles,
                       st, image, flow_image, T_final, n_contrib, n_eval, sv, tickets);
  else
    hipLaunchKernelGGL((raster_fwd_kernel<T, TS, PPT, false, false>), dim3(grid), dim3(NT), 0,
                       stream, recs, flows, n, values, ranges, fc, slots, n_views, total_tiles,
                       st, image, flow_image, T_final, n_contrib, n_eval, sv, tickets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fc.keep) return e;
  const dim3 rgrid(total_tiles < kRestGroups ? total_tiles : kRestGroups);
  if (flows)
    hipLaunchKernelGGL((raster_rest_kernel<T, TS, PPT, false, true>), rgrid, dim3(NT), 0, stream,
                       recs, flows, n, values, ranges, fc, slots, n_views, st, image, flow_image,
                       T_final, n_contrib, n_eval, sv);
  else if (n_eval)
    hipLaunchKernelGGL((raster_rest_kernel<T, TS, PPT, true, false>), rgrid, dim3(NT), 0, stream,
                       recs, flows, n, values, ranges, fc, slots, n_views, st, image, flow_image,
                       T_final, n_contrib, n_eval, sv);
  else
    hipLaunchKernelGGL((raster_rest_kernel<T, TS, PPT, false, false>), rgrid, dim3(NT), 0,
                       stream, recs, flows, n, values, ranges, fc, slots, n_views, st, image,
                       flow_image, T_final, n_contrib, n_eval, sv);
  return hipGetLastError();
}

template <typename T, int TS, int PPT>
hipError_t raster_bwd_cfg(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                          const uint32_t* values, const uint2* ranges, const ViewSlot* slots,
                          int n_views, uint32_t total_tiles, uint64_t max_items,
                          const SettingsDev& st, const T* T_final, const uint32_t* n_contrib,
                          const RasterSaved<T>& sv, const T* dL_dimage, const T* dL_dflow,
                          double* grad2d, uint32_t* work, hipStream_t stream) {
  constexpr int NT = TS * TS / PPT;
  if (total_tiles == 0) return hipSuccess;
  // work: [tickets and queue counts (64 words, zeroed by the caller) | full-segment
  //        queue (max_items pairs) | last-segment queues (kLenBuckets x tiles pairs)]
  uint32_t* tickets = work;
  uint2* q_full = reinterpret_cast<uint2*>(work + 64);
  uint2* q_last = q_full + max_items;
  hipLaunchKernelGGL(seg_queue_kernel, dim3((total_tiles + 255) / 256), dim3(256), 0, stream,
                     sv.walk, total_tiles, tickets + kQueueCounts, q_full, q_last);
  const bool flow = dL_dflow != nullptr;
  if (flow && (!flows || !sv.ckf || !sv.flow)) return hipErrorInvalidValue;
  static const uint32_t cap_plain = resident_groups(raster_bwd_kernel<T, TS, PPT, false>, NT);
  static const uint32_t cap_flow = resident_groups(raster_bwd_kernel<T, TS, PPT, true>, NT);
  // fewer workgroups than fit, so that the queue has items left to balance
  static const uint32_t limit = uint32_t(compute_units()) * (kBwdWavesPerCu * 64u / NT);
  uint32_t cap = flow ? cap_flow : cap_plain;
  if (limit > 0 && limit < cap) cap = limit;
  const uint32_t grid = uint32_t(max_items < cap ? max_items : cap);
  if (grid == 0) return hipSuccess;
  if (flow)
    hipLaunchKernelGGL((raster_bwd_kernel<T, TS, PPT, true>), dim3(grid), dim3(NT), 0, stream,
                       recs, flows, n, values, ranges, slots, n_views, st, T_final, n_contrib, sv,
                       q_full, q_last, total_tiles, dL_dimage, dL_dflow, grad2d, tickets);
  else
    hipLaunchKernelGGL((raster_bwd_kernel<T, TS, PPT, false>), dim3(grid), dim3(NT), 0, stream,
                       recs, flows, n, values, ranges, slots, n_views, st, T_final, n_contrib, sv,
                       q_full, q_last, total_tiles, dL_dimage, dL_dflow, grad2d, tickets);
  return hipGetLastError();
}

}  // namespace

size_t raster_bwd_work_bytes(uint32_t total_tiles, uint64_t max_items) {
  return 64 * 4 + (size_t(max_items) + size_t(kLenBuckets) * total_tiles) * 8;
}

bool raster_config_supported(int tile_size, int ppt) {
  switch (tile_size) {
    case 8: return ppt == 1;
    case 16: return ppt == 1 || ppt == 2 || ppt == 4;
    case 32: return ppt == 1 || ppt == 2 || ppt == 4;
    default: return false;
  }
}

// Measured on the 500k / 1352x1014 workload: the forward is fastest with one
// pixel per lane (more lanes hide the LDS and exp latency), the backward with
// four (fewer wavefront reductions per pixel).
int raster_default_ppt(int tile_size, bool backward) {
  return (backward && tile_size >= 16) ? 4 : 1;
}

#define R4D_RASTER_DISPATCH(FN, ...)                   \
  switch (tile_size * 8 + ppt) {                       \
    case 8 * 8 + 1: return FN<T, 8, 1>(__VA_ARGS__);   \
    case 16 * 8 + 1: return FN<T, 16, 1>(__VA_ARGS__); \
    case 16 * 8 + 2: return FN<T, 16, 2>(__VA_ARGS__); \
    case 16 * 8 + 4: return FN<T, 16, 4>(__VA_ARGS__); \
    case 32 * 8 + 1: return FN<T, 32, 1>(__VA_ARGS__); \
    case 32 * 8 + 2: return FN<T, 32, 2>(__VA_ARGS__); \
    case 32 * 8 + 4: return FN<T, 32, 4>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;              \
  }

template <typename T>
hipError_t launch_raster_fwd(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                             uint32_t* values, const uint2* ranges, const FrontCollect& fc,
                             const ViewSlot* slots, int n_views, uint32_t total_tiles,
                             int tile_size, const SettingsDev& st, int ppt, T* image,
                             T* flow_image, T* T_final, uint32_t* n_contrib, uint32_t* n_eval,
                             const RasterSaved<T>& sv, uint32_t* tickets, hipStream_t stream) {
  R4D_RASTER_DISPATCH(raster_fwd_cfg, recs, flows, n, values, ranges, fc, slots, n_views,
                      total_tiles, st, image, flow_image, T_final, n_contrib, n_eval, sv, tickets,
                      stream)
}

template <typename T>
hipError_t launch_raster_bwd(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                             const uint32_t* values, const uint2* ranges, const ViewSlot* slots,
                             int n_views, uint32_t total_tiles, uint64_t max_items,
                             int tile_size, const SettingsDev& st, int ppt, const T* T_final,
                             const uint32_t* n_contrib, const RasterSaved<T>& sv,
                             const T* dL_dimage, const T* dL_dflow, double* grad2d,
                             uint32_t* work, hipStream_t stream) {
  R4D_RASTER_DISPATCH(raster_bwd_cfg, recs, flows, n, values, ranges, slots, n_views,
                      total_tiles, max_items, st, T_final, n_contrib, sv, dL_dimage, dL_dflow,
                      grad2d, work, stream)
}

#undef R4D_RASTER_DISPATCH

namespace {
constexpr int64_t kL1MaxBlocks = 1024;  // workgroups per view
}  // namespace

size_t l1_partials_floats() { return size_t(kMaxViews) * kL1MaxBlocks; }

hipError_t launch_l1_grad_views(const float* images, const float* targets, const L1Views& lv,
                                float* grad, float* loss, float* partials, hipStream_t stream) {
  int64_t most = 0;
  for (int v = 0; v < lv.n_views; ++v) most = lv.count[v] > most ? lv.count[v] : most;
  if (most == 0 || lv.n_views <= 0 || lv.n_views > kMaxViews) return hipSuccess;
  // about 8 elements per thread, at most kL1MaxBlocks workgroups per view
  int64_t blocks = (most + 2047) / 2048;
  if (blocks > kL1MaxBlocks) blocks = kL1MaxBlocks;
  hipLaunchKernelGGL(l1_grad_views_kernel, dim3(uint32_t(blocks), uint32_t(lv.n_views)), dim3(256),
                     0, stream, images, targets, lv, grad, loss ? partials : nullptr);
  if (loss)
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, stream, partials,
                       uint32_t(blocks * lv.n_views), loss);
  return hipGetLastError();
}

hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, float* grad,
                          float* loss, float* partials, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  L1Views lv;
  lv.n_views = 1;
  lv.base[0] = 0;
  lv.base[1] = count;
  lv.count[0] = count;
  return launch_l1_grad_views(image, target, lv, grad, loss, partials, stream);
}

#define R4D_INST(T)                                                                          \
  template hipError_t launch_raster_fwd<T>(const Rec<T>*, const Vec2<T>*, uint32_t,           \
                                           uint32_t*, const uint2*, const FrontCollect&,      \
                                           const ViewSlot*, int, uint32_t, int,               \
                                           const SettingsDev&, int, T*, T*, T*, uint32_t*,    \
                                           uint32_t*, const RasterSaved<T>&, uint32_t*,       \
                                           hipStream_t);                                      \
  template hipError_t launch_raster_bwd<T>(const Rec<T>*, const Vec2<T>*, uint32_t,           \
                                           const uint32_t*, const uint2*, const ViewSlot*,    \
                                           int, uint32_t, uint64_t, int, const SettingsDev&,  \
                                           int, const T*, const uint32_t*,                    \
                                           const RasterSaved<T>&, const T*, const T*,         \
                                           double*, uint32_t*, hipStream_t);
R4D_INST(float)
R4D_INST(double)
#undef R4D_INST

}  // namespace r4d
