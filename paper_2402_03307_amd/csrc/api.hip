// C-ABI layer: argument checking, device memory, and the order of kernel
// launches for one render (forward) and its derivative (backward).
//
// Forward, per view:
//   preprocess (per Gaussian) -> stable radix sort by depth -> exclusive scan
//   of tile counts in depth order -> read back the entry count D -> emit tile
//   entries in depth order -> stable radix sort by tile id -> tile ranges ->
//   raster.
// Backward, per view: raster backward (screen-space gradients, atomics) ->
//   preprocess backward (chain to the parameters).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "r4d.h"
#include "r4d_internal.hpp"

using namespace r4d;

struct r4d_ctx {
  int device = 0;
  std::string last_error;
  // stage timing (measurement aid)
  bool timing = false;
  struct Pending {
    int stage;
    hipEvent_t start, stop;
  };
  std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
  std::vector<Pending> pending;
  double stage_ms[R4D_NUM_STAGES] = {};
  int64_t stage_launches[R4D_NUM_STAGES] = {};
  std::multimap<size_t, void*> free_blocks;  // size class -> block
  std::map<void*, size_t> block_size;        // every block ever allocated
  uint64_t* host_readback = nullptr;         // pinned, 2 words
  std::set<r4d_saved*> live_saved;           // saved states not yet released
};

namespace {

struct ViewSaved {
  r4d_view view;
  int tiles_x = 0, tiles_y = 0, tile_size = 0;
  uint64_t n_visible = 0, n_dup = 0;
  void* recs = nullptr;
  Rect16* rects = nullptr;
  uint32_t* depth_keys = nullptr;
  uint32_t* values = nullptr;
  uint2* ranges = nullptr;
  void* T_final = nullptr;
  uint32_t* n_contrib = nullptr;
  uint32_t* n_eval = nullptr;  // only when timing was enabled
};

}  // namespace

struct r4d_saved {
  r4d_ctx* ctx = nullptr;
  bool f64 = false;
  int n = 0, deg = 0;
  r4d_settings settings;
  std::vector<ViewSaved> views;
  std::vector<void*> blocks;
};

namespace {

r4d_status fail(r4d_ctx* ctx, r4d_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->last_error = buf;
  return s;
}

size_t size_class(size_t bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  return c;
}

// Caching allocator: blocks are never returned to the device while the
// context lives; a freed block is reused by the next request of its size class.
void* ctx_alloc(r4d_ctx* ctx, size_t bytes) {
  const size_t cls = size_class(bytes ? bytes : 1);
  auto it = ctx->free_blocks.find(cls);
  if (it != ctx->free_blocks.end()) {
    void* p = it->second;
    ctx->free_blocks.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once
    for (auto& kv : ctx->free_blocks) {
      ctx->block_size.erase(kv.second);
      (void)hipFree(kv.second);
    }
    ctx->free_blocks.clear();
    if (hipMalloc(&p, cls) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  ctx->block_size[p] = cls;
  return p;
}

void ctx_free(r4d_ctx* ctx, void* p) {
  if (!p) return;
  auto it = ctx->block_size.find(p);
  if (it != ctx->block_size.end()) ctx->free_blocks.insert({it->second, p});
}

// Temporary blocks of one call, returned to the cache when the call ends.
// (Stream order makes the reuse safe: later work on the same stream runs after
// every kernel already enqueued.)
struct Scratch {
  r4d_ctx* ctx;
  std::vector<void*> blocks;
  explicit Scratch(r4d_ctx* c) : ctx(c) {}
  ~Scratch() {
    for (void* p : blocks) ctx_free(ctx, p);
  }
  template <typename P>
  P* get(size_t bytes) {
    void* p = ctx_alloc(ctx, bytes);
    if (p) blocks.push_back(p);
    return static_cast<P*>(p);
  }
  void release(void* p) {
    for (auto& b : blocks)
      if (b == p) {
        ctx_free(ctx, p);
        b = nullptr;
      }
  }
  void keep(void* p) {  // ownership moves elsewhere
    for (auto& b : blocks)
      if (b == p) b = nullptr;
  }
};

int fwd_ppt(const r4d_settings& s) {
  return s.fwd_pixels_per_thread ? s.fwd_pixels_per_thread : raster_default_ppt(s.tile_size, false);
}
int bwd_ppt(const r4d_settings& s) {
  return s.bwd_pixels_per_thread ? s.bwd_pixels_per_thread : raster_default_ppt(s.tile_size, true);
}

bool valid_settings(const r4d_settings* s) {
  return s && (s->tile_size == 8 || s->tile_size == 16 || s->tile_size == 32) &&
         s->fwd_pixels_per_thread >= 0 && s->bwd_pixels_per_thread >= 0 &&
         raster_config_supported(s->tile_size, fwd_ppt(*s)) &&
         raster_config_supported(s->tile_size, bwd_ppt(*s)) &&
         s->near_plane >= 0.f && s->time_cull >= 0.f && s->extent_sigma > 0.f &&
         s->alpha_min > 0.f && s->alpha_max > s->alpha_min && s->alpha_max < 1.f &&
         s->T_min > 0.f && s->T_min < 1.f && s->dilation >= 0.f && s->guard_band > 0.f;
}

bool valid_view(const r4d_view& v) {
  return v.width > 0 && v.height > 0 && v.width <= 32768 && v.height <= 32768 && v.fx > 0.f &&
         v.fy > 0.f && std::isfinite(v.cx) && std::isfinite(v.cy) && std::isfinite(v.t);
}

SettingsDev make_settings(const r4d_settings& s) {
  SettingsDev d;
  d.near_plane = s.near_plane;
  d.time_cull = s.time_cull;
  d.ext2 = s.extent_sigma * s.extent_sigma;
  d.alpha_min = s.alpha_min;
  d.alpha_max = s.alpha_max;
  d.T_min = s.T_min;
  d.dilation = s.dilation;
  d.log_alpha_min = std::log(s.alpha_min);
  return d;
}

ViewDev make_view(const r4d_view& v, const r4d_settings& s) {
  ViewDev d;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) d.M[3 * r + c] = v.world_to_cam[4 * r + c];
    d.tw[r] = v.world_to_cam[4 * r + 3];
  }
  for (int c = 0; c < 3; ++c) {
    double acc = 0;
    for (int r = 0; r < 3; ++r) acc += double(d.M[3 * r + c]) * double(d.tw[r]);
    d.cam[c] = float(-acc);
  }
  d.fx = v.fx;
  d.fy = v.fy;
  d.cx = v.cx;
  d.cy = v.cy;
  d.limx = s.guard_band * 0.5f * float(v.width) / v.fx;
  d.limy = s.guard_band * 0.5f * float(v.height) / v.fy;
  d.t = v.t;
  for (int c = 0; c < 3; ++c) d.bg[c] = v.bg[c];
  d.W = v.width;
  d.H = v.height;
  d.tile_size = s.tile_size;
  d.tiles_x = (v.width + s.tile_size - 1) / s.tile_size;
  d.tiles_y = (v.height + s.tile_size - 1) / s.tile_size;
  return d;
}

int bits_for(uint64_t count) {  // bits needed for ids in [0, count)
  int b = 1;
  while ((uint64_t(1) << b) < count) ++b;
  return b;
}

enum Stage {
  kPreprocessFwd = 0,
  kDepthSort = 1,
  kCountScan = 2,
  kEmit = 3,
  kTileSort = 4,
  kTileRanges = 5,
  kRasterFwd = 6,
  kRasterBwd = 7,
  kPreprocessBwd = 8
};

// Records a pair of events around the work enqueued between start() and stop().
struct StageTimer {
  r4d_ctx* ctx;
  int stage;
  hipStream_t stream;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(r4d_ctx* c, int s, hipStream_t st) : ctx(c), stage(s), stream(st) {
    if (!ctx->timing) return;
    if (!ctx->event_pool.empty()) {
      a = ctx->event_pool.back().first;
      b = ctx->event_pool.back().second;
      ctx->event_pool.pop_back();
    } else if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, stream);
  }
  void stop() {
    if (!a) return;
    (void)hipEventRecord(b, stream);
    ctx->pending.push_back({stage, a, b});
    a = nullptr;
  }
  ~StageTimer() { stop(); }
};

#define R4D_TIMED(stage, expr)                 \
  do {                                         \
    StageTimer tm_(ctx, (stage), stream);      \
    R4D_HIP(expr);                             \
  } while (0)

#define R4D_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, R4D_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

#define R4D_ALLOC(var, type, bytes)                                                    \
  type* var = scratch.get<type>(bytes);                                                \
  if (!var) return fail(ctx, R4D_ERR_OOM, "device allocation of %zu bytes failed", (size_t)(bytes))

template <typename T>
r4d_status forward_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views, int n_views,
                        const r4d_settings* settings, T* images, r4d_saved** saved_out,
                        hipStream_t stream) {
  if (saved_out) *saved_out = nullptr;
  if (!views || n_views < 1 || !images || !valid_settings(settings))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid views, images or settings");
  if (g.n < 0 || g.deg < 0 || g.deg > 3)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid Gaussian count or SH degree");
  if (g.n > 0 && (!g.means || !g.log_scales || !g.rotors || !g.opacity || !g.sh))
    return fail(ctx, R4D_ERR_INVALID_ARG, "null Gaussian array");
  for (int i = 0; i < n_views; ++i)
    if (!valid_view(views[i])) return fail(ctx, R4D_ERR_INVALID_ARG, "invalid view %d", i);
  R4D_HIP(hipSetDevice(ctx->device));
  const SettingsDev st = make_settings(*settings);
  r4d_saved* saved = nullptr;
  if (saved_out) {
    saved = new r4d_saved();
    saved->ctx = ctx;
    ctx->live_saved.insert(saved);
    saved->f64 = sizeof(T) == 8;
    saved->n = g.n;
    saved->deg = g.deg;
    saved->settings = *settings;
    saved->views.resize(n_views);
  }
  struct SavedGuard {
    r4d_saved*& s;
    bool ok = false;
    ~SavedGuard() {
      if (!ok && s) r4d_saved_release(s);
    }
  } guard{saved};
  const uint32_t n = uint32_t(g.n);
  size_t img_off = 0;
  for (int vi = 0; vi < n_views; ++vi) {
    Scratch scratch(ctx);
    const r4d_view& view = views[vi];
    const ViewDev vd = make_view(view, *settings);
    const uint64_t hw = uint64_t(view.width) * view.height;
    const uint32_t n_tiles = uint32_t(vd.tiles_x) * uint32_t(vd.tiles_y);
    const size_t nn = n ? n : 1;
    R4D_ALLOC(recs, Rec<T>, nn * sizeof(Rec<T>));
    R4D_ALLOC(rects, Rect16, nn * sizeof(Rect16));
    R4D_ALLOC(tiles, uint32_t, nn * 4);
    R4D_ALLOC(kA, uint32_t, nn * 4);
    R4D_ALLOC(kB, uint32_t, nn * 4);
    R4D_ALLOC(vA, uint32_t, nn * 4);
    R4D_ALLOC(vB, uint32_t, nn * 4);
    R4D_ALLOC(totals, unsigned long long, 256);
    const size_t sort_tmp_bytes = sort_pairs_temp_bytes(n);
    R4D_ALLOC(sort_tmp, uint8_t, sort_tmp_bytes);
    R4D_HIP(hipMemsetAsync(totals, 0, 2 * sizeof(unsigned long long), stream));
    uint32_t* depth_saved = nullptr;
    if (saved) {
      depth_saved = scratch.get<uint32_t>(nn * 4);
      if (!depth_saved) return fail(ctx, R4D_ERR_OOM, "device allocation failed");
    }
    uint64_t D = 0, n_vis = 0;
    uint32_t* order = vA;
    if (n > 0) {
      R4D_TIMED(kPreprocessFwd, launch_preprocess_fwd<T>(g, vd, st, recs, rects, tiles, kA, vA,
                                                         totals, stream));
      if (depth_saved)
        R4D_HIP(hipMemcpyAsync(depth_saved, kA, size_t(n) * 4, hipMemcpyDeviceToDevice, stream));
      R4D_HIP(hipMemcpyAsync(ctx->host_readback, totals, 2 * sizeof(uint64_t),
                             hipMemcpyDeviceToHost, stream));
      uint32_t* kk[2] = {kA, kB};
      uint32_t* vv[2] = {vA, vB};
      int res = 0;
      R4D_TIMED(kDepthSort, sort_pairs_u32(kk, vv, n, 32, SortTemp{sort_tmp, sort_tmp_bytes},
                                           &res, stream));
      order = vv[res];
      R4D_HIP(hipStreamSynchronize(stream));
      n_vis = ctx->host_readback[0];
      D = ctx->host_readback[1];
    }
    if (D >= (uint64_t(1) << 31))
      return fail(ctx, R4D_ERR_CAPACITY, "view %d has %llu tile entries (limit 2^31)", vi,
                  (unsigned long long)D);
    const size_t dd = D ? size_t(D) : 1;
    R4D_ALLOC(ranges, uint2, size_t(n_tiles) * sizeof(uint2));
    R4D_ALLOC(T_final, T, hw * sizeof(T));
    R4D_ALLOC(n_contrib, uint32_t, hw * 4);
    uint32_t* n_eval = nullptr;
    if (ctx->timing) {
      n_eval = scratch.get<uint32_t>(hw * 4);
      if (!n_eval) return fail(ctx, R4D_ERR_OOM, "device allocation failed");
    }
    R4D_ALLOC(tvA, uint32_t, dd * 4);
    uint32_t* values = tvA;
    if (D == 0) {
      R4D_HIP(hipMemsetAsync(ranges, 0, size_t(n_tiles) * sizeof(uint2), stream));
    } else {
      // emit (tile, index) pairs in depth order, then sort them stably by tile id
      R4D_ALLOC(offsets, uint64_t, (nn + 1) * 8);
      const size_t scan_tmp_bytes = count_scan_temp_bytes(n);
      R4D_ALLOC(scan_tmp, uint8_t, scan_tmp_bytes);
      R4D_ALLOC(tkA, uint32_t, dd * 4);
      R4D_ALLOC(tkB, uint32_t, dd * 4);
      R4D_ALLOC(tvB, uint32_t, dd * 4);
      const size_t tsort_bytes = sort_pairs_temp_bytes(uint32_t(D));
      R4D_ALLOC(tsort_tmp, uint8_t, tsort_bytes);
      R4D_TIMED(kCountScan, count_scan(order, tiles, uint32_t(n_vis), offsets,
                                       SortTemp{scan_tmp, scan_tmp_bytes}, stream));
      R4D_TIMED(kEmit, emit_tile_keys(order, offsets, rects, uint32_t(n_vis), vd.tiles_x, tkA,
                                      tvA, stream));
      uint32_t* kk[2] = {tkA, tkB};
      uint32_t* vv[2] = {tvA, tvB};
      int res = 0;
      R4D_TIMED(kTileSort, sort_pairs_u32(kk, vv, uint32_t(D), bits_for(n_tiles),
                                          SortTemp{tsort_tmp, tsort_bytes}, &res, stream));
      values = vv[res];
      R4D_TIMED(kTileRanges, tile_ranges(kk[res], uint32_t(D), n_tiles, ranges, stream));
    }
    R4D_TIMED(kRasterFwd, launch_raster_fwd<T>(recs, values, ranges, vd, st, fwd_ppt(*settings),
                                              images + img_off, T_final, n_contrib, n_eval,
                                              stream));
    if (saved) {
      ViewSaved& vs = saved->views[vi];
      vs.view = view;
      vs.tiles_x = vd.tiles_x;
      vs.tiles_y = vd.tiles_y;
      vs.tile_size = vd.tile_size;
      vs.n_visible = n_vis;
      vs.n_dup = D;
      vs.recs = recs;
      vs.rects = rects;
      vs.depth_keys = depth_saved;
      vs.values = values;
      vs.ranges = ranges;
      vs.T_final = T_final;
      vs.n_contrib = n_contrib;
      vs.n_eval = n_eval;
      for (void* p : {(void*)recs, (void*)rects, (void*)depth_saved, (void*)values,
                      (void*)ranges, (void*)T_final, (void*)n_contrib, (void*)n_eval}) {
        if (!p) continue;
        scratch.keep(p);
        saved->blocks.push_back(p);
      }
    }
    img_off += 3 * hw;
  }
  guard.ok = true;
  if (saved_out) *saved_out = saved;
  return R4D_OK;
}

template <typename T>
r4d_status backward_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views,
                         int n_views, const r4d_settings* settings, const r4d_saved* saved,
                         const T* dL, const GradPtrs<T>& out, hipStream_t stream) {
  if (!views || n_views < 1 || !dL || !valid_settings(settings) || !saved)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid views, gradients, settings or saved state");
  if (g.n > 0 && (!g.means || !g.log_scales || !g.rotors || !g.opacity || !g.sh ||
                  !out.means || !out.log_scales || !out.rotors || !out.opacity || !out.sh))
    return fail(ctx, R4D_ERR_INVALID_ARG, "null Gaussian or gradient array");
  if (saved->ctx != ctx || saved->f64 != (sizeof(T) == 8) || saved->n != g.n ||
      saved->deg != g.deg || int(saved->views.size()) != n_views ||
      saved->settings.tile_size != settings->tile_size)
    return fail(ctx, R4D_ERR_STATE, "saved state does not match this backward call");
  for (int i = 0; i < n_views; ++i) {
    const r4d_view& a = saved->views[i].view;
    if (a.width != views[i].width || a.height != views[i].height || a.t != views[i].t ||
        std::memcmp(a.world_to_cam, views[i].world_to_cam, sizeof(a.world_to_cam)) != 0)
      return fail(ctx, R4D_ERR_STATE, "view %d differs from the forward call", i);
  }
  R4D_HIP(hipSetDevice(ctx->device));
  if (g.n == 0) return R4D_OK;
  const SettingsDev st = make_settings(*settings);
  Scratch scratch(ctx);
  const size_t n = size_t(g.n);
  R4D_ALLOC(grad2d, double, 9 * n * sizeof(double));
  size_t img_off = 0;
  for (int vi = 0; vi < n_views; ++vi) {
    const ViewSaved& vs = saved->views[vi];
    const ViewDev vd = make_view(views[vi], *settings);
    const uint64_t hw = uint64_t(views[vi].width) * views[vi].height;
    R4D_HIP(hipMemsetAsync(grad2d, 0, 9 * n * sizeof(double), stream));
    if (vs.n_dup > 0)
      R4D_TIMED(kRasterBwd, launch_raster_bwd<T>(static_cast<const Rec<T>*>(vs.recs), vs.values,
                                                vs.ranges, vd, st, bwd_ppt(*settings),
                                                static_cast<const T*>(vs.T_final), vs.n_contrib,
                                                dL + img_off, grad2d, uint32_t(n), stream));
    R4D_TIMED(kPreprocessBwd, launch_preprocess_bwd<T>(g, vd, st, grad2d, out, vi > 0, stream));
    img_off += 3 * hw;
  }
  return R4D_OK;
}

GaussPtrs<float> gauss_of(const r4d_gaussians* g) {
  return GaussPtrs<float>{g->n, g->sh_degree, g->means, g->log_scales, g->rotors, g->opacity,
                          g->sh};
}
GaussPtrs<double> gauss_of(const r4d_gaussians_f64* g) {
  return GaussPtrs<double>{g->n, g->sh_degree, g->means, g->log_scales, g->rotors, g->opacity,
                           g->sh};
}

}  // namespace

extern "C" {

void r4d_default_settings(r4d_settings* s) {
  if (!s) return;
  s->tile_size = 16;
  s->near_plane = 0.2f;
  s->time_cull = 16.0f;
  s->extent_sigma = 3.0f;
  s->alpha_min = 1.0f / 255.0f;
  s->alpha_max = 0.99f;
  s->T_min = 1e-4f;
  s->dilation = 0.3f;
  s->guard_band = 1.3f;
  s->fwd_pixels_per_thread = 0;
  s->bwd_pixels_per_thread = 0;
}

r4d_status r4d_create(r4d_ctx** out, int device) {
  if (!out) return R4D_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return R4D_ERR_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) return R4D_ERR_HIP;
  r4d_ctx* ctx = new r4d_ctx();
  ctx->device = device;
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->host_readback), 2 * sizeof(uint64_t),
                    hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return R4D_ERR_OOM;
  }
  *out = ctx;
  return R4D_OK;
}

void r4d_destroy(r4d_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  // saved states that outlive the context keep only their host struct
  for (r4d_saved* sv : ctx->live_saved) {
    sv->ctx = nullptr;
    sv->blocks.clear();
    sv->views.clear();
  }
  ctx->live_saved.clear();
  for (auto& kv : ctx->block_size) (void)hipFree(kv.first);
  for (auto& p : ctx->pending) ctx->event_pool.push_back({p.start, p.stop});
  for (auto& e : ctx->event_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (ctx->host_readback) (void)hipHostFree(ctx->host_readback);
  delete ctx;
}

r4d_status r4d_render_forward(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                              int n_views, const r4d_settings* settings, float* images,
                              r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return forward_impl<float>(ctx, gauss_of(g), views, n_views, settings, images, saved,
                             static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_forward_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                  const r4d_view* views, int n_views,
                                  const r4d_settings* settings, double* images,
                                  r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return forward_impl<double>(ctx, gauss_of(g), views, n_views, settings, images, saved,
                              static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                               int n_views, const r4d_settings* settings,
                               const r4d_saved* saved, const float* dL_dimages, r4d_grads* out,
                               void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GradPtrs<float> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<float>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages, o,
                              static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                   const r4d_view* views, int n_views,
                                   const r4d_settings* settings, const r4d_saved* saved,
                                   const double* dL_dimages, r4d_grads_f64* out, void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GradPtrs<double> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<double>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages, o,
                               static_cast<hipStream_t>(stream));
}

void r4d_saved_release(r4d_saved* saved) {
  if (!saved) return;
  if (saved->ctx) {  // null once the context has been destroyed
    for (void* p : saved->blocks) ctx_free(saved->ctx, p);
    saved->ctx->live_saved.erase(saved);
  }
  delete saved;
}

r4d_status r4d_l1_loss_grad(r4d_ctx* ctx, const float* image, const float* target, int64_t count,
                            float* dL_dimage, float* loss, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (count < 0 || (count > 0 && (!image || !target || !dL_dimage)))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid L1 arguments");
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(launch_l1_grad(image, target, count, dL_dimage, loss, static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_saved_stats(const r4d_saved* saved, int view, int64_t* n_visible, int64_t* n_dup,
                           int32_t* tiles_x, int32_t* tiles_y) {
  if (!saved || view < 0 || view >= int(saved->views.size())) return R4D_ERR_INVALID_ARG;
  const ViewSaved& v = saved->views[view];
  if (n_visible) *n_visible = int64_t(v.n_visible);
  if (n_dup) *n_dup = int64_t(v.n_dup);
  if (tiles_x) *tiles_x = v.tiles_x;
  if (tiles_y) *tiles_y = v.tiles_y;
  return R4D_OK;
}

r4d_status r4d_saved_copy(const r4d_saved* saved, int view, int buffer, void* dst, size_t bytes,
                          void* stream) {
  if (!saved || !saved->ctx || view < 0 || view >= int(saved->views.size()) || !dst)
    return R4D_ERR_INVALID_ARG;
  r4d_ctx* ctx = saved->ctx;
  const ViewSaved& v = saved->views[view];
  const size_t scal = saved->f64 ? 8 : 4;
  const size_t n = size_t(saved->n);
  const size_t hw = size_t(v.view.width) * v.view.height;
  const void* src = nullptr;
  size_t need = 0;
  switch (buffer) {
    case R4D_BUF_RECORDS: src = v.recs; need = n * 12 * scal; break;
    case R4D_BUF_RECT: src = v.rects; need = n * sizeof(Rect16); break;
    case R4D_BUF_DEPTHKEY: src = v.depth_keys; need = n * 4; break;
    case R4D_BUF_VALUES: src = v.values; need = size_t(v.n_dup) * 4; break;
    case R4D_BUF_RANGES: src = v.ranges; need = size_t(v.tiles_x) * v.tiles_y * 8; break;
    case R4D_BUF_TFINAL: src = v.T_final; need = hw * scal; break;
    case R4D_BUF_NCONTRIB: src = v.n_contrib; need = hw * 4; break;
    case R4D_BUF_NEVAL:
      if (!v.n_eval) return fail(ctx, R4D_ERR_STATE, "evaluation counts need timing enabled");
      src = v.n_eval;
      need = hw * 4;
      break;
    default: return fail(ctx, R4D_ERR_INVALID_ARG, "unknown buffer id %d", buffer);
  }
  if (bytes != need)
    return fail(ctx, R4D_ERR_INVALID_ARG, "buffer %d needs %zu bytes, got %zu", buffer, need,
                bytes);
  if (need == 0) return R4D_OK;
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_set_timing(r4d_ctx* ctx, int enable) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return R4D_OK;
}

r4d_status r4d_get_timings(r4d_ctx* ctx, double* ms, int64_t* launches, int reset) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  R4D_HIP(hipSetDevice(ctx->device));
  for (auto& p : ctx->pending) {
    float t = 0.f;
    R4D_HIP(hipEventSynchronize(p.stop));
    R4D_HIP(hipEventElapsedTime(&t, p.start, p.stop));
    ctx->stage_ms[p.stage] += double(t);
    ctx->stage_launches[p.stage] += 1;
    ctx->event_pool.push_back({p.start, p.stop});
  }
  ctx->pending.clear();
  for (int i = 0; i < R4D_NUM_STAGES; ++i) {
    if (ms) ms[i] = ctx->stage_ms[i];
    if (launches) launches[i] = ctx->stage_launches[i];
    if (reset) {
      ctx->stage_ms[i] = 0.0;
      ctx->stage_launches[i] = 0;
    }
  }
  return R4D_OK;
}

const char* r4d_stage_name(int stage) {
  static const char* names[R4D_NUM_STAGES] = {"preprocess_fwd", "depth_sort", "count_scan",
                                              "emit",           "tile_sort",  "tile_ranges",
                                              "raster_fwd",     "raster_bwd", "preprocess_bwd"};
  return stage >= 0 && stage < R4D_NUM_STAGES ? names[stage] : "";
}

const char* r4d_status_string(r4d_status s) {
  switch (s) {
    case R4D_OK: return "R4D_OK";
    case R4D_ERR_INVALID_ARG: return "R4D_ERR_INVALID_ARG";
    case R4D_ERR_HIP: return "R4D_ERR_HIP";
    case R4D_ERR_OOM: return "R4D_ERR_OOM";
    case R4D_ERR_CAPACITY: return "R4D_ERR_CAPACITY";
    case R4D_ERR_STATE: return "R4D_ERR_STATE";
  }
  return "R4D_ERR_UNKNOWN";
}

const char* r4d_last_error(const r4d_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

}  // extern "C"
