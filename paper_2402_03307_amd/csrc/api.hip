// C-ABI layer: argument checking, device memory, graph capture, the autotuner
// and the order of kernel launches.
//
// Work is organised in runs.  A run renders a set of views with one launch per
// stage:
//   zero-fill -> preprocess (every view) -> depth-key histogram -> segmented
//   depth sort -> tile counts, ranges and segment table -> scan of the tile
//   counts in depth order -> emit tile entries -> segmented tile sort ->
//   persistent rasteriser over the tiles of every view.
// Backward of a run: zero-fill -> persistent raster backward (screen-space
// gradients per view and Gaussian) -> preprocess backward (summed over views).
//
// Per-view mode makes every view its own run; fused and graph modes make one
// run of all views.  Outside graph mode the host reads the per-view entry
// counts back after the preprocess (while the depth sort runs) and sizes the
// tile lists exactly.  Graph mode captures the run with a fixed capacity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "front.hpp"
#include "r4d.h"
#include "r4d_internal.hpp"

using namespace r4d;

namespace {
// What one run reports back in one copy: the status words (overflow, sort
// look-back error; 16 bytes), two totals per render (visible Gaussians, tile
// entries of the whole lists) and the front-list table.
constexpr size_t kReadbackBytes = 16 + 2 * size_t(kMaxViews) * 8 + sizeof(FrontTable);
}  // namespace

// Device memory of r4d_render_forward_noalloc: every buffer of its runs lives
// in this region, one copy per GPU, held until the process ends.  Host code
// never passes `scratch` itself to a kernel or a copy (in host code it names a
// host-side stand-in); it uses the device address that r4d_create looks up on
// each GPU (noalloc_region).
constexpr size_t kNoallocBytes = size_t(R4D_NOALLOC_BYTES);
static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

namespace {

// Device address of `scratch` on each GPU, looked up once per device with that
// device current.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint8_t* g_noalloc_ptr[kMaxDevices] = {};

hipError_t noalloc_region(int device, uint8_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc_ptr[device] = static_cast<uint8_t*>(p);
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

}  // namespace

namespace {

struct GraphEntry;

// Sub-buffers of one run, laid out in two device blocks: `fixed` (sizes known
// before the run) and `entries` (the tile lists, sized by the entry capacity).
struct RunLayout {
  // fixed block
  size_t meta, recs, flows, rects, tiles, dkeys, kA, kB, vA, vB, thist, offsets, scan_tmp,
      ranges, T_final, n_contrib, n_eval, img_copy, flow_copy, walk, ptemp_fwd, keep, fcount,
      srect, queue, zero_begin, status, totals, front, rest, cover, tsums, dhist, tickets, dstatus,
      zero_end,
      fixed_bytes;
  // entries block
  size_t tkA, tkB, tvA, tvB, tdig, thi, t16, etemp, ptemp, ck, ckf, tstatus, entries_bytes;
};

constexpr int kTicketTile = 4;     // tickets[0..3] depth passes, [4..6] tile passes
constexpr int kTicketRaster = 7;   // [7] forward rasteriser
constexpr int kDepthItems = 8;  // keys per thread of the depth sort passes (measured best)

// Host-side plan of one run.
struct Plan {
  int V = 0;
  uint32_t n = 0, n_pad = 0;
  int deg = 0, ts = 16, fppt = 1, bppt = 4, sort_items = 16, mode = 0;
  std::vector<ViewSlot> slots;
  uint32_t total_tiles = 0;
  uint64_t total_pix = 0;
  uint32_t max_tiles = 0;
  int tile_passes = 1;
  bool packed = true;   // packed tile sort (see packed_tile_sort_ok)
  SegTable dseg{};
  size_t scal = 4;
  bool count_evals = false;
  bool flow = false;    // also composite the 2D flow (flow images)
  bool static3d = false;  // static 3D Gaussians (means 3, log-scales 3, quaternions 4 rows)
  // front lists (front.hpp): some render has a depth cut; the keep threshold;
  // sizes of all renders' keep bitmaps (words) and cover grids (ints)
  bool front = false;
  int32_t front_keep = 0;
  size_t keep_words_total = 0, cover_total = 0;
};

}  // namespace

struct r4d_ctx {
  int device = 0;
  std::string last_error;
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
  // pinned staging for per-call uploads (ring) and readbacks
  struct Stage {
    void* host = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<Stage> ring;
  size_t ring_next = 0;
  unsigned long long* readback = nullptr;    // pinned, 2 * kMaxViews words
  float* l1_partials = nullptr;              // device, l1_partials_floats() words
  hipStream_t capture_stream = nullptr;
  std::set<r4d_saved*> live_saved;
  std::map<std::string, std::unique_ptr<GraphEntry>> graphs;
  std::map<std::string, std::pair<int, int>> tuned;  // shape -> (tile size, sort items)
  bool tuned_loaded = false;  // the autotuner's cache file has been read
  std::string device_tag;     // architecture and compute-unit count (cache keys)
  // pinned readback areas of runs with their completion events; an area is
  // reused once its event has completed
  struct Pinned {
    unsigned long long* host = nullptr;
    hipEvent_t done = nullptr;
    int refs = 0;  // holders: a run, a graph's latest replay, a saved state, `unchecked`
  };
  std::vector<Pinned*> pinned_pool;
  // readback areas of forwards whose status words nobody has read yet (calls
  // without saved state, saved states released unchecked); read, without
  // waiting, by the next render call, which reports an overflow or sort failure
  std::vector<Pinned*> unchecked;
  // no-allocation forward: the device address of this GPU's region and the
  // readback area of its runs (set up by r4d_create, outside the pinned pool)
  uint8_t* noalloc = nullptr;
  Pinned* noalloc_slot = nullptr;
};

namespace {

// Device memory and flags of one executed run.
struct RunState {
  Plan plan;
  RunLayout L{};
  uint8_t* fixed = nullptr;
  uint8_t* entries = nullptr;
  uint64_t capacity = 0;
  uint32_t* values = nullptr;  // sorted Gaussian indices of the tile entries
  bool owns_memory = true;     // false for graph runs (buffers live in the entry)
                               // and for runs in the no-allocation region
  // no-allocation runs: bytes available to the entries block, which the sized
  // path checks instead of allocating (0: the block is allocated)
  size_t entries_limit = 0;
  // per-view counts (valid after `done`); front lists: entries in the front
  // (or whole) lists, tiles that collected a rest, rest area taken
  std::vector<uint64_t> n_visible, n_dup, n_front, rest_tiles, rest_entries;
  uint32_t flags[2] = {0, 0};  // overflow, look-back error
  bool counts_valid = false;
  // pinned readback of totals + flags, filled at the end of the run
  r4d_ctx::Pinned* slot = nullptr;
  unsigned long long* pinned = nullptr;  // kReadbackBytes: status words, totals, front table
  hipEvent_t done = nullptr;
  size_t image_offset = 0;     // first image element of this run in the call's images
  size_t flow_offset = 0;      // first flow element of this run in the call's flow images
};

struct GraphEntry {
  RunState run;
  hipGraphExec_t fwd = nullptr;
  hipGraphExec_t bwd = nullptr;
  std::string bwd_key;
  uint8_t* bwd_block = nullptr;  // grad2d + ticket of the captured backward
  uint64_t generation = 0;
  bool needs_grow = false;
};

}  // namespace

struct r4d_saved {
  r4d_ctx* ctx = nullptr;
  bool f64 = false;
  bool flow = false;            // flow render: the backward may take flow gradients
  bool static3d = false;        // static 3D Gaussians
  int n = 0, deg = 0;
  r4d_settings settings;        // as resolved (tile size chosen)
  r4d_ctx::Pinned* graph_slot = nullptr;  // graph mode: the replay's readback area
  mutable bool checked = false; // status words read (backward or r4d_saved_check)
  std::vector<r4d_view> views;
  std::vector<std::unique_ptr<RunState>> runs;  // owned runs (per-view, fused)
  GraphEntry* graph = nullptr;  // graph mode
  uint64_t generation = 0;
  std::vector<std::pair<int, int>> where;  // view -> (run, index within run)
  RunState* run_of(int r) const { return graph ? &graph->run : runs[size_t(r)].get(); }
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

void unref_slot(r4d_ctx::Pinned* q) {
  if (q && q->refs > 0) q->refs -= 1;  // reused once unheld and its event has completed
}

// unchecked: the run's status words have not been read; its readback area
// moves to the context's unchecked list instead of being freed.
void release_run(r4d_ctx* ctx, RunState* r, bool unchecked = false) {
  if (!r) return;
  if (r->owns_memory) {
    ctx_free(ctx, r->fixed);
    ctx_free(ctx, r->entries);
  }
  r->fixed = r->entries = nullptr;
  if (r->slot) {
    if (unchecked)
      ctx->unchecked.push_back(r->slot);
    else
      unref_slot(r->slot);
  }
  r->slot = nullptr;
  r->pinned = nullptr;
  r->done = nullptr;
}

int default_ppt(int tile_size, int requested, bool backward) {
  return requested ? requested : raster_default_ppt(tile_size, backward);
}

bool valid_settings(const r4d_settings* s) {
  if (!s) return false;
  if (s->tile_size != 0 && s->tile_size != 8 && s->tile_size != 16 && s->tile_size != 32)
    return false;
  if (s->fwd_pixels_per_thread < 0 || s->bwd_pixels_per_thread < 0) return false;
  if (s->tile_size != 0 &&
      (!raster_config_supported(s->tile_size, default_ppt(s->tile_size, s->fwd_pixels_per_thread, false)) ||
       !raster_config_supported(s->tile_size, default_ppt(s->tile_size, s->bwd_pixels_per_thread, true))))
    return false;
  if (s->tile_size == 0 && (s->fwd_pixels_per_thread || s->bwd_pixels_per_thread)) return false;
  if (s->mode < R4D_MODE_PER_VIEW || s->mode > R4D_MODE_GRAPH) return false;
  if (s->sort_items != 0 && s->sort_items != 8 && s->sort_items != 16) return false;
  if (!(s->front_fraction >= 0.f)) return false;  // (NaN fails too)
  return s->near_plane >= 0.f && s->time_cull >= 0.f && s->extent_sigma > 0.f &&
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

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

uint64_t round_seg(uint64_t x) { return (x + kSegAlign - 1) / kSegAlign * kSegAlign; }

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

// Records a pair of events around the work enqueued between construction and
// stop() (measurement aid; never inside a graph capture).
struct StageTimer {
  r4d_ctx* ctx;
  int stage;
  hipStream_t stream;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(r4d_ctx* c, int s, hipStream_t st, bool on) : ctx(c), stage(s), stream(st) {
    if (!on || !ctx->timing) return;
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

#define R4D_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, R4D_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

#define R4D_TIMED(stage, expr)                      \
  do {                                              \
    StageTimer tm_(ctx, (stage), stream, timed);    \
    R4D_HIP(expr);                                  \
  } while (0)

std::string view_shape_key(const r4d_view* views, int V) {
  std::string k;
  char buf[64];
  for (int i = 0; i < V; ++i) {
    snprintf(buf, sizeof(buf), "%dx%d;", views[i].width, views[i].height);
    k += buf;
  }
  return k;
}

Plan make_plan(const r4d_view* views, int V, uint32_t n, int deg, const r4d_settings& s,
               size_t scal, bool flow, bool static3d) {
  Plan p;
  p.flow = flow;
  p.static3d = static3d;
  p.V = V;
  p.n = n;
  p.n_pad = uint32_t(round_seg(n));
  p.deg = deg;
  p.ts = s.tile_size;
  p.fppt = default_ppt(s.tile_size, s.fwd_pixels_per_thread, false);
  p.bppt = default_ppt(s.tile_size, s.bwd_pixels_per_thread, true);
  p.sort_items = s.sort_items ? s.sort_items : 16;
  p.mode = s.mode;
  p.scal = scal;
  int bits = 1;
  for (int i = 0; i < V; ++i) {
    ViewSlot sl{};
    sl.v = make_view(views[i], s);
    sl.tile_base = p.total_tiles;
    sl.pix_base = p.total_pix;
    const uint64_t nt = uint64_t(sl.v.tiles_x) * uint64_t(sl.v.tiles_y);
    p.total_tiles += uint32_t(nt);
    p.total_pix += uint64_t(views[i].width) * uint64_t(views[i].height);
    bits = std::max(bits, bits_for(nt));
    p.max_tiles = std::max(p.max_tiles, uint32_t(nt));
    p.slots.push_back(sl);
  }
  p.tile_passes = (bits + 7) / 8;
  p.packed = s.sort_items == 0 && packed_tile_sort_ok(n, p.max_tiles);
  // front lists: the depth cut as a fraction of 65536 (at least 1), for the
  // renders whose tile grid fits the keep kernel
  const uint32_t f16 =
      s.front_fraction >= 1.0f
          ? 0u
          : uint32_t(std::min(65536.0, std::max(1.0, std::ceil(double(s.front_fraction) * 65536.0))));
  p.front_keep = s.front_keep;
  for (ViewSlot& sl : p.slots) {
    sl.front16 = (f16 && front_grid_ok(sl.v.tiles_x, sl.v.tiles_y)) ? f16 : 0u;
    sl.keep_base = uint32_t(p.keep_words_total);
    sl.cover_base = uint32_t(p.cover_total);
    if (sl.front16) {
      p.front = true;
      p.keep_words_total += size_t(keep_words(sl.v.tiles_x)) * size_t(sl.v.tiles_y);
      p.cover_total += size_t(sl.v.tiles_x + 1) * size_t(sl.v.tiles_y + 1);
    }
  }
  p.dseg.count = uint32_t(V);
  p.dseg.overflow = 0;
  for (int v = 0; v <= V; ++v) p.dseg.start[v] = uint32_t(uint64_t(v) * p.n_pad);
  for (int v = 0; v < V; ++v) p.dseg.len[v] = n;
  return p;
}

// Boundary-state slots of the backward's segment walks (see ck_slot).
uint64_t ck_slots(const Plan& p, uint64_t capacity) {
  return capacity / kSegment + uint64_t(p.total_tiles) + 2;
}

// Bound on the backward's (tile, segment) walks.
uint64_t bwd_items(const Plan& p, uint64_t capacity) {
  return capacity / kSegment + uint64_t(p.total_tiles) + 1;
}

RunLayout make_layout(const Plan& p, uint64_t capacity) {
  RunLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes ? bytes : 1);
    return o;
  };
  const size_t V = size_t(p.V), n = size_t(p.n), np = size_t(p.n_pad);
  const size_t rec_bytes = 12 * p.scal;
  L.meta = take(sizeof(ViewSlot) * V + 2 * sizeof(SegTable));
  L.recs = take(V * n * rec_bytes);
  L.flows = p.flow ? take(V * n * 2 * p.scal) : 0;
  L.rects = take(V * n * sizeof(Rect16));
  L.tiles = take(V * n * 4);
  L.dkeys = take(V * np * 4);
  L.kA = take(V * np * 4);
  L.kB = take(V * np * 4);
  L.vA = take(V * np * 4);
  L.vB = take(V * np * 4);
  L.thist = take(3 * size_t(kMaxViews) * 256 * 4);
  L.offsets = take((V * np + 1) * 8);
  L.scan_tmp = take(count_scan_seg_temp_bytes(p.n_pad, p.V));
  L.T_final = take(size_t(p.total_pix) * p.scal);
  L.n_contrib = take(size_t(p.total_pix) * 4);
  L.n_eval = p.count_evals ? take(size_t(p.total_pix) * 8) : 0;
  L.img_copy = take(3 * size_t(p.total_pix) * p.scal);
  L.flow_copy = p.flow ? take(2 * size_t(p.total_pix) * p.scal) : 0;
  L.walk = take(size_t(p.total_tiles) * 4);
  L.ptemp_fwd = take(preprocess_temp_bytes(p.n, p.V));
  L.keep = take(p.keep_words_total * 8);
  L.fcount = p.front ? take(V * np * 4) : 0;
  L.srect = p.front ? take(V * np * sizeof(Rect16)) : 0;
  L.queue = p.front ? take(size_t(p.total_tiles) * 4) : 0;
  L.zero_begin = off;
  L.ranges = take(size_t(p.total_tiles) * 8);  // tiles without entries keep [0, 0)
  // status words (overflow, sort look-back error) followed by the per-render
  // totals and the front-list table, so that one copy returns all a run reports
  L.status = take(kReadbackBytes);
  L.totals = L.status + 16;
  L.front = L.totals + 2 * size_t(kMaxViews) * 8;
  L.rest = take(size_t(p.total_tiles) * 8);
  L.cover = take(p.cover_total * 4);
  L.tsums = p.front ? take(count_tile_sums_bytes(p.n_pad, p.V)) : 0;
  L.dhist = take(4 * size_t(kMaxViews) * 256 * 4);
  L.tickets = take(16 * 4);
  L.dstatus = take(4 * size_t(sort_status_words(uint64_t(V) * np, kDepthItems)) * 4);
  L.zero_end = off;
  L.fixed_bytes = off;
  off = 0;
  const size_t cap = size_t(capacity);
  L.tkA = take(cap * 4);
  L.tvA = take(cap * 4);
  L.ck = take(size_t(ck_slots(p, capacity)) * size_t(p.ts) * size_t(p.ts) * 4 * p.scal);
  L.ckf = p.flow ? take(size_t(ck_slots(p, capacity)) * size_t(p.ts) * size_t(p.ts) * 2 * p.scal)
                 : 0;
  L.etemp = take(emit_temp_bytes(capacity));
  if (p.packed) {
    L.tkB = L.tvB = 0;
    L.tdig = take(cap);
    L.thi = take(cap);
    L.t16 = take(cap * 2);
    L.ptemp = take(packed_sort_temp_bytes(capacity));
    L.tstatus = off;  // nothing to zero
  } else {
    L.tkB = take(cap * 4);
    L.tvB = take(cap * 4);
    L.tdig = L.thi = L.t16 = 0;
    L.ptemp = 0;
    L.tstatus = take(size_t(p.tile_passes) * sort_status_words(capacity, p.sort_items) * 4);
  }
  L.entries_bytes = off;
  return L;
}

template <typename P>
P* at(uint8_t* base, size_t off) {
  return reinterpret_cast<P*>(base + off);
}

// Copies the run's slot table and depth segment table into device memory
// through a ring of pinned staging buffers (the copy is stream-ordered; a
// staging buffer is reused only after its previous copy has completed).
r4d_status upload_meta(r4d_ctx* ctx, const Plan& p, uint8_t* fixed, const RunLayout& L,
                       hipStream_t stream) {
  const size_t bytes = sizeof(ViewSlot) * size_t(p.V) + sizeof(SegTable);
  r4d_ctx::Stage& s = ctx->ring[ctx->ring_next];
  ctx->ring_next = (ctx->ring_next + 1) % ctx->ring.size();
  R4D_HIP(hipEventSynchronize(s.done));
  std::memcpy(s.host, p.slots.data(), sizeof(ViewSlot) * size_t(p.V));
  std::memcpy(static_cast<uint8_t*>(s.host) + sizeof(ViewSlot) * size_t(p.V), &p.dseg,
              sizeof(SegTable));
  R4D_HIP(hipMemcpyAsync(fixed + L.meta, s.host, bytes, hipMemcpyHostToDevice, stream));
  R4D_HIP(hipEventRecord(s.done, stream));
  return R4D_OK;
}

const ViewSlot* slots_of(uint8_t* fixed, const RunLayout& L) {
  return at<ViewSlot>(fixed, L.meta);
}
SegTable* dseg_of(uint8_t* fixed, const RunLayout& L, int V) {
  return reinterpret_cast<SegTable*>(fixed + L.meta + sizeof(ViewSlot) * size_t(V));
}
SegTable* tseg_of(uint8_t* fixed, const RunLayout& L, int V) {
  return dseg_of(fixed, L, V) + 1;
}

// What the backward's segment walks read, as the forward left it.
template <typename T>
RasterSaved<T> saved_of(const RunState& r) {
  uint8_t* F = r.fixed;
  uint8_t* E = r.entries;
  const bool fl = r.plan.flow;
  return RasterSaved<T>{at<Ck<T>>(E, r.L.ck), at<T>(F, r.L.img_copy), at<uint32_t>(F, r.L.walk),
                        fl ? at<Vec2<T>>(E, r.L.ckf) : nullptr,
                        fl ? at<T>(F, r.L.flow_copy) : nullptr, at<uint2>(F, r.L.rest)};
}

// Enqueues the forward of a run.  sized = false: entries block and capacity
// are already in place (graph capture); sized = true: after the preprocess the
// per-view totals are read back and the entries block is allocated exactly.
template <typename T>
r4d_status enqueue_forward(r4d_ctx* ctx, const GaussPtrs<T>& g, RunState& r, T* images,
                           T* flow_images, const SettingsDev& st, bool sized, bool timed,
                           hipStream_t stream) {
  const Plan& p = r.plan;
  RunLayout& L = r.L;
  uint8_t* F = r.fixed;
  const ViewSlot* slots = slots_of(F, L);
  SegTable* dseg = dseg_of(F, L, p.V);
  SegTable* tseg = tseg_of(F, L, p.V);
  auto* totals = at<unsigned long long>(F, L.totals);
  auto* tickets = at<uint32_t>(F, L.tickets);
  uint32_t* status = at<uint32_t>(F, L.status);  // [0] overflow, [1] look-back error
  uint32_t* error = status + 1;
  // the run's counters and status words: cleared by the preprocess, or here
  // when there is nothing to preprocess
  const size_t zero_bytes = L.zero_end - L.zero_begin;
  if (p.n == 0) R4D_HIP(fill_zero(F + L.zero_begin, zero_bytes, stream));
  const uint32_t* order = nullptr;
  if (p.n > 0) {
    StageTimer tm(ctx, kPreprocessFwd, stream, timed);
    R4D_HIP(launch_preprocess_fwd<T>(g, slots, p.V, st, p.n_pad, at<Rec<T>>(F, L.recs),
                                     p.flow ? at<Vec2<T>>(F, L.flows) : nullptr,
                                     at<Rect16>(F, L.rects), at<uint32_t>(F, L.tiles),
                                     at<uint32_t>(F, L.dkeys), totals, at<uint32_t>(F, L.kA),
                                     at<uint32_t>(F, L.vA), dseg, F + L.ptemp_fwd,
                                     F + L.zero_begin, zero_bytes, p.static3d, stream));
  }
  hipEvent_t totals_ready = nullptr;
  if (sized) {
    R4D_HIP(hipMemcpyAsync(ctx->readback, totals, 2 * size_t(p.V) * 8, hipMemcpyDeviceToHost,
                           stream));
    totals_ready = r.done;
    R4D_HIP(hipEventRecord(totals_ready, stream));
  }
  if (p.n > 0) {
    StageTimer tm(ctx, kDepthSort, stream, timed);
    // the visible Gaussians' keys and indices, compacted by the preprocess, in kA / vA
    R4D_HIP(radix_histogram(at<uint32_t>(F, L.kA), dseg, p.V, p.n, 4, at<uint32_t>(F, L.dhist),
                            stream));
    uint32_t* kb[2] = {at<uint32_t>(F, L.kB), at<uint32_t>(F, L.kA)};
    uint32_t* vb[2] = {at<uint32_t>(F, L.vB), at<uint32_t>(F, L.vA)};
    int res = 0;
    R4D_HIP(onesweep_sort(at<uint32_t>(F, L.kA), at<uint32_t>(F, L.vA), kb, vb, dseg,
                          uint64_t(p.V) * p.n_pad, 4, kDepthItems, at<uint32_t>(F, L.dhist),
                          at<uint32_t>(F, L.dstatus), tickets, error, false, &res, stream));
    order = vb[res];
  }
  if (sized) {
    R4D_HIP(hipEventSynchronize(totals_ready));
    uint64_t cap = 0;
    for (int v = 0; v < p.V; ++v) {
      const uint64_t d = ctx->readback[2 * v + 1];
      if (d >= (uint64_t(1) << 30))
        return fail(ctx, R4D_ERR_CAPACITY, "view %d has %llu tile entries (limit 2^30)", v,
                    (unsigned long long)d);
      cap += seg_extent(d, p.slots[size_t(v)]);
    }
    if (cap >= (uint64_t(1) << 32))
      return fail(ctx, R4D_ERR_CAPACITY, "%llu tile entries in one call (limit 2^32)",
                  (unsigned long long)cap);
    r.capacity = cap;
    const RunLayout L2 = make_layout(p, cap);
    L.tkA = L2.tkA;
    L.tkB = L2.tkB;
    L.tvA = L2.tvA;
    L.tvB = L2.tvB;
    L.tdig = L2.tdig;
    L.thi = L2.thi;
    L.t16 = L2.t16;
    L.etemp = L2.etemp;
    L.ptemp = L2.ptemp;
    L.ck = L2.ck;
    L.ckf = L2.ckf;
    L.tstatus = L2.tstatus;
    L.entries_bytes = L2.entries_bytes;
    if (r.entries_limit) {
      // no-allocation run: the entries block is already in place
      if (L.entries_bytes > r.entries_limit)
        return fail(ctx, R4D_ERR_CAPACITY,
                    "%llu tile entries need %zu bytes of tile lists; the no-allocation region "
                    "has %zu left after the per-Gaussian buffers",
                    (unsigned long long)cap, L.entries_bytes, r.entries_limit);
    } else {
      r.entries = static_cast<uint8_t*>(ctx_alloc(ctx, L.entries_bytes));
      if (!r.entries)
        return fail(ctx, R4D_ERR_OOM, "device allocation of %zu bytes failed", L.entries_bytes);
    }
  }
  uint8_t* E = r.entries;
  auto* ranges = at<uint2>(F, L.ranges);
  // the segment table of the emitted list (with the count scan when there are Gaussians)
  if (p.n == 0) R4D_HIP(seg_table(totals, slots, p.V, r.capacity, tseg, status, stream));
  uint32_t* values = at<uint32_t>(E, L.tvA);
  const void* sorted_tiles = nullptr;
  if (p.n > 0) {
    auto* offsets = at<uint64_t>(F, L.offsets);
    {
      StageTimer tm(ctx, kCountScan, stream, timed);
      if (p.front) {
        // front lists: which tiles keep their whole list, then the entry counts
        R4D_HIP(front_keep(slots, p.V, at<Rect16>(F, L.rects), order, totals, p.n, p.n_pad,
                           p.front_keep, at<int32_t>(F, L.cover), at<uint64_t>(F, L.keep),
                           stream));
        R4D_HIP(front_counts<T>(order, at<uint32_t>(F, L.tiles), at<Rect16>(F, L.rects),
                                at<Rec<T>>(F, L.recs), slots, totals, at<uint64_t>(F, L.keep),
                                p.n, p.n_pad, p.V, at<uint32_t>(F, L.fcount),
                                at<Rect16>(F, L.srect), at<uint64_t>(F, L.tsums), r.capacity,
                                tseg, status, stream));
      }
      R4D_HIP(count_scan_seg(order, at<uint32_t>(F, L.tiles),
                             p.front ? at<uint32_t>(F, L.fcount) : nullptr, totals, slots, p.n,
                             p.n_pad, p.V, offsets, F + L.scan_tmp, r.capacity, tseg,
                             p.front ? at<FrontTable>(F, L.front) : nullptr, status,
                             at<uint32_t>(E, L.etemp),
                             p.front ? at<uint64_t>(F, L.tsums) : nullptr, stream));
    }
    // packed: (index | high tile byte) words into tvA and low tile bytes into
    // tdig; otherwise tile ids into tkA and indices into tvA
    uint32_t* out_a = p.packed ? at<uint32_t>(E, L.tvA) : at<uint32_t>(E, L.tkA);
    void* out_b = p.packed ? static_cast<void*>(E + L.tdig) : static_cast<void*>(E + L.tvA);
    R4D_TIMED(kEmit, emit_blocks<T>(order, offsets, at<Rect16>(F, L.rects),
                                    at<Rec<T>>(F, L.recs), slots, tseg, totals,
                                    p.front ? at<uint64_t>(F, L.keep) : nullptr,
                                    p.front ? at<uint32_t>(F, L.fcount) : nullptr, p.n, p.n_pad,
                                    p.V, r.capacity, p.packed, E + L.etemp, out_a, out_b,
                                    p.packed ? E + L.ptemp : nullptr, stream));
    if (p.packed) {
      // low tile byte pass into (tkA, thi), high byte pass into (tvA, t16)
      R4D_TIMED(kTileSort, packed_tile_sort(at<uint32_t>(E, L.tvA), E + L.tdig, tseg,
                                            p.max_tiles, r.capacity, E + L.ptemp,
                                            at<uint32_t>(E, L.tkA), E + L.thi,
                                            at<uint32_t>(E, L.tvA), at<uint16_t>(E, L.t16),
                                            stream));
      values = at<uint32_t>(E, L.tvA);
      sorted_tiles = E + L.t16;
    } else {
      StageTimer tm(ctx, kTileSort, stream, timed);
      R4D_HIP(tile_key_histogram(at<uint32_t>(E, L.tkA), tseg, r.capacity, p.tile_passes,
                                 at<uint32_t>(F, L.thist), stream));
      R4D_HIP(fill_zero(E + L.tstatus, L.entries_bytes - L.tstatus, stream));
      uint32_t* kb[2] = {at<uint32_t>(E, L.tkB), at<uint32_t>(E, L.tkA)};
      uint32_t* vb[2] = {at<uint32_t>(E, L.tvB), at<uint32_t>(E, L.tvA)};
      int res = 0;
      R4D_HIP(onesweep_sort(at<uint32_t>(E, L.tkA), at<uint32_t>(E, L.tvA), kb, vb, tseg,
                            r.capacity, p.tile_passes, p.sort_items, at<uint32_t>(F, L.thist),
                            at<uint32_t>(E, L.tstatus), tickets + kTicketTile, error, true, &res,
                            stream));
      values = vb[res];
      sorted_tiles = kb[res];
    }
  }
  R4D_TIMED(kTileRanges, tile_ranges(sorted_tiles, p.packed, tseg, slots, p.total_tiles,
                                     p.n > 0 ? r.capacity : 0, ranges, stream));
  r.values = values;
  const RasterSaved<T> sv = saved_of<T>(r);
  FrontCollect fc{};
  if (p.front && p.n > 0)
    fc = FrontCollect{at<uint64_t>(F, L.keep), order,       at<Rect16>(F, L.srect),
                      totals,                  at<FrontTable>(F, L.front), at<uint32_t>(F, L.queue),
                      status,                  p.n_pad};
  R4D_TIMED(kRasterFwd,
            launch_raster_fwd<T>(at<Rec<T>>(F, L.recs),
                                 p.flow ? at<Vec2<T>>(F, L.flows) : nullptr, p.n, values, ranges,
                                 fc, slots, p.V, p.total_tiles, p.ts, st, p.fppt, images,
                                 p.flow ? flow_images : nullptr, at<T>(F, L.T_final),
                                 at<uint32_t>(F, L.n_contrib),
                                 p.count_evals ? at<uint32_t>(F, L.n_eval) : nullptr, sv,
                                 tickets + kTicketRaster, stream));
  return R4D_OK;
}

// Copies totals and flags to the run's pinned area and records its `done`
// event (outside any capture).
r4d_status finish_run(r4d_ctx* ctx, RunState& r, hipStream_t stream) {
  // status words, totals and front table in one copy: pinned[0] = (overflow,
  // error), pinned[1] unused, pinned[2 + 2v], [3 + 2v] = render v's totals,
  // the front table from pinned[2 + 2 kMaxViews] on
  R4D_HIP(hipMemcpyAsync(r.pinned, r.fixed + r.L.status, kReadbackBytes, hipMemcpyDeviceToHost,
                         stream));
  R4D_HIP(hipEventRecord(r.done, stream));
  r.counts_valid = false;
  return R4D_OK;
}

r4d_status wait_run(r4d_ctx* ctx, RunState& r) {
  if (r.counts_valid) return R4D_OK;
  R4D_HIP(hipEventSynchronize(r.done));
  const int V = r.plan.V;
  r.n_visible.assign(size_t(V), 0);
  r.n_dup.assign(size_t(V), 0);
  const FrontTable* ft = reinterpret_cast<const FrontTable*>(r.pinned + 2 + 2 * kMaxViews);
  r.n_front.assign(size_t(V), 0);
  r.rest_tiles.assign(size_t(V), 0);
  r.rest_entries.assign(size_t(V), 0);
  for (int v = 0; v < V; ++v) {
    r.n_visible[size_t(v)] = r.pinned[2 + 2 * v];
    r.n_dup[size_t(v)] = r.pinned[3 + 2 * v];
    r.n_front[size_t(v)] = r.plan.front ? ft->n_front[v] : r.n_dup[size_t(v)];
    r.rest_tiles[size_t(v)] = ft->rest_tiles[v];
    r.rest_entries[size_t(v)] = ft->cursor[v];
  }
  const uint32_t* fl = reinterpret_cast<const uint32_t*>(r.pinned);
  r.flags[0] = fl[0];
  r.flags[1] = fl[1];
  r.counts_valid = true;
  return R4D_OK;
}

// A readback area nobody holds whose last copy has completed (or a new one),
// returned with one reference.
// Entries of render vi's part of the list buffer that VALUES copies (after
// wait_run): its front (or whole) lists, and with rest ranges the rest area
// up to the last one.
uint64_t values_count(const RunState& r, int vi) {
  const uint64_t nf = r.n_front[size_t(vi)], rest = r.rest_entries[size_t(vi)];
  return rest ? (nf + kSegment - 1) / kSegment * kSegment + rest : nf;
}

r4d_status acquire_slot(r4d_ctx* ctx, r4d_ctx::Pinned** out) {
  r4d_ctx::Pinned* slot = nullptr;
  for (r4d_ctx::Pinned* q : ctx->pinned_pool) {
    if (q->refs) continue;
    const hipError_t e = hipEventQuery(q->done);
    if (e == hipSuccess) {
      slot = q;
      break;
    }
    (void)hipGetLastError();
  }
  if (!slot) {
    auto q = std::make_unique<r4d_ctx::Pinned>();
    R4D_HIP(hipHostMalloc(reinterpret_cast<void**>(&q->host), kReadbackBytes,
                          hipHostMallocDefault));
    const hipError_t e = hipEventCreateWithFlags(&q->done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipHostFree(q->host);
      return fail(ctx, R4D_ERR_HIP, "event creation failed: %s", hipGetErrorString(e));
    }
    slot = q.release();
    ctx->pinned_pool.push_back(slot);
  }
  slot->refs = 1;
  *out = slot;
  return R4D_OK;
}

void attach_slot(RunState& r, r4d_ctx::Pinned* slot) {
  r.slot = slot;
  r.pinned = slot->host;
  r.done = slot->done;
}

r4d_status init_run(r4d_ctx* ctx, RunState& r, const Plan& p) {
  r.plan = p;
  r4d_ctx::Pinned* slot = nullptr;
  r4d_status s = acquire_slot(ctx, &slot);
  if (s != R4D_OK) return s;
  attach_slot(r, slot);
  return R4D_OK;
}

// Status of a forward from its status words: (overflow, look-back error).
r4d_status flags_status(r4d_ctx* ctx, const unsigned long long* pinned, const char* what) {
  const uint32_t* fl = reinterpret_cast<const uint32_t*>(pinned);
  if (fl[1]) return fail(ctx, R4D_ERR_HIP, "%ssort look-back did not complete", what);
  if (fl[0]) return fail(ctx, R4D_ERR_CAPACITY, "%stile lists overflowed the capacity", what);
  return R4D_OK;
}

// Reads the status words of unchecked forwards that have completed (all of
// them with wait = true) and reports the first failure among them.
r4d_status drain_unchecked(r4d_ctx* ctx, bool wait) {
  r4d_status result = R4D_OK;
  std::vector<r4d_ctx::Pinned*> keep;
  for (r4d_ctx::Pinned* q : ctx->unchecked) {
    const hipError_t e = wait ? hipEventSynchronize(q->done) : hipEventQuery(q->done);
    if (e == hipErrorNotReady) {
      (void)hipGetLastError();
      keep.push_back(q);
      continue;
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (result == R4D_OK)
        result = fail(ctx, R4D_ERR_HIP, "waiting for an earlier forward: %s", hipGetErrorString(e));
    } else if (result == R4D_OK) {
      result = flags_status(ctx, q->host, "an earlier forward whose state was not checked: ");
    }
    unref_slot(q);
  }
  ctx->unchecked.swap(keep);
  return result;
}

// Screen-space gradient components per Gaussian and render.
size_t grad_comps(const Plan& p, bool flow_grads) { return p.flow && flow_grads ? 11 : 9; }

// dLf: the flow images' gradient (flow runs; null = colour loss only).
// Densification statistics accumulated by a backward (both null: none).
struct StatsOut {
  float* accum = nullptr;
  int32_t* count = nullptr;
};

template <typename T>
r4d_status enqueue_backward(r4d_ctx* ctx, const GaussPtrs<T>& g, RunState& r, const T* dL,
                            const T* dLf, uint8_t* bwd_block, const SettingsDev& st,
                            const GradPtrs<T>& out, bool timed, hipStream_t stream,
                            StatsOut stats = StatsOut{}) {
  const Plan& p = r.plan;
  uint8_t* F = r.fixed;
  if (dLf && !p.flow) return fail(ctx, R4D_ERR_STATE, "flow gradients for a render without flow");
  const size_t nc = grad_comps(p, dLf != nullptr);
  const size_t g2_bytes = align256(size_t(p.V) * nc * size_t(p.n) * 8);
  auto* grad2d = reinterpret_cast<double*>(bwd_block);
  auto* work = reinterpret_cast<uint32_t*>(bwd_block + g2_bytes);
  R4D_HIP(fill_zero(bwd_block, g2_bytes + 256, stream));
  const RasterSaved<T> sv = saved_of<T>(r);
  R4D_TIMED(kRasterBwd,
            launch_raster_bwd<T>(at<Rec<T>>(F, r.L.recs),
                                 p.flow ? at<Vec2<T>>(F, r.L.flows) : nullptr, p.n, r.values,
                                 at<uint2>(F, r.L.ranges), slots_of(F, r.L), p.V, p.total_tiles,
                                 bwd_items(p, r.capacity), p.ts, st, p.bppt,
                                 at<T>(F, r.L.T_final), at<uint32_t>(F, r.L.n_contrib), sv, dL,
                                 dLf, grad2d, work, stream));
  if (stats.accum)
    R4D_HIP(launch_densify_stats(grad2d, int(nc), at<uint32_t>(F, r.L.dkeys), p.n_pad,
                                 slots_of(F, r.L), p.V, p.n, stats.accum, stats.count, stream));
  R4D_TIMED(kPreprocessBwd, launch_preprocess_bwd<T>(g, slots_of(F, r.L), p.V, st, grad2d,
                                                     nc == 11, p.static3d, out, stream));
  return R4D_OK;
}

size_t bwd_block_bytes(const Plan& p, uint64_t capacity) {
  return align256(size_t(p.V) * grad_comps(p, true) * size_t(p.n) * 8) +
         align256(raster_bwd_work_bytes(p.total_tiles, bwd_items(p, capacity)));
}

GaussPtrs<float> gauss_of(const r4d_gaussians* g) {
  return GaussPtrs<float>{g->n, g->sh_degree, g->means, g->log_scales, g->rotors, g->opacity,
                          g->sh};
}
GaussPtrs<double> gauss_of(const r4d_gaussians_f64* g) {
  return GaussPtrs<double>{g->n, g->sh_degree, g->means, g->log_scales, g->rotors, g->opacity,
                           g->sh};
}

template <typename T>
r4d_status check_gaussians(r4d_ctx* ctx, const GaussPtrs<T>& g) {
  if (g.n < 0 || g.deg < 0 || g.deg > 3)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid Gaussian count or SH degree");
  if (g.n > 0 && (!g.means || !g.log_scales || !g.rotors || !g.opacity || !g.sh))
    return fail(ctx, R4D_ERR_INVALID_ARG, "null Gaussian array");
  return R4D_OK;
}

// ---- plain (per-view / fused) forward: allocates, runs sized, records done
template <typename T>
r4d_status run_sized(r4d_ctx* ctx, const GaussPtrs<T>& g, const Plan& p, T* images,
                     T* flow_images, const SettingsDev& st, bool timed, hipStream_t stream,
                     std::unique_ptr<RunState>& out) {
  auto r = std::make_unique<RunState>();
  struct Guard {
    r4d_ctx* ctx;
    RunState* r;
    bool ok = false;
    ~Guard() {
      if (!ok) release_run(ctx, r);
    }
  } guard{ctx, r.get()};
  r4d_status s = init_run(ctx, *r, p);
  if (s != R4D_OK) return s;
  r->L = make_layout(p, 0);
  r->fixed = static_cast<uint8_t*>(ctx_alloc(ctx, r->L.fixed_bytes));
  if (!r->fixed)
    return fail(ctx, R4D_ERR_OOM, "device allocation of %zu bytes failed", r->L.fixed_bytes);
  if ((s = upload_meta(ctx, p, r->fixed, r->L, stream)) != R4D_OK) return s;
  if ((s = enqueue_forward<T>(ctx, g, *r, images, flow_images, st, true, timed, stream)) !=
      R4D_OK)
    return s;
  if ((s = finish_run(ctx, *r, stream)) != R4D_OK) return s;
  guard.ok = true;
  out = std::move(r);
  return R4D_OK;
}

template <typename T>
std::string fwd_graph_key(const GaussPtrs<T>& g, const void* images, const void* flows,
                          const r4d_view* views, int V, const r4d_settings& s, bool static3d) {
  char buf[640];
  snprintf(buf, sizeof(buf),
           "%zu|%d|%d|%d|%p|%p|%p|%p|%p|%p|%p|%d|%d|%d|%d|%a|%a|%a|%a|%a|%a|%a|%a|%a|%d|",
           sizeof(T), int(static3d), g.n, g.deg, (const void*)g.means, (const void*)g.log_scales,
           (const void*)g.rotors, (const void*)g.opacity, (const void*)g.sh, images, flows,
           s.tile_size,
           s.fwd_pixels_per_thread, s.bwd_pixels_per_thread, s.sort_items, s.near_plane,
           s.time_cull, s.extent_sigma, s.alpha_min, s.alpha_max, s.T_min, s.dilation,
           s.guard_band, s.front_fraction, s.front_keep);
  return std::string(buf) + view_shape_key(views, V);
}

// ---- graph forward
template <typename T>
r4d_status run_graph(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views, int V,
                     const r4d_settings& s, T* images, T* flow_images, const SettingsDev& st,
                     bool static3d, hipStream_t stream, GraphEntry** entry_out) {
  const std::string key = fwd_graph_key(g, images, flow_images, views, V, s, static3d);
  auto it = ctx->graphs.find(key);
  GraphEntry* e = it == ctx->graphs.end() ? nullptr : it->second.get();
  const Plan p = make_plan(views, V, uint32_t(g.n), g.deg, s, sizeof(T), flow_images != nullptr,
                           static3d);
  if (e && e->run.done) {
    // an overflow of an earlier replay grows the capacity (checked without waiting)
    if (hipEventQuery(e->run.done) == hipSuccess) {
      const uint32_t* fl = reinterpret_cast<const uint32_t*>(e->run.pinned);
      if (fl[0]) e->needs_grow = true;
    } else {
      (void)hipGetLastError();
    }
  }
  if (!e || e->needs_grow) {
    uint64_t cap = 0;
    if (e) {
      // the overflowed replay still counted every view's entries
      uint64_t needed = 0;
      for (int v = 0; v < V; ++v)
        needed += seg_extent(e->run.pinned[3 + 2 * v], p.slots[size_t(v)]);
      cap = std::max(e->run.capacity * 2, needed + needed / 4 + uint64_t(V) * kSegAlign);
      R4D_HIP(hipStreamSynchronize(stream));
      if (e->fwd) (void)hipGraphExecDestroy(e->fwd);
      if (e->bwd) (void)hipGraphExecDestroy(e->bwd);
      e->fwd = e->bwd = nullptr;
      e->bwd_key.clear();
      ctx_free(ctx, e->run.entries);
      ctx_free(ctx, e->run.fixed);
      ctx_free(ctx, e->bwd_block);
      e->run.fixed = e->run.entries = e->bwd_block = nullptr;
    } else {
      // size from one exact (fused) run
      std::unique_ptr<RunState> probe;
      r4d_status st_ = run_sized<T>(ctx, g, p, images, flow_images, st, false, stream, probe);
      if (st_ != R4D_OK) return st_;
      cap = probe->capacity + probe->capacity / 4 + uint64_t(V) * kSegAlign;
      R4D_HIP(hipEventSynchronize(probe->done));
      release_run(ctx, probe.get());
      auto ne = std::make_unique<GraphEntry>();
      e = ne.get();
      ctx->graphs[key] = std::move(ne);
      r4d_status s2 = init_run(ctx, e->run, p);
      if (s2 != R4D_OK) return s2;
      e->run.owns_memory = false;
    }
    if (cap >= (uint64_t(1) << 32)) cap = (uint64_t(1) << 32) - kSegAlign;
    e->needs_grow = false;
    e->run.plan = p;
    e->run.capacity = cap;
    e->run.L = make_layout(p, cap);
    e->run.fixed = static_cast<uint8_t*>(ctx_alloc(ctx, e->run.L.fixed_bytes));
    e->run.entries = static_cast<uint8_t*>(ctx_alloc(ctx, e->run.L.entries_bytes));
    if (!e->run.fixed || !e->run.entries)
      return fail(ctx, R4D_ERR_OOM, "graph buffers of %zu + %zu bytes", e->run.L.fixed_bytes,
                  e->run.L.entries_bytes);
    // capture on the context's own stream (the caller's may be the null stream)
    hipStream_t cs = ctx->capture_stream;
    R4D_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    r4d_status cst = enqueue_forward<T>(ctx, g, e->run, images, flow_images, st, false, false, cs);
    hipGraph_t graph = nullptr;
    const hipError_t end = hipStreamEndCapture(cs, &graph);
    if (cst != R4D_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cst;
    }
    R4D_HIP(end);
    const hipError_t inst = hipGraphInstantiate(&e->fwd, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    R4D_HIP(inst);
  }
  e->run.plan = p;  // camera and time of this call (uploaded below)
  r4d_status s3 = upload_meta(ctx, p, e->run.fixed, e->run.L, stream);
  if (s3 != R4D_OK) return s3;
  // each replay reports into a readback area of its own, so that the status
  // words of an earlier replay survive until whoever holds them reads them
  r4d_ctx::Pinned* slot = nullptr;
  if ((s3 = acquire_slot(ctx, &slot)) != R4D_OK) return s3;
  unref_slot(e->run.slot);
  attach_slot(e->run, slot);
  R4D_HIP(hipGraphLaunch(e->fwd, stream));
  e->generation += 1;
  if ((s3 = finish_run(ctx, e->run, stream)) != R4D_OK) return s3;
  // the sorted values sit where the captured sort left them
  *entry_out = e;
  return R4D_OK;
}

// ---- the autotuner's choices, kept across processes in a text file of lines
// "key<TAB>tile size<TAB>sort items" (path: R4D_TUNE_CACHE; unset: under
// XDG_CACHE_HOME or HOME; empty: nothing is read or written).  Keys carry the
// cache format, the device and the call shape; unreadable lines are ignored.
constexpr const char* kTuneVersion = "r4d-tune-1";

std::string tune_cache_path() {
  if (const char* e = std::getenv("R4D_TUNE_CACHE")) return std::string(e);
  const char* xdg = std::getenv("XDG_CACHE_HOME");
  if (xdg && *xdg) return std::string(xdg) + "/r4d/autotune.txt";
  const char* home = std::getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/r4d/autotune.txt";
  return std::string();
}

void load_tune_cache(r4d_ctx* ctx) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[4096];
  while (std::fgets(line, sizeof(line), f)) {
    char* tab1 = std::strchr(line, '\t');
    if (!tab1) continue;
    *tab1 = '\0';
    int ts = 0, items = -1;
    if (std::sscanf(tab1 + 1, "%d\t%d", &ts, &items) != 2) continue;
    if ((ts != 8 && ts != 16 && ts != 32) || (items != 0 && items != 8 && items != 16)) continue;
    ctx->tuned[std::string(line)] = {ts, items};  // later lines win
  }
  std::fclose(f);
}

void store_tune_cache(const std::string& key, int ts, int items) {
  const std::string path = tune_cache_path();
  if (path.empty()) return;
  // create the missing directories of the path (errors show up at fopen)
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;  // the choice still holds for this context
  std::fprintf(f, "%s\t%d\t%d\n", key.c_str(), ts, items);
  std::fclose(f);
}

// ---- autotuner: forward + backward of the call's renders (fused), each
// candidate (tile size, tile-sort keys per lane) timed twice after a warm-up.
template <typename T>
r4d_status autotune(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views, int V,
                    const r4d_settings& base, T* images, bool static3d, hipStream_t stream,
                    int* ts_out, int* items_out) {
  // Gaussian counts in half-octave buckets: a set that densification grows or
  // prunes a little keeps its choice
  const int nbucket = g.n > 0 ? int(std::floor(2.0 * std::log2(double(g.n)))) : -1;
  const std::string key = std::string(kTuneVersion) + "|" + ctx->device_tag + "|" +
                          std::to_string(sizeof(T)) + "|" + std::to_string(int(static3d)) + "|" +
                          std::to_string(nbucket) + "|" + std::to_string(g.deg) + "|" +
                          std::to_string(base.mode) + "|" + view_shape_key(views, V);
  if (!ctx->tuned_loaded) {
    load_tune_cache(ctx);
    ctx->tuned_loaded = true;
  }
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    *ts_out = it->second.first;
    *items_out = it->second.second;
    return R4D_OK;
  }
  const SettingsDev st = make_settings(base);
  uint64_t pix = 0;
  for (int v = 0; v < V; ++v) pix += uint64_t(views[v].width) * uint64_t(views[v].height);
  // a unit image gradient and scratch parameter gradients
  const size_t k3 = 3 * size_t((g.deg + 1) * (g.deg + 1));
  const size_t n = size_t(std::max(g.n, 1));
  T* dl = static_cast<T*>(ctx_alloc(ctx, 3 * pix * sizeof(T)));
  T* gbuf = static_cast<T*>(ctx_alloc(ctx, (17 + k3) * n * sizeof(T)));
  if (!dl || !gbuf) {
    ctx_free(ctx, dl);
    ctx_free(ctx, gbuf);
    return fail(ctx, R4D_ERR_OOM, "autotuner buffers");
  }
  R4D_HIP(fill_const(dl, 3 * pix, 1e-3, sizeof(T) == 8, stream));
  const GradPtrs<T> out{gbuf, gbuf + 4 * n, gbuf + 8 * n, gbuf + 16 * n, gbuf + 17 * n};
  hipEvent_t e0, e1;
  R4D_HIP(hipEventCreate(&e0));
  R4D_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_ts = 16, best_items = 16;
  r4d_status result = R4D_OK;
  for (int ts : {8, 16, 32}) {
    for (int items : {0, 16}) {
      r4d_settings s = base;
      s.tile_size = ts;
      s.sort_items = items;
      s.fwd_pixels_per_thread = s.bwd_pixels_per_thread = 0;
      const Plan p = make_plan(views, V, uint32_t(g.n), g.deg, s, sizeof(T), false, static3d);
      float total = 0.f;
      for (int rep = 0; rep < 3 && result == R4D_OK; ++rep) {
        if (rep == 1) {
          if (hipEventRecord(e0, stream) != hipSuccess) result = R4D_ERR_HIP;
        }
        std::unique_ptr<RunState> r;
        result = run_sized<T>(ctx, g, p, images, nullptr, st, false, stream, r);
        if (result != R4D_OK) break;
        uint8_t* bb = static_cast<uint8_t*>(ctx_alloc(ctx, bwd_block_bytes(p, r->capacity)));
        if (!bb) {
          release_run(ctx, r.get());
          result = fail(ctx, R4D_ERR_OOM, "autotuner buffers");
          break;
        }
        result = enqueue_backward<T>(ctx, g, *r, dl, nullptr, bb, st, out, false, stream);
        (void)hipStreamSynchronize(stream);
        ctx_free(ctx, bb);
        release_run(ctx, r.get());
      }
      if (result != R4D_OK) break;
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&total, e0, e1) != hipSuccess) {
        result = fail(ctx, R4D_ERR_HIP, "autotuner timing failed");
        break;
      }
      if (total < best) {
        best = total;
        best_ts = ts;
        best_items = items;
      }
    }
    if (result != R4D_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx_free(ctx, dl);
  ctx_free(ctx, gbuf);
  if (result != R4D_OK) return result;
  ctx->tuned[key] = {best_ts, best_items};
  store_tune_cache(key, best_ts, best_items);
  *ts_out = best_ts;
  *items_out = best_items;
  return R4D_OK;
}

// flows: null for a colour render, else the flow images ([2][H][W] per view,
// views back to back).
template <typename T>
r4d_status forward_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views, int n_views,
                        const r4d_settings* settings, T* images, T* flows, r4d_saved** saved_out,
                        hipStream_t stream, bool static3d = false) {
  if (saved_out) *saved_out = nullptr;
  if (!views || n_views < 1 || n_views > kMaxViews || !images || !valid_settings(settings))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid views, images or settings");
  r4d_status s = check_gaussians(ctx, g);
  if (s != R4D_OK) return s;
  for (int i = 0; i < n_views; ++i)
    if (!valid_view(views[i])) return fail(ctx, R4D_ERR_INVALID_ARG, "invalid view %d", i);
  if (uint64_t(round_seg(uint64_t(g.n))) * uint64_t(n_views) >= (uint64_t(1) << 32))
    return fail(ctx, R4D_ERR_CAPACITY, "%d views of %d Gaussians exceed 2^32 sort slots", n_views,
                g.n);
  R4D_HIP(hipSetDevice(ctx->device));
  if ((s = drain_unchecked(ctx, false)) != R4D_OK) return s;
  r4d_settings rs = *settings;
  if (rs.tile_size == 0) {
    int ts = 16, items = 16;
    if ((s = autotune<T>(ctx, g, views, n_views, rs, images, static3d, stream, &ts, &items)) !=
        R4D_OK)
      return s;
    rs.tile_size = ts;
    rs.sort_items = items;
  }
  const SettingsDev st = make_settings(rs);
  auto saved = std::make_unique<r4d_saved>();
  saved->ctx = ctx;
  saved->f64 = sizeof(T) == 8;
  saved->flow = flows != nullptr;
  saved->static3d = static3d;
  saved->n = g.n;
  saved->deg = g.deg;
  saved->settings = rs;
  saved->views.assign(views, views + n_views);
  const bool timed = ctx->timing && rs.mode != R4D_MODE_GRAPH;
  const bool flow = flows != nullptr;
  if (rs.mode == R4D_MODE_GRAPH) {
    GraphEntry* e = nullptr;
    if ((s = run_graph<T>(ctx, g, views, n_views, rs, images, flows, st, static3d, stream, &e)) !=
        R4D_OK)
      return s;
    saved->graph = e;
    saved->generation = e->generation;
    saved->graph_slot = e->run.slot;
    saved->graph_slot->refs += 1;
    for (int v = 0; v < n_views; ++v) saved->where.push_back({0, v});
  } else if (rs.mode == R4D_MODE_FUSED) {
    Plan p = make_plan(views, n_views, uint32_t(g.n), g.deg, rs, sizeof(T), flow, static3d);
    p.count_evals = timed && !flow;
    std::unique_ptr<RunState> r;
    if ((s = run_sized<T>(ctx, g, p, images, flows, st, timed, stream, r)) != R4D_OK) return s;
    saved->runs.push_back(std::move(r));
    for (int v = 0; v < n_views; ++v) saved->where.push_back({0, v});
  } else {
    size_t off = 0, foff = 0;
    for (int v = 0; v < n_views; ++v) {
      Plan p = make_plan(views + v, 1, uint32_t(g.n), g.deg, rs, sizeof(T), flow, static3d);
      p.count_evals = timed && !flow;
      std::unique_ptr<RunState> r;
      if ((s = run_sized<T>(ctx, g, p, images + off, flow ? flows + foff : nullptr, st, timed,
                            stream, r)) != R4D_OK) {
        for (auto& rr : saved->runs) release_run(ctx, rr.get());
        return s;
      }
      r->image_offset = off;
      r->flow_offset = foff;
      off += 3 * size_t(views[v].width) * size_t(views[v].height);
      foff += 2 * size_t(views[v].width) * size_t(views[v].height);
      saved->runs.push_back(std::move(r));
      saved->where.push_back({v, 0});
    }
  }
  if (saved_out) {
    r4d_saved* raw = saved.release();
    ctx->live_saved.insert(raw);
    *saved_out = raw;
  } else {
    // inference: the run buffers return to the cache (stream order keeps the
    // queued kernels safe); the status words are read by a later call
    for (auto& rr : saved->runs) release_run(ctx, rr.get(), true);
    if (saved->graph_slot) ctx->unchecked.push_back(saved->graph_slot);
    saved->graph_slot = nullptr;
  }
  return R4D_OK;
}

// Waits for the previous no-allocation call's runs to finish (if their status
// is still unread) and reports its sort failure; its readback area is then free.
r4d_status settle_noalloc(r4d_ctx* ctx) {
  r4d_ctx::Pinned* q = ctx->noalloc_slot;
  if (!q->refs) return R4D_OK;
  auto it = std::find(ctx->unchecked.begin(), ctx->unchecked.end(), q);
  if (it != ctx->unchecked.end()) ctx->unchecked.erase(it);
  q->refs = 0;
  R4D_HIP(hipEventSynchronize(q->done));
  return flags_status(ctx, q->host, "the previous no-allocation forward: ");
}

// Forward without saved state whose buffers all lie in the no-allocation
// region: one run of every view (fused mode) or one run per view in turn
// (per-view mode), each sized from its entry count like a plain run.
template <typename T>
r4d_status forward_noalloc_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views,
                                int n_views, const r4d_settings* settings, T* images,
                                hipStream_t stream) {
  if (!views || n_views < 1 || n_views > kMaxViews || !images || !valid_settings(settings))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid views, images or settings");
  if (settings->tile_size == 0)
    return fail(ctx, R4D_ERR_INVALID_ARG,
                "the no-allocation forward needs a tile size (the autotuner allocates)");
  if (settings->mode == R4D_MODE_GRAPH)
    return fail(ctx, R4D_ERR_INVALID_ARG, "the no-allocation forward has no graph mode");
  r4d_status s = check_gaussians(ctx, g);
  if (s != R4D_OK) return s;
  for (int i = 0; i < n_views; ++i)
    if (!valid_view(views[i])) return fail(ctx, R4D_ERR_INVALID_ARG, "invalid view %d", i);
  if (uint64_t(round_seg(uint64_t(g.n))) * uint64_t(n_views) >= (uint64_t(1) << 32))
    return fail(ctx, R4D_ERR_CAPACITY, "%d views of %d Gaussians exceed 2^32 sort slots", n_views,
                g.n);
  const bool fused = settings->mode == R4D_MODE_FUSED;
  // the per-Gaussian and per-pixel buffers must fit before anything is launched
  for (int v = 0; v < (fused ? 1 : n_views); ++v) {
    const Plan p = make_plan(fused ? views : views + v, fused ? n_views : 1, uint32_t(g.n), g.deg,
                             *settings, sizeof(T), false, false);
    const size_t fixed = align256(make_layout(p, 0).fixed_bytes);
    if (fixed >= kNoallocBytes)
      return fail(ctx, R4D_ERR_CAPACITY,
                  "%d Gaussians in %d view(s) need %zu bytes of per-Gaussian and per-pixel "
                  "buffers; the no-allocation region holds %zu",
                  g.n, p.V, fixed, kNoallocBytes);
  }
  R4D_HIP(hipSetDevice(ctx->device));
  if ((s = drain_unchecked(ctx, false)) != R4D_OK) return s;
  if ((s = settle_noalloc(ctx)) != R4D_OK) return s;
  const SettingsDev st = make_settings(*settings);
  size_t off = 0;
  for (int v = 0; v < (fused ? 1 : n_views); ++v) {
    if (v > 0) {
      // the previous view's run reads the region until it completes; its
      // status words are read before this run's readback reuses the area
      R4D_HIP(hipEventSynchronize(ctx->noalloc_slot->done));
      if ((s = flags_status(ctx, ctx->noalloc_slot->host, "")) != R4D_OK) return s;
    }
    RunState r;
    r.plan = make_plan(fused ? views : views + v, fused ? n_views : 1, uint32_t(g.n), g.deg,
                       *settings, sizeof(T), false, false);
    r.owns_memory = false;
    attach_slot(r, ctx->noalloc_slot);
    r.L = make_layout(r.plan, 0);
    const size_t fixed = align256(r.L.fixed_bytes);
    r.fixed = ctx->noalloc;
    r.entries = ctx->noalloc + fixed;
    r.entries_limit = kNoallocBytes - fixed;
    if ((s = upload_meta(ctx, r.plan, r.fixed, r.L, stream)) != R4D_OK) return s;
    if ((s = enqueue_forward<T>(ctx, g, r, images + off, nullptr, st, true, false, stream)) !=
        R4D_OK)
      return s;
    if ((s = finish_run(ctx, r, stream)) != R4D_OK) return s;
    for (int u = v; u < (fused ? n_views : v + 1); ++u)
      off += 3 * size_t(views[u].width) * size_t(views[u].height);
  }
  // the last run's status words are read by the next call (this entry point's,
  // any render call of the context, or r4d_check_pending)
  ctx->noalloc_slot->refs = 1;
  ctx->unchecked.push_back(ctx->noalloc_slot);
  return R4D_OK;
}

// Waits for the forward of a saved state and reports its overflow or sort
// failure.
r4d_status check_saved(r4d_ctx* ctx, const r4d_saved* saved) {
  if (saved->graph) {
    if (!saved->graph_slot) return fail(ctx, R4D_ERR_STATE, "saved state without readback");
    R4D_HIP(hipEventSynchronize(saved->graph_slot->done));
    saved->checked = true;
    return flags_status(ctx, saved->graph_slot->host, "");
  }
  for (const auto& r : saved->runs) {
    r4d_status s = wait_run(ctx, *r);
    if (s != R4D_OK) return s;
    if ((s = flags_status(ctx, r->pinned, "")) != R4D_OK) {
      saved->checked = true;
      return s;
    }
  }
  saved->checked = true;
  return R4D_OK;
}

bool same_view(const r4d_view& a, const r4d_view& b) {
  return a.width == b.width && a.height == b.height && a.t == b.t &&
         std::memcmp(a.world_to_cam, b.world_to_cam, sizeof(a.world_to_cam)) == 0 &&
         a.fx == b.fx && a.fy == b.fy && a.cx == b.cx && a.cy == b.cy;
}

// dLf: the flow images' gradient (null: none; needs a flow render otherwise).
template <typename T>
r4d_status backward_enqueue(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views,
                            int n_views, const r4d_settings* settings, const r4d_saved* saved,
                            const T* dL, const T* dLf, const GradPtrs<T>& out, hipStream_t stream,
                            StatsOut stats, bool static3d) {
  if (!views || n_views < 1 || !dL || !valid_settings(settings) || !saved)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid views, gradients, settings or saved state");
  r4d_status s = check_gaussians(ctx, g);
  if (s != R4D_OK) return s;
  if (g.n > 0 && (!out.means || !out.log_scales || !out.rotors || !out.opacity || !out.sh))
    return fail(ctx, R4D_ERR_INVALID_ARG, "null gradient array");
  if (saved->ctx != ctx || saved->f64 != (sizeof(T) == 8) || saved->n != g.n ||
      saved->deg != g.deg || int(saved->views.size()) != n_views ||
      settings->mode != saved->settings.mode ||
      (settings->tile_size != 0 && settings->tile_size != saved->settings.tile_size))
    return fail(ctx, R4D_ERR_STATE, "saved state does not match this backward call");
  for (int i = 0; i < n_views; ++i)
    if (!same_view(saved->views[size_t(i)], views[i]))
      return fail(ctx, R4D_ERR_STATE, "view %d differs from the forward call", i);
  if (saved->graph && saved->generation != saved->graph->generation)
    return fail(ctx, R4D_ERR_STATE, "a later graph forward of this shape reused the buffers");
  if (dLf && !saved->flow)
    return fail(ctx, R4D_ERR_STATE, "flow gradients given for a forward without flow");
  if (saved->static3d != static3d)
    return fail(ctx, R4D_ERR_STATE, "static and 4D Gaussian calls do not mix");
  R4D_HIP(hipSetDevice(ctx->device));
  if ((s = drain_unchecked(ctx, false)) != R4D_OK) return s;
  if (g.n == 0) return R4D_OK;
  const SettingsDev st = make_settings(saved->settings);
  const bool timed = ctx->timing && !saved->graph;
  if (saved->graph) {
    GraphEntry* e = saved->graph;
    char buf[320];
    snprintf(buf, sizeof(buf), "%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p", (const void*)dL,
             (const void*)dLf, (const void*)stats.accum, (const void*)stats.count,
             (const void*)out.means, (const void*)out.log_scales, (const void*)out.rotors,
             (const void*)out.opacity, (const void*)out.sh, (const void*)g.means,
             (const void*)g.log_scales, (const void*)g.rotors, (const void*)g.opacity,
             (const void*)g.sh, (const void*)e->run.fixed);
    if (!e->bwd || e->bwd_key != buf) {
      if (e->bwd) {
        R4D_HIP(hipStreamSynchronize(stream));
        (void)hipGraphExecDestroy(e->bwd);
        e->bwd = nullptr;
      }
      if (!e->bwd_block) {
        e->bwd_block = static_cast<uint8_t*>(ctx_alloc(ctx, bwd_block_bytes(e->run.plan, e->run.capacity)));
        if (!e->bwd_block) return fail(ctx, R4D_ERR_OOM, "graph backward buffers");
      }
      hipStream_t cs = ctx->capture_stream;
      R4D_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      r4d_status cst =
          enqueue_backward<T>(ctx, g, e->run, dL, dLf, e->bwd_block, st, out, false, cs, stats);
      hipGraph_t graph = nullptr;
      const hipError_t end = hipStreamEndCapture(cs, &graph);
      if (cst != R4D_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return cst;
      }
      R4D_HIP(end);
      const hipError_t inst = hipGraphInstantiate(&e->bwd, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      R4D_HIP(inst);
      e->bwd_key = buf;
    }
    R4D_HIP(hipGraphLaunch(e->bwd, stream));
    return R4D_OK;
  }
  if (saved->runs.size() == 1) {
    RunState& r = *saved->runs[0];
    uint8_t* bb = static_cast<uint8_t*>(ctx_alloc(ctx, bwd_block_bytes(r.plan, r.capacity)));
    if (!bb) return fail(ctx, R4D_ERR_OOM, "backward buffers");
    s = enqueue_backward<T>(ctx, g, r, dL + r.image_offset, dLf ? dLf + r.flow_offset : nullptr,
                            bb, st, out, timed, stream, stats);
    ctx_free(ctx, bb);
    return s;
  }
  // several runs (per-view mode): the first run writes `out`, every later run
  // writes a temporary that is added to `out`
  const size_t n = size_t(g.n);
  const size_t k3 = 3 * size_t((g.deg + 1) * (g.deg + 1));
  T* tmp = static_cast<T*>(ctx_alloc(ctx, (17 + k3) * n * sizeof(T)));
  if (!tmp) return fail(ctx, R4D_ERR_OOM, "backward buffers");
  // the five arrays back to back (static 3D Gaussians: 3, 3, 4 rows)
  const size_t rm = static3d ? 3 : 4, rl = rm, rr = static3d ? 4 : 8;
  const GradPtrs<T> gt{tmp, tmp + rm * n, tmp + (rm + rl) * n, tmp + (rm + rl + rr) * n,
                       tmp + (rm + rl + rr + 1) * n};
  for (size_t ri = 0; ri < saved->runs.size() && s == R4D_OK; ++ri) {
    RunState& r = *saved->runs[ri];
    uint8_t* bb = static_cast<uint8_t*>(ctx_alloc(ctx, bwd_block_bytes(r.plan, r.capacity)));
    if (!bb) {
      s = fail(ctx, R4D_ERR_OOM, "backward buffers");
      break;
    }
    s = enqueue_backward<T>(ctx, g, r, dL + r.image_offset, dLf ? dLf + r.flow_offset : nullptr,
                            bb, st, ri == 0 ? out : gt, timed, stream, stats);
    ctx_free(ctx, bb);
    if (s == R4D_OK && ri > 0) {
      const hipError_t e = add_grads<T>(out, tmp, n, k3, static3d, stream);
      if (e != hipSuccess) s = fail(ctx, R4D_ERR_HIP, "gradient sum: %s", hipGetErrorString(e));
    }
  }
  ctx_free(ctx, tmp);
  return s;
}

// The backward is enqueued first, then the forward's status words are read
// (the forward precedes the backward on the stream, so the device stays busy
// while the host waits): gradients of a forward whose tile lists overflowed or
// whose sort failed are reported as an error, not returned as zeros.
template <typename T>
r4d_status backward_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const r4d_view* views,
                         int n_views, const r4d_settings* settings, const r4d_saved* saved,
                         const T* dL, const T* dLf, const GradPtrs<T>& out, hipStream_t stream,
                         StatsOut stats = StatsOut{}, bool static3d = false) {
  r4d_status s = backward_enqueue<T>(ctx, g, views, n_views, settings, saved, dL, dLf, out, stream,
                                     stats, static3d);
  if (s != R4D_OK) return s;
  return check_saved(ctx, saved);
}

template <typename T>
r4d_status consistency_impl(r4d_ctx* ctx, const GaussPtrs<T>& g, const int32_t* neighbours,
                            int32_t k, T weight, T* loss, T* grad_rotors, T* grad_log_scales,
                            void* stream) {
  if (g.n < 2 || k < 1 || k >= g.n || !g.rotors || !g.log_scales || !neighbours)
    return fail(ctx, R4D_ERR_INVALID_ARG, "need n >= 2, 1 <= k < n, rotors, log_scales, neighbours");
  if ((grad_rotors == nullptr) != (grad_log_scales == nullptr))
    return fail(ctx, R4D_ERR_INVALID_ARG, "give both gradient arrays or neither");
  if (uint64_t(g.n) * uint64_t(k) >= (uint64_t(1) << 31))
    return fail(ctx, R4D_ERR_CAPACITY, "n * k must stay below 2^31");
  R4D_HIP(hipSetDevice(ctx->device));
  void* temp = ctx_alloc(ctx, consistency_temp_bytes<T>(uint32_t(g.n)));
  if (!temp) return fail(ctx, R4D_ERR_OOM, "consistency-loss buffers");
  const hipError_t e = launch_consistency<T>(g, neighbours, k, weight, loss, grad_rotors,
                                             grad_log_scales, temp,
                                             static_cast<hipStream_t>(stream));
  ctx_free(ctx, temp);
  if (e != hipSuccess)
    return fail(ctx, R4D_ERR_HIP, "consistency-loss launch: %s", hipGetErrorString(e));
  return R4D_OK;
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
  s->mode = R4D_MODE_PER_VIEW;
  s->sort_items = 0;
  s->front_fraction = 0.1f;
  s->front_keep = 1024;
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
  auto ctx = std::make_unique<r4d_ctx>();
  ctx->device = device;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      char tag[320];
      snprintf(tag, sizeof(tag), "%s:%d", prop.gcnArchName, prop.multiProcessorCount);
      ctx->device_tag = tag;
    } else {
      (void)hipGetLastError();
      ctx->device_tag = "unknown";
    }
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->readback), 2 * kMaxViews * 8,
                    hipHostMallocDefault) != hipSuccess)
    return R4D_ERR_OOM;
  if (hipMalloc(reinterpret_cast<void**>(&ctx->l1_partials),
                l1_partials_floats() * sizeof(float)) != hipSuccess) {
    (void)hipHostFree(ctx->readback);
    return R4D_ERR_OOM;
  }
  ctx->ring.resize(8);
  const size_t stage_bytes = sizeof(ViewSlot) * kMaxViews + sizeof(SegTable);
  for (auto& s : ctx->ring) {
    if (hipHostMalloc(&s.host, stage_bytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      r4d_destroy(ctx.release());
      return R4D_ERR_OOM;
    }
  }
  if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    r4d_destroy(ctx.release());
    return R4D_ERR_HIP;
  }
  // the no-allocation forward's region (this device's copy) and readback area
  if (noalloc_region(device, &ctx->noalloc) != hipSuccess) {
    (void)hipGetLastError();
    r4d_destroy(ctx.release());
    return R4D_ERR_HIP;
  }
  ctx->noalloc_slot = new r4d_ctx::Pinned();
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->noalloc_slot->host), kReadbackBytes,
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->noalloc_slot->done, hipEventDisableTiming) != hipSuccess) {
    r4d_destroy(ctx.release());
    return R4D_ERR_OOM;
  }
  ctx->unchecked.reserve(64);
  *out = ctx.release();
  return R4D_OK;
}

void r4d_destroy(r4d_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  // saved states that outlive the context keep only their host struct
  for (r4d_saved* sv : ctx->live_saved) {
    for (auto& r : sv->runs) {
      r->owns_memory = false;
      release_run(ctx, r.get());
    }
    sv->runs.clear();
    sv->graph = nullptr;
    sv->graph_slot = nullptr;
    sv->ctx = nullptr;
  }
  ctx->live_saved.clear();
  for (auto& kv : ctx->graphs) {
    GraphEntry* e = kv.second.get();
    if (e->fwd) (void)hipGraphExecDestroy(e->fwd);
    if (e->bwd) (void)hipGraphExecDestroy(e->bwd);
    e->run.owns_memory = false;
    release_run(ctx, &e->run);
  }
  ctx->graphs.clear();
  for (auto& kv : ctx->block_size) (void)hipFree(kv.first);
  for (auto& p : ctx->pending) ctx->event_pool.push_back({p.start, p.stop});
  for (auto& e : ctx->event_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto& s : ctx->ring) {
    if (s.host) (void)hipHostFree(s.host);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  for (r4d_ctx::Pinned* q : ctx->pinned_pool) {
    (void)hipHostFree(q->host);
    (void)hipEventDestroy(q->done);
    delete q;
  }
  ctx->pinned_pool.clear();
  if (ctx->noalloc_slot) {
    if (ctx->noalloc_slot->host) (void)hipHostFree(ctx->noalloc_slot->host);
    if (ctx->noalloc_slot->done) (void)hipEventDestroy(ctx->noalloc_slot->done);
    delete ctx->noalloc_slot;
    ctx->noalloc_slot = nullptr;
  }
  ctx->unchecked.clear();
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  if (ctx->readback) (void)hipHostFree(ctx->readback);
  if (ctx->l1_partials) (void)hipFree(ctx->l1_partials);
  delete ctx;
}

r4d_status r4d_render_forward(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                              int n_views, const r4d_settings* settings, float* images,
                              r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return forward_impl<float>(ctx, gauss_of(g), views, n_views, settings, images, nullptr, saved,
                             static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_forward_noalloc(r4d_ctx* ctx, const r4d_gaussians* g,
                                      const r4d_view* views, int n_views,
                                      const r4d_settings* settings, float* images, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return forward_noalloc_impl<float>(ctx, gauss_of(g), views, n_views, settings, images,
                                     static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_forward_flow(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                                   int n_views, const r4d_settings* settings, float* images,
                                   float* flows, r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  if (!flows) return fail(ctx, R4D_ERR_INVALID_ARG, "null flow images");
  return forward_impl<float>(ctx, gauss_of(g), views, n_views, settings, images, flows, saved,
                             static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_forward_flow_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                       const r4d_view* views, int n_views,
                                       const r4d_settings* settings, double* images,
                                       double* flows, r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  if (!flows) return fail(ctx, R4D_ERR_INVALID_ARG, "null flow images");
  return forward_impl<double>(ctx, gauss_of(g), views, n_views, settings, images, flows, saved,
                              static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_forward_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                  const r4d_view* views, int n_views,
                                  const r4d_settings* settings, double* images,
                                  r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return forward_impl<double>(ctx, gauss_of(g), views, n_views, settings, images, nullptr, saved,
                              static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                               int n_views, const r4d_settings* settings,
                               const r4d_saved* saved, const float* dL_dimages, r4d_grads* out,
                               void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GradPtrs<float> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<float>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages,
                              nullptr, o, static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward_flow(r4d_ctx* ctx, const r4d_gaussians* g, const r4d_view* views,
                                    int n_views, const r4d_settings* settings,
                                    const r4d_saved* saved, const float* dL_dimages,
                                    const float* dL_dflows, r4d_grads* out, void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  if (!dL_dflows) return fail(ctx, R4D_ERR_INVALID_ARG, "null flow gradient");
  const GradPtrs<float> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<float>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages,
                              dL_dflows, o, static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward_flow_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                        const r4d_view* views, int n_views,
                                        const r4d_settings* settings, const r4d_saved* saved,
                                        const double* dL_dimages, const double* dL_dflows,
                                        r4d_grads_f64* out, void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  if (!dL_dflows) return fail(ctx, R4D_ERR_INVALID_ARG, "null flow gradient");
  const GradPtrs<double> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<double>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages,
                               dL_dflows, o, static_cast<hipStream_t>(stream));
}

r4d_status r4d_render_backward_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                   const r4d_view* views, int n_views,
                                   const r4d_settings* settings, const r4d_saved* saved,
                                   const double* dL_dimages, r4d_grads_f64* out, void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GradPtrs<double> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<double>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages,
                               nullptr, o, static_cast<hipStream_t>(stream));
}

r4d_status r4d_knn4d(r4d_ctx* ctx, const float* means, int32_t n, int32_t k,
                     float spatial_scale, float temporal_scale, int32_t* neighbours,
                     void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!means || !neighbours) return fail(ctx, R4D_ERR_INVALID_ARG, "null argument");
  if (n < 2 || k < 1 || k > 32 || k >= n)
    return fail(ctx, R4D_ERR_INVALID_ARG, "need n >= 2 and 1 <= k <= min(32, n - 1)");
  if (!(spatial_scale > 0.f) || !(temporal_scale > 0.f) || !std::isfinite(spatial_scale) ||
      !std::isfinite(temporal_scale))
    return fail(ctx, R4D_ERR_INVALID_ARG, "scene scales must be positive and finite");
  if (uint64_t(n) * uint64_t(k) >= (uint64_t(1) << 31))
    return fail(ctx, R4D_ERR_CAPACITY, "n * k must stay below 2^31");
  R4D_HIP(hipSetDevice(ctx->device));
  const float inv_s = float(1.0 / double(spatial_scale));
  const float inv_t = float(1.0 / double(temporal_scale));
  void* temp = ctx_alloc(ctx, knn4d_temp_bytes(uint32_t(n)));
  if (!temp) return fail(ctx, R4D_ERR_OOM, "KNN buffers");
  const hipError_t e = launch_knn4d(means, uint32_t(n), k, inv_s, inv_t, neighbours, temp,
                                    static_cast<hipStream_t>(stream));
  ctx_free(ctx, temp);
  if (e != hipSuccess) return fail(ctx, R4D_ERR_HIP, "KNN launch: %s", hipGetErrorString(e));
  return R4D_OK;
}


r4d_status r4d_consistency4d_loss_grad(r4d_ctx* ctx, const r4d_gaussians* g,
                                       const int32_t* neighbours, int32_t k, float weight,
                                       float* loss, r4d_grads* grads, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return consistency_impl<float>(ctx, gauss_of(g), neighbours, k, weight, loss,
                                 grads ? grads->rotors : nullptr,
                                 grads ? grads->log_scales : nullptr, stream);
}

r4d_status r4d_consistency4d_loss_grad_f64(r4d_ctx* ctx, const r4d_gaussians_f64* g,
                                           const int32_t* neighbours, int32_t k, double weight,
                                           double* loss, r4d_grads_f64* grads, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  return consistency_impl<double>(ctx, gauss_of(g), neighbours, k, weight, loss,
                                  grads ? grads->rotors : nullptr,
                                  grads ? grads->log_scales : nullptr, stream);
}

void r4d_default_adam_config(r4d_adam_config* c) {
  if (!c) return;
  c->lr_means_init = 1.6e-4f;
  c->lr_means_final = 1.6e-6f;
  c->lr_means_steps = 30000;
  c->lr_log_scales = 5e-3f;
  c->lr_rotors = 1e-3f;
  c->lr_opacity = 0.05f;
  c->lr_sh_dc = 2.5e-3f;
  c->lr_sh_rest = 2.5e-3f / 20.0f;
  c->beta1 = 0.9f;
  c->beta2 = 0.999f;
  c->eps = 1e-15f;
}

r4d_status r4d_adam_step(r4d_ctx* ctx, const r4d_train_state* st, const r4d_grads* grads,
                         const r4d_adam_config* cfg, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!st || !grads || !cfg) return fail(ctx, R4D_ERR_INVALID_ARG, "null argument");
  if (st->n < 0 || st->sh_degree < 0 || st->sh_degree > 3)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid Gaussian count or SH degree");
  if (st->n == 0) return R4D_OK;
  if (!st->means || !st->log_scales || !st->rotors || !st->opacity || !st->sh ||
      !st->opacity_logit || !st->adam_m || !st->adam_v || !st->step || !grads->means ||
      !grads->log_scales || !grads->rotors || !grads->opacity || !grads->sh)
    return fail(ctx, R4D_ERR_INVALID_ARG, "null array in the train state or gradients");
  if (!(cfg->lr_means_init > 0.f) || !(cfg->lr_means_final > 0.f) || !(cfg->beta1 >= 0.f) ||
      !(cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f) || !(cfg->beta2 < 1.f) || !(cfg->eps >= 0.f))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid Adam settings");
  const uint64_t n = uint64_t(st->n);
  const uint64_t k3 = 3 * uint64_t((st->sh_degree + 1) * (st->sh_degree + 1));
  AdamGroups G{};
  float* ps[5] = {st->means, st->log_scales, st->rotors, st->opacity, st->sh};
  const float* gs[5] = {grads->means, grads->log_scales, grads->rotors, grads->opacity, grads->sh};
  const uint64_t rows[5] = {4, 4, 8, 1, k3};
  uint64_t off = 0;
  for (int q = 0; q < 5; ++q) {
    G.p[q] = ps[q];
    G.g[q] = gs[q];
    G.off[q] = off;
    off += rows[q] * n;
  }
  G.off[5] = off;
  G.n = uint32_t(n);
  const AdamConfig c{cfg->lr_means_init, cfg->lr_means_final, cfg->lr_means_steps,
                     cfg->lr_log_scales, cfg->lr_rotors,      cfg->lr_opacity,
                     cfg->lr_sh_dc,      cfg->lr_sh_rest,     cfg->beta1,
                     cfg->beta2,         cfg->eps};
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(launch_adam(G, st->opacity_logit, st->adam_m, st->adam_v, st->step, c,
                      static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_train_state_init(r4d_ctx* ctx, const r4d_train_state* st, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!st || !st->step || st->n < 0 || st->sh_degree < 0 || st->sh_degree > 3 ||
      (st->n > 0 && (!st->opacity || !st->opacity_logit || !st->adam_m || !st->adam_v)))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid optimiser state");
  const uint64_t n = uint64_t(st->n);
  const uint64_t k = uint64_t(st->sh_degree + 1) * uint64_t(st->sh_degree + 1);
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(launch_state_init(uint32_t(n), n * (17 + 3 * k), st->opacity, st->opacity_logit,
                            st->adam_m, st->adam_v, st->step, static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_opacity_reset(r4d_ctx* ctx, const r4d_train_state* st, float cap, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!st || !st->opacity_logit || !st->opacity || !st->adam_m || !st->adam_v || st->n < 0 ||
      st->sh_degree < 0 || st->sh_degree > 3 || !(cap > 0.f) || !(cap < 1.f))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid opacity reset arguments");
  const uint64_t n = uint64_t(st->n);
  const uint64_t op_off = 16 * n;  // after means, log_scales, rotors
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(launch_opacity_reset(uint32_t(n), cap, st->opacity_logit, st->opacity,
                               st->adam_m + op_off, st->adam_v + op_off,
                               static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_entropy_loss_grad(r4d_ctx* ctx, const float* opacity, int32_t n, float weight,
                                 float* loss, float* grad_opacity, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (n < 0 || (n > 0 && !opacity)) return fail(ctx, R4D_ERR_INVALID_ARG, "invalid entropy arguments");
  if (n == 0) return R4D_OK;
  R4D_HIP(hipSetDevice(ctx->device));
  void* temp = ctx_alloc(ctx, entropy_temp_bytes(uint32_t(n)));
  if (!temp) return fail(ctx, R4D_ERR_OOM, "entropy buffers");
  const hipError_t e = launch_entropy(opacity, uint32_t(n), weight, loss, grad_opacity, temp,
                                      static_cast<hipStream_t>(stream));
  ctx_free(ctx, temp);
  if (e != hipSuccess) return fail(ctx, R4D_ERR_HIP, "entropy launch: %s", hipGetErrorString(e));
  return R4D_OK;
}

r4d_status r4d_render_backward_stats(r4d_ctx* ctx, const r4d_gaussians* g,
                                     const r4d_view* views, int n_views,
                                     const r4d_settings* settings, const r4d_saved* saved,
                                     const float* dL_dimages, const float* dL_dflows,
                                     r4d_grads* out, float* grad_accum, int32_t* vis_count,
                                     void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  if (g->n > 0 && (!grad_accum || !vis_count))
    return fail(ctx, R4D_ERR_INVALID_ARG, "null statistics array");
  const GradPtrs<float> o{out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  return backward_impl<float>(ctx, gauss_of(g), views, n_views, settings, saved, dL_dimages,
                              dL_dflows, o, static_cast<hipStream_t>(stream),
                              StatsOut{grad_accum, vis_count});
}

void r4d_default_densify_config(r4d_densify_config* c) {
  if (!c) return;
  c->grad_threshold = 2e-4f;
  c->size_threshold = 0.01f;
  c->min_opacity = 0.005f;
  c->max_size = 0.0f;
}

r4d_status r4d_densify(r4d_ctx* ctx, const r4d_train_state* in, const float* grad_accum,
                       const int32_t* vis_count, const float* normals,
                       const r4d_densify_config* cfg, const r4d_train_state* out, int32_t* n_out,
                       void* stream_) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!in || !out || !cfg || !n_out || !grad_accum || !vis_count || !normals)
    return fail(ctx, R4D_ERR_INVALID_ARG, "null argument");
  if (in->n < 0 || in->sh_degree < 0 || in->sh_degree > 3 || out->sh_degree != in->sh_degree ||
      out->n < 0)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid Gaussian counts or SH degrees");
  if (!(cfg->grad_threshold >= 0.f) || !(cfg->size_threshold > 0.f) || !(cfg->max_size >= 0.f) ||
      !std::isfinite(cfg->min_opacity))
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid densification settings");
  const float* pin[5] = {in->means, in->log_scales, in->rotors, in->opacity, in->sh};
  float* pout[5] = {out->means, out->log_scales, out->rotors, out->opacity, out->sh};
  for (int q = 0; q < 5; ++q)
    if ((in->n > 0 && !pin[q]) || (out->n > 0 && !pout[q]))
      return fail(ctx, R4D_ERR_INVALID_ARG, "null parameter array");
  if ((in->n > 0 && (!in->opacity_logit || !in->adam_m || !in->adam_v || !in->step)) ||
      (out->n > 0 && (!out->opacity_logit || !out->adam_m || !out->adam_v)) || !out->step)
    return fail(ctx, R4D_ERR_INVALID_ARG, "null optimiser array");
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  R4D_HIP(hipSetDevice(ctx->device));
  *n_out = 0;
  if (in->n == 0) return R4D_OK;
  const uint32_t k3 = 3 * uint32_t((in->sh_degree + 1) * (in->sh_degree + 1));
  DensifyArgs d{};
  d.n_in = uint32_t(in->n);
  d.log_scales = in->log_scales;
  d.opacity = in->opacity;
  d.accum = grad_accum;
  d.count = vis_count;
  d.normals = normals;
  d.grad_threshold = cfg->grad_threshold;
  d.size_log = float(std::log(double(cfg->size_threshold)));
  d.min_opacity = cfg->min_opacity;
  d.has_big = cfg->max_size > 0.f ? 1 : 0;
  d.big_log = d.has_big ? float(std::log(double(cfg->max_size))) : 0.f;
  d.shrink = float(std::log(1.6));
  const uint32_t rows[5] = {4, 4, 8, 1, k3};
  for (int q = 0; q < 5; ++q) {
    d.pin[q] = pin[q];
    d.pout[q] = pout[q];
    d.rows[q] = rows[q];
  }
  d.logit_in = in->opacity_logit;
  d.logit_out = out->opacity_logit;
  d.m_in = in->adam_m;
  d.v_in = in->adam_v;
  d.m_out = out->adam_m;
  d.v_out = out->adam_v;
  void* temp = ctx_alloc(ctx, densify_temp_bytes(d.n_in));
  if (!temp) return fail(ctx, R4D_ERR_OOM, "densification buffers");
  struct Free {
    r4d_ctx* c;
    void* p;
    ~Free() { ctx_free(c, p); }
  } guard{ctx, temp};
  // the three totals come back through the context's pinned read-back words
  uint32_t* totals = reinterpret_cast<uint32_t*>(ctx->readback);
  R4D_HIP(densify_count(d, temp, totals, stream));
  R4D_HIP(hipStreamSynchronize(stream));
  const uint64_t total = uint64_t(totals[0]) + totals[1] + totals[2];
  const uint32_t keep = totals[0], clone = totals[1];
  if (total > uint64_t(out->n)) {
    *n_out = int32_t(total);
    return fail(ctx, R4D_ERR_CAPACITY, "densification makes %llu Gaussians, capacity %d",
                (unsigned long long)total, out->n);
  }
  *n_out = int32_t(total);
  R4D_HIP(hipMemcpyAsync(out->step, in->step, sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
  if (total == 0) return R4D_OK;
  R4D_HIP(densify_scatter(d, temp, keep, clone, uint32_t(total), stream));
  return R4D_OK;
}

r4d_status r4d_render_forward_3d(r4d_ctx* ctx, const r4d_gaussians3d* g, const r4d_view* views,
                                 int n_views, const r4d_settings* settings, float* images,
                                 r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GaussPtrs<float> gp{g->n, g->sh_degree, g->means, g->log_scales, g->quats, g->opacity,
                            g->sh};
  return forward_impl<float>(ctx, gp, views, n_views, settings, images, nullptr, saved,
                             static_cast<hipStream_t>(stream), true);
}

r4d_status r4d_render_forward_3d_f64(r4d_ctx* ctx, const r4d_gaussians3d_f64* g,
                                     const r4d_view* views, int n_views,
                                     const r4d_settings* settings, double* images,
                                     r4d_saved** saved, void* stream) {
  if (!ctx || !g) return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GaussPtrs<double> gp{g->n, g->sh_degree, g->means, g->log_scales, g->quats, g->opacity,
                             g->sh};
  return forward_impl<double>(ctx, gp, views, n_views, settings, images, nullptr, saved,
                              static_cast<hipStream_t>(stream), true);
}

r4d_status r4d_render_backward_3d(r4d_ctx* ctx, const r4d_gaussians3d* g, const r4d_view* views,
                                  int n_views, const r4d_settings* settings,
                                  const r4d_saved* saved, const float* dL_dimages,
                                  r4d_grads3d* out, void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GaussPtrs<float> gp{g->n, g->sh_degree, g->means, g->log_scales, g->quats, g->opacity,
                            g->sh};
  const GradPtrs<float> o{out->means, out->log_scales, out->quats, out->opacity, out->sh};
  return backward_impl<float>(ctx, gp, views, n_views, settings, saved, dL_dimages, nullptr, o,
                              static_cast<hipStream_t>(stream), StatsOut{}, true);
}

r4d_status r4d_render_backward_3d_f64(r4d_ctx* ctx, const r4d_gaussians3d_f64* g,
                                      const r4d_view* views, int n_views,
                                      const r4d_settings* settings, const r4d_saved* saved,
                                      const double* dL_dimages, r4d_grads3d_f64* out,
                                      void* stream) {
  if (!ctx || !g || !out)
    return ctx ? fail(ctx, R4D_ERR_INVALID_ARG, "null argument") : R4D_ERR_INVALID_ARG;
  const GaussPtrs<double> gp{g->n, g->sh_degree, g->means, g->log_scales, g->quats, g->opacity,
                             g->sh};
  const GradPtrs<double> o{out->means, out->log_scales, out->quats, out->opacity, out->sh};
  return backward_impl<double>(ctx, gp, views, n_views, settings, saved, dL_dimages, nullptr, o,
                               static_cast<hipStream_t>(stream), StatsOut{}, true);
}

void r4d_saved_release(r4d_saved* saved) {
  if (!saved) return;
  if (saved->ctx) {  // null once the context has been destroyed
    // status words nobody has read are reported by the context's next call
    const bool unchecked = !saved->checked;
    for (auto& r : saved->runs) release_run(saved->ctx, r.get(), unchecked);
    if (saved->graph_slot) {
      if (unchecked)
        saved->ctx->unchecked.push_back(saved->graph_slot);
      else
        unref_slot(saved->graph_slot);
    }
    saved->graph_slot = nullptr;
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
  R4D_HIP(launch_l1_grad(image, target, count, dL_dimage, loss, ctx->l1_partials,
                         static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_l1_loss_grad_views(r4d_ctx* ctx, const float* images, const float* targets,
                                  const r4d_view* views, int n_views, float* dL_dimages,
                                  float* loss, void* stream) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  if (!views || n_views < 1 || n_views > kMaxViews || !images || !targets || !dL_dimages)
    return fail(ctx, R4D_ERR_INVALID_ARG, "invalid L1 arguments");
  L1Views lv{};
  lv.n_views = n_views;
  int64_t off = 0;
  for (int v = 0; v < n_views; ++v) {
    if (!valid_view(views[v])) return fail(ctx, R4D_ERR_INVALID_ARG, "invalid view %d", v);
    lv.base[v] = off;
    lv.count[v] = 3 * int64_t(views[v].width) * int64_t(views[v].height);
    off += lv.count[v];
  }
  lv.base[n_views] = off;
  R4D_HIP(hipSetDevice(ctx->device));
  R4D_HIP(launch_l1_grad_views(images, targets, lv, dL_dimages, loss, ctx->l1_partials,
                               static_cast<hipStream_t>(stream)));
  return R4D_OK;
}

r4d_status r4d_saved_check(const r4d_saved* saved) {
  if (!saved || !saved->ctx) return R4D_ERR_INVALID_ARG;
  r4d_ctx* ctx = saved->ctx;
  R4D_HIP(hipSetDevice(ctx->device));
  return check_saved(ctx, saved);
}

r4d_status r4d_check_pending(r4d_ctx* ctx) {
  if (!ctx) return R4D_ERR_INVALID_ARG;
  R4D_HIP(hipSetDevice(ctx->device));
  return drain_unchecked(ctx, true);
}

r4d_status r4d_saved_config(const r4d_saved* saved, int32_t* tile_size, int32_t* sort_items,
                            int32_t* mode) {
  if (!saved) return R4D_ERR_INVALID_ARG;
  if (tile_size) *tile_size = saved->settings.tile_size;
  if (sort_items) *sort_items = saved->settings.sort_items;
  if (mode) *mode = saved->settings.mode;
  return R4D_OK;
}

r4d_status r4d_saved_stats(const r4d_saved* saved, int view, int64_t* n_visible, int64_t* n_dup,
                           int32_t* tiles_x, int32_t* tiles_y) {
  if (!saved || !saved->ctx || view < 0 || view >= int(saved->views.size()))
    return R4D_ERR_INVALID_ARG;
  if (saved->graph && saved->generation != saved->graph->generation) return R4D_ERR_STATE;
  const auto [ri, vi] = saved->where[size_t(view)];
  RunState* r = saved->run_of(ri);
  r4d_status s = wait_run(saved->ctx, *r);
  if (s != R4D_OK) return s;
  if (n_visible) *n_visible = int64_t(r->n_visible[size_t(vi)]);
  if (n_dup) *n_dup = int64_t(r->n_dup[size_t(vi)]);
  if (tiles_x) *tiles_x = r->plan.slots[size_t(vi)].v.tiles_x;
  if (tiles_y) *tiles_y = r->plan.slots[size_t(vi)].v.tiles_y;
  return R4D_OK;
}

r4d_status r4d_saved_front_stats(const r4d_saved* saved, int view, int64_t* n_front,
                                 int64_t* n_values, int64_t* rest_tiles, int64_t* rest_entries) {
  if (!saved || !saved->ctx || view < 0 || view >= int(saved->views.size()))
    return R4D_ERR_INVALID_ARG;
  if (saved->graph && saved->generation != saved->graph->generation) return R4D_ERR_STATE;
  const auto [ri, vi] = saved->where[size_t(view)];
  RunState* r = saved->run_of(ri);
  r4d_status s = wait_run(saved->ctx, *r);
  if (s != R4D_OK) return s;
  if (n_front) *n_front = int64_t(r->n_front[size_t(vi)]);
  if (n_values) *n_values = int64_t(values_count(*r, vi));
  if (rest_tiles) *rest_tiles = int64_t(r->rest_tiles[size_t(vi)]);
  if (rest_entries) *rest_entries = int64_t(r->rest_entries[size_t(vi)]);
  return R4D_OK;
}

r4d_status r4d_saved_copy(const r4d_saved* saved, int view, int buffer, void* dst, size_t bytes,
                          void* stream_) {
  if (!saved || !saved->ctx || view < 0 || view >= int(saved->views.size()) || !dst)
    return R4D_ERR_INVALID_ARG;
  r4d_ctx* ctx = saved->ctx;
  if (saved->graph && saved->generation != saved->graph->generation) return R4D_ERR_STATE;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  const auto [ri, vi] = saved->where[size_t(view)];
  RunState* r = saved->run_of(ri);
  r4d_status s = wait_run(ctx, *r);
  if (s != R4D_OK) return s;
  const Plan& p = r->plan;
  const ViewSlot& sl = p.slots[size_t(vi)];
  const size_t scal = saved->f64 ? 8 : 4;
  const size_t n = size_t(saved->n);
  const size_t hw = size_t(sl.v.W) * size_t(sl.v.H);
  const size_t ntiles = size_t(sl.v.tiles_x) * size_t(sl.v.tiles_y);
  uint8_t* F = r->fixed;
  const void* src = nullptr;
  size_t need = 0;
  SegTable tseg{};
  switch (buffer) {
    case R4D_BUF_RECORDS: src = F + r->L.recs + size_t(vi) * n * 12 * scal; need = n * 12 * scal; break;
    case R4D_BUF_RECT: src = F + r->L.rects + size_t(vi) * n * 8; need = n * 8; break;
    case R4D_BUF_DEPTHKEY: src = F + r->L.dkeys + size_t(vi) * size_t(p.n_pad) * 4; need = n * 4; break;
    case R4D_BUF_VALUES:
    case R4D_BUF_RANGES: {
      R4D_HIP(hipSetDevice(ctx->device));
      R4D_HIP(hipMemcpy(&tseg, tseg_of(F, r->L, p.V), sizeof(SegTable), hipMemcpyDeviceToHost));
      if (buffer == R4D_BUF_VALUES) {
        src = r->values + tseg.start[vi];
        need = size_t(values_count(*r, vi)) * 4;
      } else {
        need = ntiles * 8;
      }
      break;
    }
    case R4D_BUF_REST:
      R4D_HIP(hipSetDevice(ctx->device));
      R4D_HIP(hipMemcpy(&tseg, tseg_of(F, r->L, p.V), sizeof(SegTable), hipMemcpyDeviceToHost));
      need = ntiles * 8;
      break;
    case R4D_BUF_TFINAL: src = F + r->L.T_final + size_t(sl.pix_base) * scal; need = hw * scal; break;
    case R4D_BUF_NCONTRIB: src = F + r->L.n_contrib + size_t(sl.pix_base) * 4; need = hw * 4; break;
    case R4D_BUF_FLOW:
      if (!p.flow) return fail(ctx, R4D_ERR_STATE, "the forward rendered no flow");
      src = F + r->L.flows + size_t(vi) * n * 2 * scal;
      need = n * 2 * scal;
      break;
    case R4D_BUF_NEVAL:
    case R4D_BUF_NBLEND:
      if (!p.count_evals) return fail(ctx, R4D_ERR_STATE, "evaluation counts need timing enabled");
      // (evaluated, blended) pairs per pixel
      src = F + r->L.n_eval + size_t(sl.pix_base) * 8 + (buffer == R4D_BUF_NBLEND ? 4 : 0);
      need = hw * 4;
      break;
    default: return fail(ctx, R4D_ERR_INVALID_ARG, "unknown buffer id %d", buffer);
  }
  if (bytes != need)
    return fail(ctx, R4D_ERR_INVALID_ARG, "buffer %d needs %zu bytes, got %zu", buffer, need,
                bytes);
  if (need == 0) return R4D_OK;
  R4D_HIP(hipSetDevice(ctx->device));
  if (buffer == R4D_BUF_RANGES || buffer == R4D_BUF_REST) {
    R4D_HIP(copy_ranges_rebased(
        at<uint2>(F, buffer == R4D_BUF_RANGES ? r->L.ranges : r->L.rest) + sl.tile_base,
        uint32_t(ntiles), tseg.start[vi], static_cast<uint2*>(dst), stream));
    return R4D_OK;
  }
  if (buffer == R4D_BUF_NEVAL || buffer == R4D_BUF_NBLEND) {
    R4D_HIP(hipMemcpy2DAsync(dst, 4, src, 8, 4, hw, hipMemcpyDeviceToDevice, stream));
    return R4D_OK;
  }
  R4D_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, stream));
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
