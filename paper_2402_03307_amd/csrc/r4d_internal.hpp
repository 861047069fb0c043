// Internal launch interface between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gauss_math.hpp"

namespace r4d {

// Device pointers of a Gaussian set in SoA layout (see r4d.h).
template <typename T>
struct GaussPtrs {
  int n, deg;
  const T* means;
  const T* log_scales;
  const T* rotors;
  const T* opacity;
  const T* sh;
};

template <typename T>
struct GradPtrs {
  T* means;
  T* log_scales;
  T* rotors;
  T* opacity;
  T* sh;
};

// Bounding box of the tiles a Gaussian is listed in: tile x0, y0, x1, y1 (x1, y1
// exclusive); inside it, the listed tiles of each row are the run of columns
// row_span (tileset.hpp) gives.
struct Rect16 {
  uint16_t x0, y0, x1, y1;
};

// ---- several renders in one launch
constexpr int kMaxViews = 64;      // renders per call
constexpr uint32_t kSegAlign = 4096;  // segment starts of the segmented sorts

// Device-side description of one render of a batch.
struct ViewSlot {
  ViewDev v;
  uint32_t tile_base;   // index of the render's first tile among all tiles of the batch
  uint64_t pix_base;    // index of its first pixel among all pixels of the batch
  // front lists (front.hpp): depth cut fraction x 65536 (0: whole lists), the
  // render's keep bitmap (word offset) and cover grid (int offset,
  // (tiles_y + 1) x (tiles_x + 1))
  uint32_t front16;
  uint32_t keep_base;
  uint32_t cover_base;
};

// Per-render state of the front lists: where the rest area starts (absolute
// list position, a multiple of kSegment) and ends, the rest entries taken so
// far (each tile's share rounded up to kSegment), the tiles that took one,
// and the front entries.  Zeroed with the run's counters; app_base, app_end
// and n_front are set by the count scan.
struct FrontTable {
  uint32_t app_base[kMaxViews];
  uint32_t app_end[kMaxViews];
  uint32_t cursor[kMaxViews];
  uint32_t rest_tiles[kMaxViews];
  uint32_t n_front[kMaxViews];
  uint32_t queued;  // tiles the forward's main pass left to its rest pass
};

// Segments of a segmented sort: segment s holds len[s] elements starting at
// start[s] (a multiple of kSegAlign); start[count] is the padded end.
struct SegTable {
  uint32_t count;
  uint32_t overflow;  // the tile entries did not fit the capacity: all segments empty
  uint32_t start[kMaxViews + 1];
  uint32_t len[kMaxViews];
};

// ---- preprocess (per Gaussian and render)
// Render v = blockIdx.y.  Per render: recs/rects/tiles_touched at [v][n],
// depth_keys at [v * n_pad + i] (0xffffffff for a Gaussian that is not
// visible); totals[2v] = visible Gaussians, totals[2v+1] = tile entries.  The
// visible Gaussians' depth keys and indices are also written compacted, in
// index order, to vis_keys / vis_index at [v * n_pad + 0 .. totals[2v]), and
// dseg->len[v] = totals[2v] (the depth sort sorts only them).  flows
// (nullable): [v][n] 2D flow of each visible Gaussian.  temp:
// preprocess_temp_bytes(n, n_views).  zero / zero_bytes (16-byte aligned and
// sized): memory the preprocess clears for the later stages of the run.
size_t preprocess_temp_bytes(uint32_t n, int n_views);
template <typename T>
hipError_t launch_preprocess_fwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, uint32_t n_pad, Rec<T>* recs,
                                 Vec2<T>* flows, Rect16* rects, uint32_t* tiles_touched,
                                 uint32_t* depth_keys, unsigned long long* totals,
                                 uint32_t* vis_keys, uint32_t* vis_index, SegTable* dseg,
                                 void* temp, void* zero, size_t zero_bytes, bool static3d,
                                 hipStream_t stream);

// grad2d: [V][n][C] double (Gaussian-major), C = 9 (mean2 x, y, Sigma_2D (0,0),
// (0,1), (1,1), opacity_t, r, g, b) or, with flow, 11 (then flow x, y).  Writes the parameter
// gradients summed over the renders.
template <typename T>
hipError_t launch_preprocess_bwd(const GaussPtrs<T>& g, const ViewSlot* slots, int n_views,
                                 const SettingsDev& st, const double* grad2d, bool flow,
                                 bool static3d, const GradPtrs<T>& out, hipStream_t stream);

// ---- binning and sorting
// Zeroes `bytes` (a multiple of 16) at p (16-byte aligned) with a kernel, so
// that it may be captured in a graph.
hipError_t fill_zero(void* p, size_t bytes, hipStream_t stream);

// Status words one onesweep pass needs for `capacity` elements at `items` keys
// per lane (4 or 16).
uint32_t sort_status_words(uint64_t capacity_elems, int items);

// hist[p][s][256] += digit-p counts (bits 8p..8p+7) of the keys of each segment.
hipError_t radix_histogram(const uint32_t* keys, const SegTable* seg, int n_segments,
                           uint32_t max_len, int passes, uint32_t* hist, hipStream_t stream);

// Stable segmented LSD radix sort, `passes` 8-bit digits.  Pass 0 reads
// keys_in / vals_in (vals_in null: the value is the element's index within its
// segment); pass p writes bufs[p & 1] and pass p > 0 reads bufs[(p - 1) & 1].
// bufs[1] may alias the inputs.  The sorted data end in bufs[(passes - 1) & 1]
// (*result_index).  hist: [passes][kMaxViews][256]; status: passes x
// sort_status_words, zeroed; tickets: `passes` words, zeroed.  keys_needed =
// false skips writing the keys in the last pass.
hipError_t onesweep_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* key_bufs[2],
                         uint32_t* val_bufs[2], const SegTable* seg, uint64_t capacity_elems,
                         int passes, int items, const uint32_t* hist, uint32_t* status,
                         uint32_t* tickets, uint32_t* error, bool keys_needed, int* result_index,
                         hipStream_t stream);

// Segment table of the emitted list from the per-render entry counts
// (totals[2v + 1]): render v starts at the sum of the earlier renders'
// segment extents (seg_extent: the count, with a depth cut plus room for the
// rest ranges, rounded up to kSegAlign); all segments empty and `overflow`
// set when they exceed `capacity` (also written to *overflow_out when not
// null).
hipError_t seg_table(const unsigned long long* totals, const ViewSlot* slots, int n_views,
                     unsigned long long capacity, SegTable* seg, uint32_t* overflow_out,
                     hipStream_t stream);

size_t count_scan_seg_temp_bytes(uint32_t n_pad, int n_views);
// Bytes of the scan's tile sums when front_counts adds them up itself (they
// must be zero before front_counts runs).
size_t count_tile_sums_bytes(uint32_t n_pad, int n_views);
// offsets[v * n_pad + k] = sum over renders u < v of all their entries plus the
// entries of render v's Gaussians order[v][0..k-1]; offsets[V * n_pad] = total.
// order[v] holds render v's totals[2v] visible Gaussians (the rest is unset).
// Also writes the segment table of the emitted list (as seg_table, for
// `capacity`) and first[b], the depth position of the Gaussian whose entries
// hold the first entry of emission block b (emit_blocks' temp).  The counts
// are counts[v][order[v][k]] (whole lists) or, when front_counts is not null,
// front_counts[v * n_pad + k] (front lists, front_counts below); then the
// segment lengths become the renders' front entry counts and `front` gets
// their rest areas; front_counts has then also written the segment table and
// the scan's tile sums (tile_sums), so the scan starts from those.
hipError_t count_scan_seg(const uint32_t* order, const uint32_t* counts,
                          const uint32_t* front_counts, const unsigned long long* totals,
                          const ViewSlot* slots, uint32_t n, uint32_t n_pad, int n_views,
                          uint64_t* offsets, void* temp, unsigned long long capacity,
                          SegTable* seg, FrontTable* front, uint32_t* overflow_out,
                          uint32_t* first, uint64_t* tile_sums, hipStream_t stream);

// ---- front lists (front.hpp)
// Keep bitmaps (rows of keep_words(tiles_x) words at each render's keep_base)
// of the renders with front16 != 0: a tile is kept when at most `keep` tile
// boxes of the render's front Gaussians (depth order order[v * n_pad + k],
// k below the cut of totals[2 v] visible Gaussians) cover it.  cover: the
// renders' cover grids (at cover_base), zeroed beforehand.  front_grid_ok:
// the render's tile grid fits the kernels (otherwise the host gives it no
// cut).
bool front_grid_ok(int tiles_x, int tiles_y);
hipError_t front_keep(const ViewSlot* slots, int n_views, const Rect16* rects,
                      const uint32_t* order, const unsigned long long* totals, uint32_t n,
                      uint32_t n_pad, int32_t keep, int32_t* cover, uint64_t* bits,
                      hipStream_t stream);
// counts[v * n_pad + k]: entries of the front lists from render v's Gaussian at
// depth position k (order[v][k]); whole: per-Gaussian counts of the whole
// lists ([v][n]); srect[v * n_pad + k] = its tile box for k from the render's
// depth cut to its visible count.  Also adds the counts up per tile of the
// count scan into tile_sums (count_tile_sums_bytes, zeroed beforehand) and
// writes the segment table of the emitted list for `capacity` (as seg_table),
// the count scan's first step.
template <typename T>
hipError_t front_counts(const uint32_t* order, const uint32_t* whole, const Rect16* rects,
                        const Rec<T>* recs, const ViewSlot* slots,
                        const unsigned long long* totals, const uint64_t* bits, uint32_t n,
                        uint32_t n_pad, int n_views, uint32_t* counts, Rect16* srect,
                        uint64_t* tile_sums, unsigned long long capacity, SegTable* seg,
                        uint32_t* overflow_out, hipStream_t stream);

// Emission of every render's tile entries in depth order (each Gaussian's
// tiles row by row, its row runs from tileset.hpp) into its segment, one
// 4096-entry block per workgroup.  packed: out_a[e] = Gaussian index |
// (tile >> 8) << 24 and out_b[e] = tile & 255 (bytes), the packed sort's
// input; otherwise out_a[e] = tile id, out_b[e] = Gaussian index (words).
// temp: emit_temp_bytes(capacity), holding the first-Gaussian map of the count
// scan.  packed: sort_temp is packed_tile_sort's temp, where the emission
// writes the low-byte digit counts of its blocks (the sort's first histogram).
// keep (nullable): the keep bitmaps; the Gaussians from a render's depth cut
// on (totals[2v] visible) list only their kept tiles, counts[v * n_pad + k]
// of them (front_counts).
size_t emit_temp_bytes(uint64_t capacity);
template <typename T>
hipError_t emit_blocks(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                       const Rec<T>* recs, const ViewSlot* slots, const SegTable* seg,
                       const unsigned long long* totals, const uint64_t* keep,
                       const uint32_t* counts, uint32_t n,
                       uint32_t n_pad, int n_views, uint64_t capacity, bool packed, void* temp,
                       uint32_t* out_a, void* out_b, void* sort_temp, hipStream_t stream);

// Tile ranges (ranges[tile_base + t] = [start, end) in the emitted list, [0, 0)
// for a tile without entries) from every segment's sorted tile ids (16 or 32
// bits).  ranges must be zero on entry (only the tiles with entries are
// written).
hipError_t tile_ranges(const void* sorted_tiles, bool tiles16, const SegTable* seg,
                       const ViewSlot* slots, uint32_t total_tiles, uint64_t capacity,
                       uint2* ranges, hipStream_t stream);

// hist[p][s][256] = digit-p counts of the emitted tile ids of segment s
// (zeroes hist first), for the onesweep tile sort.
hipError_t tile_key_histogram(const uint32_t* keys, const SegTable* seg, uint64_t capacity,
                              int passes, uint32_t* hist, hipStream_t stream);

// Tile sort on packed 32-bit entries (see binning.hip), usable when
// packed_tile_sort_ok: a low-digit pass on (packed, digits) into (mid,
// mid_hi), then a high-digit pass into values (the sorted Gaussian indices)
// and tiles (their 16-bit tile ids).  seg: the tile segment table; max_tiles:
// the largest tile count of the renders; temp: packed_sort_temp_bytes(capacity)
// bytes; every other array holds capacity elements.
bool packed_tile_sort_ok(uint32_t n, uint32_t max_tiles_per_view);
size_t packed_sort_temp_bytes(uint64_t capacity);
hipError_t packed_tile_sort(const uint32_t* packed, const uint8_t* digits, const SegTable* seg,
                            uint32_t max_tiles, uint64_t capacity, void* temp, uint32_t* mid,
                            uint8_t* mid_hi, uint32_t* values, uint16_t* tiles,
                            hipStream_t stream);

// Exclusive scan of a[0..n) into out[0..n] (out[n] = total); temp holds
// scan_u32_temp_bytes(n).
size_t scan_u32_temp_bytes(uint32_t n);
hipError_t scan_u32(const uint32_t* a, uint32_t n, uint32_t* out, void* temp, hipStream_t stream);

// ---- rasterisation
// The backward walks each tile's list in independent segments of kSegment
// entries.  The forward saves, at every segment boundary inside a tile's
// list, each pixel's transmittance and accumulated colour (Ck) in slot
// ck_slot(list start, global tile, boundary index) of TS*TS pixels, the final
// colour of every pixel, and each tile's walk length (its furthest last
// contributor).  Slots stay below capacity / kSegment + tiles + 1.  With
// front lists a tile's list is its front range followed by its rest range
// (front.hpp: list_pos, boundary_slot).
constexpr uint32_t kSegment = 256;

template <typename T>
struct Ck {
  T t, r, g, b;
};

__host__ __device__ __forceinline__ uint32_t ck_slot(uint32_t list_start, uint32_t gtile,
                                                     uint32_t m) {
  return list_start / kSegment + gtile + m;
}

template <typename T>
struct RasterSaved {
  Ck<T>* ck;       // boundary states
  T* img;          // final colour per pixel, laid out like the images
  uint32_t* walk;  // per global tile
  // flow renders: boundary flow sums (slots like ck) and the final flow per
  // pixel, laid out like the flow images; null otherwise
  Vec2<T>* ckf;
  T* flow;
  // per global tile, [start, end) of its rest range ([0, 0): none), zeroed
  // before the forward
  uint2* rest;
};

// What the forward needs to collect a front list's rest (front.hpp); keep
// null: whole lists.  order and srect: [V][n_pad], the depth order and the
// tile boxes in depth order from each render's cut on; totals[2v]: visible
// Gaussians; table: the rest areas (cursors and tile counts advanced) and the
// count of queue, the tiles left to the rest pass (room for every tile);
// overflow: set if a rest area were too small (its size rules that out).
struct FrontCollect {
  const uint64_t* keep;
  const uint32_t* order;
  const Rect16* srect;
  const unsigned long long* totals;
  FrontTable* table;
  uint32_t* queue;
  uint32_t* overflow;
  uint32_t n_pad;
};

// (tile size, pixels per lane) pairs the rasteriser is compiled for.
bool raster_config_supported(int tile_size, int ppt);
int raster_default_ppt(int tile_size, bool backward);

// Persistent launch over all tiles of all renders; tickets: 1 word, zeroed.
// recs: [V][n]; image: [3][pixels of render v] at 3 * pix_base; T_final,
// n_contrib per pixel at pix_base, n_eval (nullable) per pixel the pair
// (entries evaluated, entries blended) at 2 * pix_base; sv: what the backward's
// segment walks need (see kSegment).  A flow render (flows: [V][n] per-Gaussian
// 2D flow, not null) also composites the flow into flow_image ([2][pixels] at
// 2 * pix_base, background 0) and fills sv.ckf and sv.flow; it counts no
// evaluations (n_eval must be null).  Front lists (fc.keep not null): a tile
// whose front list runs out before its pixels stop collects its rest entries
// into `values` and records them in sv.rest.
template <typename T>
hipError_t launch_raster_fwd(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                             uint32_t* values, const uint2* ranges, const FrontCollect& fc,
                             const ViewSlot* slots,
                             int n_views, uint32_t total_tiles, int tile_size,
                             const SettingsDev& st, int ppt, T* image, T* flow_image, T* T_final,
                             uint32_t* n_contrib, uint32_t* n_eval, const RasterSaved<T>& sv,
                             uint32_t* tickets, hipStream_t stream);

// Persistent launch over the (tile, segment) walks.  grad2d: [V][n][C] double
// accumulators, added to, C = 9, or 11 when dL_dflow is given (a flow render's
// saved state with the flow images' gradient, laid out like them).  max_items:
// bound on the number of walks (capacity / kSegment + tiles + 1); work:
// raster_bwd_work_bytes, its first 256 bytes zeroed.
size_t raster_bwd_work_bytes(uint32_t total_tiles, uint64_t max_items);
template <typename T>
hipError_t launch_raster_bwd(const Rec<T>* recs, const Vec2<T>* flows, uint32_t n,
                             const uint32_t* values, const uint2* ranges, const ViewSlot* slots,
                             int n_views, uint32_t total_tiles, uint64_t max_items,
                             int tile_size, const SettingsDev& st, int ppt, const T* T_final,
                             const uint32_t* n_contrib, const RasterSaved<T>& sv,
                             const T* dL_dimage, const T* dL_dflow, double* grad2d,
                             uint32_t* work, hipStream_t stream);

// L1 loss (mean absolute difference) and its gradient.  The loss (when `loss`
// is not null) is summed through per-workgroup partial sums in `partials`
// (device memory of l1_partials_floats() floats), not through atomics on one
// address.
size_t l1_partials_floats();
hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, float* grad,
                          float* loss, float* partials, hipStream_t stream);

// Per-view L1: view v covers elements [base[v], base[v + 1]) and is normalised
// by its own count; the loss sums the views' means.
struct L1Views {
  int n_views;
  int64_t base[kMaxViews + 1];
  int64_t count[kMaxViews];
};
hipError_t launch_l1_grad_views(const float* images, const float* targets, const L1Views& lv,
                                float* grad, float* loss, float* partials, hipStream_t stream);

// ---- 4D nearest neighbours and the 4D consistency loss
// out: [n][k] int32, the k nearest other points of each point (nearest first,
// ties by index) in the scaled coordinates u = x * inv (inv_spatial for x, y,
// z; inv_temporal for t) of means ([4][n] float32).  1 <= k <= 32, k < n.
// temp: knn4d_temp_bytes(n).
size_t knn4d_temp_bytes(uint32_t n);
hipError_t launch_knn4d(const float* means, uint32_t n, int k, float inv_spatial,
                        float inv_temporal, int32_t* out, void* temp, hipStream_t stream);

// L = (1/n) sum_i |s_i - mean_{j in nb[i]} s_j|_1, s = V / W; *loss = L (when
// not null); grad_rotors / grad_log_scales (when both are given) += weight *
// dL/d(raw rotor, log-scales).  nb: [n][k]; entries outside [0, n) are
// skipped.  temp: consistency_temp_bytes<T>(n).
template <typename T>
size_t consistency_temp_bytes(uint32_t n);
template <typename T>
hipError_t launch_consistency(const GaussPtrs<T>& g, const int32_t* nb, int k, T weight, T* loss,
                              T* grad_rotors, T* grad_log_scales, void* temp,
                              hipStream_t stream);

// ---- optimisation step
// The five parameter groups (means, log_scales, rotors, opacity, sh) of n
// Gaussians: p[k] the render's arrays, g[k] their gradients (the opacity one
// w.r.t. the activated opacity), off[k] the group's first element in the
// concatenated moment arrays (off[5] = total).
struct AdamGroups {
  float* p[5];
  const float* g[5];
  uint64_t off[6];
  uint32_t n;
};
struct AdamConfig {
  float lr_means_init, lr_means_final;
  int32_t lr_means_steps;
  float lr_log_scales, lr_rotors, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
};
// One Adam step of every group at step count *step (steps already taken),
// then *step += 1.  The opacity group updates `logit` and writes the activated
// opacity back into p[3].
hipError_t launch_adam(const AdamGroups& groups, float* logit, float* m, float* v, int32_t* step,
                       const AdamConfig& cfg, hipStream_t stream);
hipError_t launch_state_init(uint32_t n, uint64_t total, const float* opacity, float* logit,
                             float* m, float* v, int32_t* step, hipStream_t stream);
hipError_t launch_opacity_reset(uint32_t n, float cap, float* logit, float* opacity, float* m_op,
                                float* v_op, hipStream_t stream);
// Entropy (1/n) sum -o ln o into *loss (nullable); grad (nullable) += weight *
// its gradient.  temp: entropy_temp_bytes(n).
size_t entropy_temp_bytes(uint32_t n);
hipError_t launch_entropy(const float* opacity, uint32_t n, float weight, float* loss, float* grad,
                          void* temp, hipStream_t stream);

// ---- density control
// accum[i] += sum over the renders where Gaussian i is listed (dkeys not
// 0xffffffff) of the NDC norm of its projected-mean gradient (grad2d
// components 0, 1 of the nc per Gaussian and render); count[i] += those renders.
hipError_t launch_densify_stats(const double* grad2d, int nc, const uint32_t* dkeys,
                                uint32_t n_pad, const ViewSlot* slots, int n_views, uint32_t n,
                                float* accum, int32_t* count, hipStream_t stream);

// Clone / split / prune (see r4d_densify).  densify_count classifies and scans
// and copies the three totals (kept, clones, children) to pinned host memory;
// after they have arrived, densify_scatter writes the new set.
struct DensifyArgs {
  uint32_t n_in;
  const float* log_scales;
  const float* opacity;
  const float* accum;
  const int32_t* count;
  const float* normals;
  float grad_threshold, size_log, min_opacity, big_log, shrink;
  int has_big;
  const float* pin[5];
  float* pout[5];
  uint32_t rows[5];
  const float* logit_in;
  float* logit_out;
  const float* m_in;
  const float* v_in;
  float* m_out;
  float* v_out;
};
size_t densify_temp_bytes(uint32_t n);
hipError_t densify_count(const DensifyArgs& d, void* temp, uint32_t* totals_host,
                         hipStream_t stream);
hipError_t densify_scatter(const DensifyArgs& d, const void* temp, uint32_t total_keep,
                           uint32_t total_clone, uint32_t n_out, hipStream_t stream);

// ---- small helpers
// p[0..count) = value (float or double elements).
hipError_t fill_const(void* p, size_t count, double value, bool f64, hipStream_t stream);
// out += tmp, tmp holding the five gradient arrays back to back
// (means 4n, log_scales 4n, rotors 8n, opacity n, sh k3 n; for static 3D
// Gaussians 3n, 3n, 4n, n, k3 n).
template <typename T>
hipError_t add_grads(const GradPtrs<T>& out, const T* tmp, size_t n, size_t k3, bool static3d,
                     hipStream_t stream);
// dst[t] = src[t] - (base, base); empty ranges stay [0, 0).
hipError_t copy_ranges_rebased(const uint2* src, uint32_t count, uint32_t base, uint2* dst,
                               hipStream_t stream);

}  // namespace r4d
