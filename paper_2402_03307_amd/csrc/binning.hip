// Tile binning: per-tile entry counts, tile ranges, tile-key emission and a
// segmented onesweep radix sort (one kernel per 8-bit digit).
//
// The (tile, depth) order the rasteriser needs is produced in two stable
// stages.  The Gaussians of every render are sorted by the float32 bit pattern
// of their depth (positive floats order like their bit patterns; culled
// Gaussians carry 0xffffffff and sort last); each Gaussian's tiles are then
// emitted in that depth order and the emitted list is stably sorted by tile id.
// The result is ordered by (tile, depth, Gaussian index): a radix sort of that
// composite key whose depth part is sorted once per Gaussian instead of once
// per tile entry.
//
// Several renders are processed at once as segments of one array: segment s
// starts at a multiple of 4096 elements and every sort pass works within
// segments only.  Per-tile entry counts do not need the emitted keys: every
// row run of every Gaussian (tileset.hpp) adds +1 at its first tile and -1
// after its last into a difference grid, and the grid's prefix sum along rows
// is the count of every tile.  Their exclusive scan is the tile ranges, and
// their digit sums are the digit histograms of the tile sort.
//
// Onesweep pass: every workgroup takes a ticket (its position in the sort
// order, in launch order, so that every lower ticket belongs to a workgroup
// that is already running), ranks its 4096 keys stably in LDS, publishes its
// per-digit counts, and adds up the counts of the workgroups before it in the
// same segment (decoupled look-back), stopping at the first one that has
// published its inclusive prefix.  The spin on a predecessor is bounded: past
// the bound the pass raises an error flag and finishes with in-bounds (but
// wrong) positions instead of hanging.
#include <hip/hip_runtime.h>

#include "r4d_internal.hpp"
#include "tileset.hpp"

namespace r4d {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kStatAgg = 1u << 30;   // published: this workgroup's count only
constexpr uint32_t kStatPre = 2u << 30;   // published: inclusive prefix within the segment
constexpr uint32_t kStatMask = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a workgroup of NT threads;
// *total receives the sum.  s_w must hold NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* s_w, T* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T inc = wave_incl_scan(x, lane);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const T s = s_w[w];
    off += w < wave ? s : T(0);
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - x;
}

// ---- device-wide exclusive scan (multi-level: tile sums are scanned recursively)
constexpr int kScanItems = 4;
constexpr int kScanTile = kThreads * kScanItems;

// Row-run constants of a Gaussian from its record and the bounding box of its
// runs.
template <typename T>
__device__ __forceinline__ SpanGeom geom_of(const Rec<T>& r, const Rect16& box, const ViewDev& v) {
  return span_geom(double(r.mx), double(r.my), double(r.ca), double(r.cb), double(r.cc),
                   double(r.qmax), v.W, v.H, __builtin_ctz(unsigned(v.tile_size)), box.x0,
                   box.x1);
}

// Entries [q0, q1) of one Gaussian (indices local to the Gaussian, in the
// order of its tile list: rows top to bottom, columns left to right), the
// whole wavefront cooperating: lane l takes tile row y0 + l (then + 64, ...),
// a wave scan of the run lengths places every row, and each lane calls
// put(j, tile) for the entries j of its row in [q0, q1).  Every lane must call
// it with the same arguments.
template <typename Put>
__device__ __forceinline__ void wave_runs(const SpanGeom& sg, int y0, int y1, uint32_t tiles_x,
                                          uint32_t q0, uint32_t q1, int lane, Put put) {
  uint32_t carry = 0;
  for (int yb = y0; yb < y1 && carry < q1; yb += 64) {
    const int y = yb + lane;
    int a = 0, b = 0;
    if (y < y1) row_span(sg, y, a, b);
    const uint32_t len = uint32_t(b - a);
    const uint32_t incl = wave_incl_scan(len, lane);
    const uint32_t start = carry + incl - len;
    const uint32_t j0 = start > q0 ? start : q0;
    const uint32_t j1 = start + len < q1 ? start + len : q1;
    const uint32_t t0 = uint32_t(y) * tiles_x + uint32_t(a) - start;  // tile of entry j: t0 + j
    for (uint32_t j = j0; j < j1; ++j) put(j, t0 + j);
    carry += __shfl(incl, 63, 64);
  }
}

template <typename T>
struct LoadT {
  const T* p;
  uint64_t n;
  __device__ T operator()(uint64_t i) const { return i < n ? p[i] : T(0); }
};

template <typename T, typename Loader>
__global__ __launch_bounds__(kThreads) void scan_tiles_kernel(Loader ld, T* out, T* tile_sums,
                                                              uint64_t n) {
  __shared__ T s_w[kThreads / 64];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = ld(base + j);
    sum += v[j];
  }
  T total;
  T run = block_excl_scan<kThreads>(sum, s_w, &total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scan_add_kernel(T* out, const T* tile_offsets,
                                                            uint64_t n) {
  const T add = tile_offsets[blockIdx.x];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint64_t i = base + uint64_t(j) * kThreads + threadIdx.x;
    if (i < n) out[i] += add;
  }
}

uint64_t scan_temp_elems(uint64_t n) {
  uint64_t total = 0, m = n;
  while (m > uint64_t(kScanTile)) {
    m = (m + kScanTile - 1) / kScanTile;
    total += m;
  }
  return total;
}

// Exclusive scan of ld(0..n-1) into out[0..n-1]; temp holds scan_temp_elems(n) T's.
template <typename T, typename Loader>
hipError_t device_exclusive_scan(Loader ld, T* out, uint64_t n, T* temp, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    hipLaunchKernelGGL((scan_tiles_kernel<T, Loader>), dim3(1), dim3(kThreads), 0, stream, ld,
                       out, (T*)nullptr, n);
    return hipGetLastError();
  }
  T* sums = temp;
  hipLaunchKernelGGL((scan_tiles_kernel<T, Loader>), dim3(uint32_t(tiles)), dim3(kThreads), 0,
                     stream, ld, out, sums, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_exclusive_scan<T, LoadT<T>>(LoadT<T>{sums, tiles}, sums, tiles, temp + tiles, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_add_kernel<T>, dim3(uint32_t(tiles)), dim3(kThreads), 0, stream, out,
                     (const T*)sums, n);
  return hipGetLastError();
}

// Largest segment whose start is <= e (empty segments share their start with
// the next one, so the non-empty segment holding e is found).
__device__ __forceinline__ uint32_t segment_of(const SegTable* t, uint32_t e) {
  uint32_t lo = 0, hi = t->count - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (t->start[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kThreads) void fill_zero_kernel(uint4* __restrict__ p, uint64_t n16) {
  const uint64_t stride = uint64_t(gridDim.x) * kThreads;
  for (uint64_t i = uint64_t(blockIdx.x) * kThreads + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Digit histograms of keys, PASSES digits of 8 bits, per segment (blockIdx.y).
template <int PASSES>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              const SegTable* __restrict__ seg,
                                                              uint32_t chunk,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[PASSES][256];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) h[p][threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t s = blockIdx.y;
  if (s < seg->count) {
    const uint32_t s0 = seg->start[s];
    const uint32_t begin = s0 + blockIdx.x * chunk;
    const uint32_t send = s0 + seg->len[s];
    const uint32_t end = send < begin + chunk ? send : begin + chunk;
    for (uint32_t i = begin + threadIdx.x; i < end; i += kThreads) {
      const uint32_t key = keys[i];
#pragma unroll
      for (int p = 0; p < PASSES; ++p) atomicAdd(&h[p][(key >> (8 * p)) & 255u], 1u);
    }
  }
  __syncthreads();
  if (s < seg->count) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const uint32_t c = h[p][threadIdx.x];
      if (c) atomicAdd(&hist[(size_t(p) * kMaxViews + s) * 256 + threadIdx.x], c);
    }
  }
}

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void onesweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const SegTable* __restrict__ seg, const uint32_t* __restrict__ hist,
    uint32_t* __restrict__ status, uint32_t* __restrict__ ticket, uint32_t* __restrict__ error,
    int shift) {
  constexpr uint32_t TILE = kThreads * ITEMS;
  __shared__ uint32_t s_keys[TILE];
  __shared__ uint32_t s_vals[TILE];
  __shared__ uint32_t s_wh[kThreads / 64][256];  // per-wave digit counts, then wave prefixes
  __shared__ uint32_t s_start[256];              // workgroup-local start of each digit
  __shared__ uint32_t s_gofs[256];               // output position minus local position
  __shared__ uint32_t s_w[kThreads / 64];
  __shared__ uint32_t s_bid;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_bid = atomicAdd(ticket, 1u);
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s_wh[w][tid] = 0u;
  __syncthreads();
  const uint32_t b = s_bid;
  const uint32_t e0 = b * TILE;
  if (seg->count == 0u || e0 >= seg->start[seg->count]) return;
  const uint32_t s = segment_of(seg, e0);
  const uint32_t sstart = seg->start[s];
  const uint32_t send = sstart + seg->len[s];
  const uint32_t first_b = sstart / TILE;
  const uint32_t nvalid = send > e0 ? (send - e0 < TILE ? send - e0 : TILE) : 0u;

  // load: wave w holds elements [w * 64 * ITEMS, (w + 1) * 64 * ITEMS) of the tile
  uint32_t k[ITEMS], v[ITEMS], r[ITEMS];
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t loc = wbase + uint32_t(i) * 64u + uint32_t(lane);
    const bool ok = loc < nvalid;
    k[i] = ok ? keys_in[e0 + loc] : 0u;
    v[i] = !ok ? 0u : vals_in ? vals_in[e0 + loc] : e0 + loc - sstart;
  }
  // stable rank within the wave: lanes with equal digits found with 8 ballots;
  // the wave's running digit counts live in its own LDS row, so no atomics and
  // no barriers are needed (a wave's LDS accesses complete in program order)
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool ok = wbase + uint32_t(i) * 64u + uint32_t(lane) < nvalid;
    const uint32_t d = (k[i] >> shift) & 255u;
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool x = (d >> bit) & 1u;
      const unsigned long long m = __ballot(x);
      peers &= x ? m : ~m;
    }
    const uint32_t base = s_wh[wave][d];
    const unsigned long long before = peers & lt;
    r[i] = base + uint32_t(__popcll(before));
    if (ok && before == 0ull) s_wh[wave][d] = base + uint32_t(__popcll(peers));
  }
  __syncthreads();
  // thread tid = digit: wave prefixes and the workgroup count of the digit
  uint32_t cnt = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t t = s_wh[w][tid];
    s_wh[w][tid] = cnt;
    cnt += t;
  }
  uint32_t* my = status + size_t(b) * 256u + uint32_t(tid);
  store_relaxed(my, (b == first_b ? kStatPre : kStatAgg) | cnt);
  uint32_t tot;
  s_start[tid] = block_excl_scan<kThreads>(cnt, s_w, &tot);
  const uint32_t hb = block_excl_scan<kThreads>(hist[size_t(s) * 256u + uint32_t(tid)], s_w, &tot);
  uint32_t prev = 0;
  if (b != first_b) {
    uint32_t j = b - 1u, spins = 0;
    for (;;) {
      const uint32_t val = load_relaxed(status + size_t(j) * 256u + uint32_t(tid));
      const uint32_t fl = val & ~kStatMask;
      if (fl == 0u) {
        if (++spins > kSpinLimit) {
          atomicOr(error, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        continue;
      }
      prev += val & kStatMask;
      if (fl == kStatPre || j == first_b) break;
      --j;
    }
    store_relaxed(my, kStatPre | (prev + cnt));
  }
  s_gofs[tid] = sstart + hb + prev - s_start[tid];
  __syncthreads();
  // local scatter into digit order, then runs of equal digits to consecutive addresses
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (wbase + uint32_t(i) * 64u + uint32_t(lane) < nvalid) {
      const uint32_t d = (k[i] >> shift) & 255u;
      const uint32_t p = s_start[d] + s_wh[wave][d] + r[i];
      s_keys[p] = k[i];
      s_vals[p] = v[i];
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < nvalid; p += kThreads) {
    const uint32_t key = s_keys[p];
    const uint32_t g = s_gofs[(key >> shift) & 255u] + p;
    if (keys_out) keys_out[g] = key;
    vals_out[g] = s_vals[p];
  }
}

// Difference grids: every row run [x0, x1) of row y adds +1 at (y, x0) and -1
// at (y, x1) (skipped when x1 is past the last column), so the prefix sum of a
// grid row is the entry count of each of its tiles.
//
// tile_grid_kernel (blockIdx.y = render): with LDS_GRID every workgroup adds
// the runs of its share of the Gaussians into a private grid in LDS and
// writes that grid out as one partial; otherwise (grids too large for LDS) it
// adds them into one global grid with atomics.
template <typename T, bool LDS_GRID>
__global__ __launch_bounds__(kThreads) void tile_grid_kernel(const Rect16* __restrict__ rects,
                                                             const Rec<T>* __restrict__ recs,
                                                             const ViewSlot* __restrict__ slots,
                                                             uint32_t n, int* __restrict__ partials,
                                                             int* __restrict__ grid) {
  extern __shared__ int s_grid[];
  const int v = blockIdx.y;
  const ViewSlot& sl = slots[v];
  const ViewDev vd = sl.v;
  const int tx = vd.tiles_x, ty = vd.tiles_y;
  const int W1 = tx + 1;
  const int cells = W1 * (ty + 1);
  if (LDS_GRID) {
    for (int i = threadIdx.x; i < cells; i += kThreads) s_grid[i] = 0;
    __syncthreads();
  }
  int* gd = LDS_GRID ? s_grid : grid + sl.grid_base;
  const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t begin = blockIdx.x * per;
  const uint32_t end = begin + per < n ? begin + per : n;
  const Rect16* rv = rects + size_t(v) * n;
  const Rec<T>* cv = recs + size_t(v) * n;
  for (uint32_t i = begin + threadIdx.x; i < end; i += kThreads) {
    const Rect16 r = rv[i];
    if (r.x1 == r.x0) continue;  // culled: empty box
    const SpanGeom sg = geom_of(cv[i], r, vd);
    for (int y = r.y0; y < r.y1; ++y) {
      int x0, x1;
      row_span(sg, y, x0, x1);
      atomicAdd(&gd[y * W1 + x0], 1);
      if (x1 < tx) atomicAdd(&gd[y * W1 + x1], -1);
    }
  }
  if (LDS_GRID) {
    __syncthreads();
    int* out = partials + size_t(sl.grid_base) * gridDim.x + size_t(blockIdx.x) * cells;
    for (int i = threadIdx.x; i < cells; i += kThreads) out[i] = s_grid[i];
  }
}

// grid[c] = sum of the partial grids at cell c (cells of all renders).
__global__ __launch_bounds__(kThreads) void grid_sum_kernel(const ViewSlot* __restrict__ slots,
                                                            int n_views, const int* __restrict__ partials,
                                                            int n_partials, uint32_t total_cells,
                                                            int* __restrict__ grid) {
  const uint32_t c = blockIdx.x * kThreads + threadIdx.x;
  if (c >= total_cells) return;
  int v = 0;
  while (v + 1 < n_views && slots[v + 1].grid_base <= c) ++v;
  const uint32_t gb = slots[v].grid_base;
  const uint32_t cells = uint32_t(slots[v].v.tiles_x + 1) * uint32_t(slots[v].v.tiles_y + 1);
  const int* pv = partials + size_t(gb) * n_partials + (c - gb);
  int acc = 0;
#pragma unroll 8
  for (int b = 0; b < n_partials; ++b) acc += pv[size_t(b) * cells];
  grid[c] = acc;
}

// One workgroup per render: takes the prefix sum of every grid row (in LDS when
// the grid fits) to get every tile's entry count,
// and scans the counts in tile order into the tile ranges inside the render's
// segment of the emitted list; their digit sums give the tile sort's
// histograms.  Also lays out the segments (render v starts at the sum of the
// earlier renders' counts, each rounded up to 4096) and reports overflow of the
// entry capacity, in which case every segment is empty and every range is
// [0, 0).
constexpr int kTcThreads = 1024;

template <bool LDS_GRID>
__global__ __launch_bounds__(kTcThreads) void tile_count_kernel(
    const ViewSlot* __restrict__ slots, int n_views, int* __restrict__ grid,
    const unsigned long long* __restrict__ totals,
    unsigned long long capacity, uint2* __restrict__ ranges, uint32_t* __restrict__ hist,
    SegTable* __restrict__ seg) {
  extern __shared__ int s_grid[];
  __shared__ uint32_t s_h[3][256];
  __shared__ uint32_t s_w[kTcThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int v = blockIdx.x;
  for (int i = tid; i < 3 * 256; i += kTcThreads) (&s_h[0][0])[i] = 0u;
  unsigned long long base = 0, total = 0;
  bool too_long = false;
  for (int u = 0; u < n_views; ++u) {
    const unsigned long long d = totals[2 * u + 1];
    const unsigned long long pd = (d + kSegAlign - 1) / kSegAlign * kSegAlign;
    if (u < v) base += pd;
    total += pd;
    too_long |= d > kStatMask;
  }
  const bool overflow = too_long || total > capacity;
  const unsigned long long Dv = totals[2 * v + 1];
  if (tid == 0) {
    seg->start[v] = overflow ? 0u : uint32_t(base);
    seg->len[v] = overflow ? 0u : uint32_t(Dv);
    if (v == n_views - 1) seg->start[n_views] = overflow ? 0u : uint32_t(total);
    if (v == 0) {
      seg->count = uint32_t(n_views);
      seg->overflow = overflow ? 1u : 0u;
    }
  }
  const ViewSlot& sl = slots[v];
  const int tx = sl.v.tiles_x, ty = sl.v.tiles_y;
  const uint32_t ntiles = uint32_t(tx) * uint32_t(ty);
  if (overflow) {
    for (uint32_t t = tid; t < ntiles; t += kTcThreads) ranges[sl.tile_base + t] = make_uint2(0u, 0u);
  } else {
    const int W1 = tx + 1, H1 = ty + 1, cells = W1 * H1;
    int* gd = grid + sl.grid_base;
    if (LDS_GRID) {
      for (int i = tid; i < cells; i += kTcThreads) s_grid[i] = gd[i];
      gd = s_grid;
    }
    __syncthreads();
    for (int row = wave; row < ty; row += kTcThreads / 64) {
      int carry = 0;
      for (int c0 = 0; c0 < tx; c0 += 64) {
        const int x = c0 + lane;
        const int val = x < tx ? gd[row * W1 + x] : 0;
        const int inc = wave_incl_scan(val, lane) + carry;
        if (x < tx) gd[row * W1 + x] = inc;
        carry = __shfl(inc, 63, 64);
      }
    }
    __syncthreads();
    uint32_t run = uint32_t(base);
    const uint32_t seg_end = uint32_t(base + Dv);
    for (uint32_t t0 = 0; t0 < ntiles; t0 += kTcThreads) {
      const uint32_t t = t0 + tid;
      const uint32_t c = t < ntiles ? uint32_t(gd[int(t / tx) * W1 + int(t % tx)]) : 0u;
      uint32_t tot;
      const uint32_t ex = block_excl_scan<kTcThreads>(c, s_w, &tot) + run;
      if (t < ntiles) {
        // (clamped to the segment: the grid and the per-Gaussian counts follow
        // the same runs, so this only guards the reads of the rasteriser)
        const uint32_t e0 = ex < seg_end ? ex : seg_end;
        const uint32_t e1 = ex + c < seg_end ? ex + c : seg_end;
        ranges[sl.tile_base + t] = c ? make_uint2(e0, e1) : make_uint2(0u, 0u);
        if (c) {
          atomicAdd(&s_h[0][t & 255u], c);
          atomicAdd(&s_h[1][(t >> 8) & 255u], c);
          atomicAdd(&s_h[2][(t >> 16) & 255u], c);
        }
      }
      run += tot;
    }
  }
  __syncthreads();
  for (int i = tid; i < 3 * 256; i += kTcThreads)
    hist[(size_t(i >> 8) * kMaxViews + v) * 256 + (i & 255)] = (&s_h[0][0])[i];
}

// Exclusive scan input: tile counts of every render's Gaussians in depth order,
// render-major, each render padded to n_pad entries with zeros.
struct LoadCountGatherSeg {
  const uint32_t* order;  // [V][n_pad] Gaussian index in depth order
  const uint32_t* counts; // [V][n]
  uint32_t n, n_pad;
  uint64_t total;         // V * n_pad
  __device__ uint64_t operator()(uint64_t i) const {
    if (i >= total) return 0;
    const uint32_t v = uint32_t(i / n_pad), k = uint32_t(i % n_pad);
    return k < n ? uint64_t(counts[size_t(v) * n + order[i]]) : uint64_t(0);
  }
};

// Tile-key emission: each wavefront takes 64 consecutive Gaussians of one
// render's depth order and writes their tile entries one Gaussian at a time,
// the lanes on its tile rows (wave_runs).  Keys are render-local tile ids.
template <typename T>
__global__ __launch_bounds__(256) void emit_kernel(const uint32_t* __restrict__ order,
                                                   const uint64_t* __restrict__ offsets,
                                                   const Rect16* __restrict__ rects,
                                                   const Rec<T>* __restrict__ recs,
                                                   const ViewSlot* __restrict__ slots,
                                                   const SegTable* __restrict__ seg, uint32_t n,
                                                   uint32_t n_pad, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  const uint32_t v = blockIdx.y;
  const int lane = threadIdx.x & 63;
  if (seg->overflow) return;
  const uint32_t kk = uint32_t(i);
  uint32_t idx = 0, cnt = 0, off = 0;
  const size_t row = size_t(v) * n_pad;
  if (kk < n) {
    idx = order[row + kk];
    off = seg->start[v] + uint32_t(offsets[row + kk] - offsets[row]);
    cnt = uint32_t(offsets[row + kk + 1] - offsets[row + kk]);
  }
  const ViewDev vd = slots[v].v;
  const uint32_t tiles_x = uint32_t(vd.tiles_x);
  unsigned long long todo = __ballot(cnt > 0);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1ull;
    const uint32_t s_idx = __shfl(idx, src, 64);
    const uint32_t s_cnt = __shfl(cnt, src, 64);
    const uint32_t s_off = __shfl(off, src, 64);
    const Rect16 r = rects[size_t(v) * n + s_idx];
    const SpanGeom sg = geom_of(recs[size_t(v) * n + s_idx], r, vd);
    wave_runs(sg, r.y0, r.y1, tiles_x, 0u, s_cnt, lane, [&](uint32_t j, uint32_t tile) {
      keys[s_off + j] = tile;
      vals[s_off + j] = s_idx;
    });
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_const_kernel(T* __restrict__ p, size_t count,
                                                              T value) {
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < count; i += stride) p[i] = value;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void add_grads_kernel(GradPtrs<T> out,
                                                             const T* __restrict__ tmp, size_t n,
                                                             size_t k3) {
  const size_t total = (17 + k3) * n;
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
    T* dst;
    if (i < 4 * n)
      dst = out.means + i;
    else if (i < 8 * n)
      dst = out.log_scales + (i - 4 * n);
    else if (i < 16 * n)
      dst = out.rotors + (i - 8 * n);
    else if (i < 17 * n)
      dst = out.opacity + (i - 16 * n);
    else
      dst = out.sh + (i - 17 * n);
    *dst += tmp[i];
  }
}

__global__ __launch_bounds__(kThreads) void rebase_ranges_kernel(const uint2* __restrict__ src,
                                                                 uint32_t count, uint32_t base,
                                                                 uint2* __restrict__ dst) {
  const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i < count) {
    const uint2 r = src[i];
    dst[i] = r.y > r.x ? make_uint2(r.x - base, r.y - base) : make_uint2(0u, 0u);
  }
}

uint32_t grid_for(size_t count) {
  const size_t b = (count + kThreads - 1) / kThreads;
  return uint32_t(b < 4096 ? (b ? b : 1) : 4096);
}

// ---- packed tile sort
// For renders with at most 65536 tiles and at most 2^24 Gaussians the tile
// sort runs on one 32-bit word per entry: Gaussian index in bits 0..23, the
// high 8 bits of the tile id in bits 24..31.  The entries of a render are
// numbered in emission order (Gaussians in depth order, each one's tiles
// row-major) and cut into blocks of 4096; block b of the render is also block
// b of its segment of the sorted output.  Both passes are reduce-then-scan:
// per-block digit counts, a column scan of those counts, then a stable
// scatter, so no workgroup waits on another.  The first (low-digit) pass
// generates its block's entries itself from the Gaussians' rectangles, so
// the emitted list is never written.
constexpr int kChunk = 4096;   // entries per block

__device__ __forceinline__ bool block_span(const SegTable* seg, uint32_t e0, uint32_t& s,
                                           uint32_t& sstart, uint32_t& nvalid) {
  if (seg->count == 0u || e0 >= seg->start[seg->count]) return false;
  s = segment_of(seg, e0);
  sstart = seg->start[s];
  const uint32_t send = sstart + seg->len[s];
  nvalid = send > e0 ? (send - e0 < uint32_t(kChunk) ? send - e0 : uint32_t(kChunk)) : 0u;
  return true;
}

// first[b] = depth position of the Gaussian whose entries contain the first
// entry of block b.
__global__ __launch_bounds__(kThreads) void first_gaussian_kernel(
    const uint64_t* __restrict__ offsets, const SegTable* __restrict__ seg, uint32_t n,
    uint32_t n_pad, uint32_t* __restrict__ first) {
  const uint32_t v = blockIdx.y;
  const uint32_t k = blockIdx.x * kThreads + threadIdx.x;
  if (seg->overflow || k >= n) return;
  const size_t row = size_t(v) * n_pad;
  const uint64_t o0 = offsets[row];
  const uint32_t a = uint32_t(offsets[row + k] - o0), b = uint32_t(offsets[row + k + 1] - o0);
  if (a == b) return;
  const uint32_t sb = seg->start[v] / uint32_t(kChunk);
  for (uint32_t blk = (a + kChunk - 1) / kChunk; blk * uint32_t(kChunk) < b; ++blk)
    first[sb + blk] = k;
}

// Adds the low digits of tiles [t, t + len) (consecutive ids) to a 256-bin
// difference array (plus a count added to every bin).
__device__ __forceinline__ void add_digit_range(int* diff, uint32_t* all, uint32_t t, uint32_t len) {
  if (len >= 256u) atomicAdd(all, len >> 8);
  const uint32_t rem = len & 255u;
  if (!rem) return;
  const uint32_t a = t & 255u, e = a + rem;
  atomicAdd(&diff[a], 1);
  if (e <= 256u) {
    atomicAdd(&diff[e], -1);
  } else {
    atomicAdd(&diff[256], -1);
    atomicAdd(&diff[0], 1);
    atomicAdd(&diff[e - 256u], -1);
  }
}

// Low-digit counts of every block's entries, from the row runs: the part of a
// Gaussian inside a block is a few runs of consecutive tile ids.  One thread
// per Gaussian walks its rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void lo_count_kernel(
    const uint32_t* __restrict__ order, const uint64_t* __restrict__ offsets,
    const Rect16* __restrict__ rects, const Rec<T>* __restrict__ recs,
    const ViewSlot* __restrict__ slots,
    const SegTable* __restrict__ seg, const uint32_t* __restrict__ first, uint32_t n,
    uint32_t n_pad, uint32_t* __restrict__ cnt) {
  __shared__ int s_diff[257];
  __shared__ uint32_t s_all;
  __shared__ uint32_t s_w[kThreads / 64];
  const uint32_t b = blockIdx.x;
  s_diff[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    s_diff[256] = 0;
    s_all = 0u;
  }
  __syncthreads();
  uint32_t s = 0, sstart = 0, nvalid = 0;
  if (!seg->overflow && block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) && nvalid) {
    const uint32_t lo = b * uint32_t(kChunk) - sstart, hi = lo + nvalid;  // render-local entries
    const size_t row = size_t(s) * n_pad;
    const uint64_t o0 = offsets[row];
    const ViewDev vd = slots[s].v;
    const uint32_t tiles_x = uint32_t(vd.tiles_x);
    const uint32_t k0 = first[b];
    for (uint32_t base = k0;; base += kThreads) {
      const uint32_t k = base + threadIdx.x;
      bool more = false;
      if (k < n) {
        const uint32_t a = uint32_t(offsets[row + k] - o0);
        const uint32_t e = uint32_t(offsets[row + k + 1] - o0);
        const uint32_t gi = order[row + k];
        if (a < hi) {
          more = true;
          const uint32_t c0 = a > lo ? a : lo, c1 = e < hi ? e : hi;
          if (c0 < c1) {
            const Rect16 r = rects[size_t(s) * n + gi];
            const SpanGeom sg = geom_of(recs[size_t(s) * n + gi], r, vd);
            const uint32_t q0 = c0 - a, q1 = c1 - a;
            uint32_t start = 0;  // local index of the row's first entry
            for (int y = r.y0; y < r.y1 && start < q1; ++y) {
              int x0, x1;
              row_span(sg, y, x0, x1);
              const uint32_t len = uint32_t(x1 - x0);
              const uint32_t j0 = start > q0 ? start : q0;
              const uint32_t j1 = start + len < q1 ? start + len : q1;
              if (j0 < j1)
                add_digit_range(s_diff, &s_all, uint32_t(y) * tiles_x + uint32_t(x0) + (j0 - start),
                                j1 - j0);
              start += len;
            }
          }
        }
      }
      if (!__syncthreads_or(more)) break;
    }
  }
  __syncthreads();
  uint32_t tot;
  const int x = s_diff[threadIdx.x];
  const uint32_t incl = block_excl_scan<kThreads>(uint32_t(x), s_w, &tot) + uint32_t(x);
  cnt[size_t(b) * 256 + threadIdx.x] = nvalid ? incl + s_all : 0u;
}

// Exclusive prefix of M[rows][256] along rows, per column: P[r][d] =
// sum_{r' < r} M[r'][d] for r <= rows.  Three steps: per-stripe prefixes and
// stripe totals, a scan of the stripe totals (one workgroup per column), and
// their addition.
constexpr int kStripe = 32;

__global__ __launch_bounds__(256) void col_scan_stripes_kernel(const uint32_t* __restrict__ M,
                                                               uint32_t rows,
                                                               uint32_t* __restrict__ P,
                                                               uint32_t* __restrict__ T) {
  const uint32_t d = threadIdx.x, st = blockIdx.x;
  const uint32_t r0 = st * kStripe;
  uint32_t vals[kStripe];
#pragma unroll
  for (int i = 0; i < kStripe; ++i) {
    const uint32_t r = r0 + i;
    vals[i] = r < rows ? M[size_t(r) * 256 + d] : 0u;
  }
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < kStripe; ++i) {
    const uint32_t r = r0 + i;
    if (r < rows) P[size_t(r) * 256 + d] = run;
    run += vals[i];
  }
  T[size_t(st) * 256 + d] = run;
}

__global__ __launch_bounds__(256) void col_scan_totals_kernel(uint32_t* __restrict__ T,
                                                              uint32_t stripes,
                                                              uint32_t* __restrict__ P,
                                                              uint32_t rows) {
  __shared__ uint32_t s_w[256 / 64];
  const uint32_t d = blockIdx.x;
  uint32_t run = 0;
  for (uint32_t s0 = 0; s0 < stripes; s0 += 256) {
    const uint32_t st = s0 + threadIdx.x;
    const uint32_t t = st < stripes ? T[size_t(st) * 256 + d] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<256>(t, s_w, &tot);
    if (st < stripes) T[size_t(st) * 256 + d] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) P[size_t(rows) * 256 + d] = run;
}

__global__ __launch_bounds__(256) void col_scan_add_kernel(uint32_t* __restrict__ P, uint32_t rows,
                                                           const uint32_t* __restrict__ T) {
  const uint32_t d = threadIdx.x, st = blockIdx.x;
  const uint32_t add = T[size_t(st) * 256 + d];
  const uint32_t r0 = st * kStripe;
#pragma unroll 8
  for (int i = 0; i < kStripe; ++i) {
    const uint32_t r = r0 + i;
    if (r < rows) P[size_t(r) * 256 + d] += add;
  }
}

// Per-digit output base of block b of the segment [first, end) of blocks:
// segment start + counts of lower digits in the segment + counts of digit d
// in the segment's earlier blocks.
__device__ __forceinline__ uint32_t digit_out_base(const uint32_t* __restrict__ P, uint32_t first,
                                                   uint32_t end, uint32_t b, uint32_t seg_start,
                                                   uint32_t* s_w) {
  const uint32_t d = threadIdx.x;
  const uint32_t pf = P[size_t(first) * 256 + d];
  const uint32_t tot_d = P[size_t(end) * 256 + d] - pf;
  uint32_t tot;
  const uint32_t lower = block_excl_scan<kThreads>(tot_d, s_w, &tot);
  return seg_start + lower + (P[size_t(b) * 256 + d] - pf);
}

// Stable rank of a block's entries by a digit of `nbits` bits (entries held in
// registers, wave w owning entries [w * 64 * ITEMS, (w + 1) * 64 * ITEMS)).
// pos[i] receives the entry's position in the block sorted by digit; s_start
// the exclusive prefix of the digit counts.
template <int ITEMS>
__device__ __forceinline__ void rank_block(const uint32_t (&dg)[ITEMS], uint32_t cn, int nbits,
                                           uint32_t (*s_wh)[256], uint32_t* s_start,
                                           uint32_t* s_w, uint32_t (&pos)[ITEMS]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s_wh[w][tid] = 0u;
  __syncthreads();
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool ok = wbase + uint32_t(i) * 64u + uint32_t(lane) < cn;
    const uint32_t d = dg[i];
    unsigned long long peers = __ballot(ok);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool x = (d >> bit) & 1u;
      const unsigned long long m = __ballot(x);
      peers &= x ? m : ~m;
    }
    const uint32_t base = s_wh[wave][d];
    const unsigned long long before = peers & lt;
    pos[i] = base + uint32_t(__popcll(before));
    if (ok && before == 0ull) s_wh[wave][d] = base + uint32_t(__popcll(peers));
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t t = s_wh[w][tid];
    s_wh[w][tid] = c;
    c += t;
  }
  uint32_t tot;
  s_start[tid] = block_excl_scan<kThreads>(c, s_w, &tot);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) pos[i] += s_start[dg[i]] + s_wh[wave][dg[i]];
}

// Low-digit pass: block b generates its entries (Gaussians from first[b] on,
// each one's part inside the block written by the lanes of one wavefront, one
// lane per tile row), ranks them stably by the low 8 bits of the tile id and
// writes them, as packed words, in runs of equal digit to their place in the
// segment.
template <typename T>
__global__ __launch_bounds__(kThreads) void lo_pass_kernel(
    const uint32_t* __restrict__ order, const uint64_t* __restrict__ offsets,
    const Rect16* __restrict__ rects, const Rec<T>* __restrict__ recs,
    const ViewSlot* __restrict__ slots,
    const SegTable* __restrict__ seg, const uint32_t* __restrict__ first,
    const uint32_t* __restrict__ P, uint32_t n, uint32_t n_pad, uint32_t* __restrict__ out) {
  constexpr int ITEMS = kChunk / kThreads;
  __shared__ uint32_t s_val[kChunk];
  __shared__ uint8_t s_dig[kChunk];
  __shared__ uint32_t s_base[256], s_start[256];
  __shared__ uint32_t s_wh[kThreads / 64][256];
  __shared__ uint32_t s_w[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid;
  if (seg->overflow || !block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid)
    return;
  const uint32_t send = sstart + seg->len[s];
  s_base[tid] = digit_out_base(P, sstart / uint32_t(kChunk),
                               (send + uint32_t(kChunk) - 1) / uint32_t(kChunk), b, sstart, s_w);
  const uint32_t lo = b * uint32_t(kChunk) - sstart, hi = lo + nvalid;  // render-local entries
  const size_t row = size_t(s) * n_pad;
  const uint64_t o0 = offsets[row];
  const ViewDev vd = slots[s].v;
  const uint32_t tiles_x = uint32_t(vd.tiles_x);
  // generate: wave w takes the Gaussians first[b] + 64 w + lane, then + 256, ...
  // every slot is written below; zeroed first so that no slot can hold a
  // stale value whatever the runs are
  for (uint32_t q = tid; q < nvalid; q += kThreads) {
    s_val[q] = 0u;
    s_dig[q] = 0u;
  }
  __syncthreads();
  const uint32_t k0 = first[b];
  for (uint32_t base = k0 + uint32_t(wave) * 64u;; base += kThreads) {
    const uint32_t k = base + uint32_t(lane);
    uint32_t a = hi, e = hi, gi = 0;
    if (k < n) {  // independent loads, issued together
      a = uint32_t(offsets[row + k] - o0);
      e = uint32_t(offsets[row + k + 1] - o0);
      gi = order[row + k];
    }
    const uint32_t c0 = a > lo ? a : lo, c1 = e < hi ? e : hi;
    const bool has = c0 < c1;
    unsigned long long todo = __ballot(has);
    while (todo) {
      const int src = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const uint32_t sa = __shfl(a, src, 64), s0 = __shfl(c0, src, 64), s1 = __shfl(c1, src, 64);
      const uint32_t sgi = __shfl(gi, src, 64);
      const Rect16 r = rects[size_t(s) * n + sgi];
      const SpanGeom sg = geom_of(recs[size_t(s) * n + sgi], r, vd);
      const uint32_t base_q = sa - lo;  // block slot of the Gaussian's entry 0
      wave_runs(sg, r.y0, r.y1, tiles_x, s0 - sa, s1 - sa, lane, [&](uint32_t j, uint32_t tile) {
        s_val[base_q + j] = sgi | ((tile >> 8) << 24);
        s_dig[base_q + j] = uint8_t(tile & 255u);
      });
    }
    // Gaussians start in increasing order: stop once every lane is past the block
    if (!__any(k < n && a < hi)) break;
  }
  __syncthreads();
  uint32_t v[ITEMS], dg[ITEMS], pos[ITEMS];
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    v[i] = q < nvalid ? s_val[q] : 0u;
    dg[i] = q < nvalid ? uint32_t(s_dig[q]) : 0u;
  }
  rank_block<ITEMS>(dg, nvalid, 8, s_wh, s_start, s_w, pos);
  // (rank_block's barriers separate the reads above from the writes below)
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    if (q < nvalid) {
      s_val[pos[i]] = v[i];
      s_dig[pos[i]] = uint8_t(dg[i]);
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < nvalid; p += kThreads) {
    const uint32_t d = s_dig[p];
    const uint32_t pos = s_base[d] + (p - s_start[d]);
    if (pos < send) out[pos] = s_val[p];
  }
}

// High-digit counts per block of the low-digit pass output.
__global__ __launch_bounds__(kThreads) void hi_count_kernel(const uint32_t* __restrict__ in,
                                                            const SegTable* __restrict__ seg,
                                                            uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_h[kThreads / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s_h[w][tid] = 0u;
  __syncthreads();
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid = 0;
  if (block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid)) {
    const uint32_t e0 = b * uint32_t(kChunk);
    for (uint32_t q = tid; q < nvalid; q += kThreads) atomicAdd(&s_h[wave][in[e0 + q] >> 24], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) c += s_h[w][tid];
  cnt[size_t(b) * 256 + tid] = c;
}

// High-digit pass: stable scatter of each block's entries by the high tile
// digit (nbits significant bits); writes the Gaussian index (bits 0..23).
__global__ __launch_bounds__(kThreads) void hi_pass_kernel(const uint32_t* __restrict__ in,
                                                           const SegTable* __restrict__ seg,
                                                           const uint32_t* __restrict__ P,
                                                           int nbits,
                                                           uint32_t* __restrict__ values) {
  constexpr int ITEMS = kChunk / kThreads;
  __shared__ uint32_t s_sorted[kChunk];
  __shared__ uint32_t s_base[256], s_start[256];
  __shared__ uint32_t s_wh[kThreads / 64][256];
  __shared__ uint32_t s_w[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid;
  if (!block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid) return;
  const uint32_t send = sstart + seg->len[s];
  const uint32_t e0 = b * uint32_t(kChunk);
  uint32_t x[ITEMS], dg[ITEMS], pos[ITEMS];
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    x[i] = q < nvalid ? in[e0 + q] : 0u;
    dg[i] = x[i] >> 24;
  }
  s_base[tid] = digit_out_base(P, sstart / uint32_t(kChunk),
                               (send + uint32_t(kChunk) - 1) / uint32_t(kChunk), b, sstart, s_w);
  rank_block<ITEMS>(dg, nvalid, nbits, s_wh, s_start, s_w, pos);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    if (q < nvalid) s_sorted[pos[i]] = x[i];
  }
  __syncthreads();
  for (uint32_t p = tid; p < nvalid; p += kThreads) {
    const uint32_t y = s_sorted[p];
    const uint32_t d = y >> 24;
    values[s_base[d] + (p - s_start[d])] = y & 0xffffffu;
  }
}

}  // namespace

hipError_t fill_const(void* p, size_t count, double value, bool f64, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(fill_const_kernel<double>, dim3(grid_for(count)), dim3(kThreads), 0, stream,
                       static_cast<double*>(p), count, value);
  else
    hipLaunchKernelGGL(fill_const_kernel<float>, dim3(grid_for(count)), dim3(kThreads), 0, stream,
                       static_cast<float*>(p), count, float(value));
  return hipGetLastError();
}

template <typename T>
hipError_t add_grads(const GradPtrs<T>& out, const T* tmp, size_t n, size_t k3,
                     hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(add_grads_kernel<T>, dim3(grid_for((17 + k3) * n)), dim3(kThreads), 0, stream,
                     out, tmp, n, k3);
  return hipGetLastError();
}
template hipError_t add_grads<float>(const GradPtrs<float>&, const float*, size_t, size_t,
                                     hipStream_t);
template hipError_t add_grads<double>(const GradPtrs<double>&, const double*, size_t, size_t,
                                      hipStream_t);

hipError_t copy_ranges_rebased(const uint2* src, uint32_t count, uint32_t base, uint2* dst,
                               hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(rebase_ranges_kernel, dim3((count + kThreads - 1) / kThreads), dim3(kThreads),
                     0, stream, src, count, base, dst);
  return hipGetLastError();
}

hipError_t fill_zero(void* p, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return hipSuccess;
  if ((bytes & 15u) || (reinterpret_cast<uintptr_t>(p) & 15u)) return hipErrorInvalidValue;
  const uint64_t n16 = bytes / 16;
  uint64_t blocks = (n16 + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(uint32_t(blocks)), dim3(kThreads), 0, stream,
                     static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

uint32_t sort_status_words(uint64_t capacity_elems, int items) {
  const uint64_t tile = uint64_t(kThreads) * items;
  return uint32_t((capacity_elems + tile - 1) / tile * 256u);
}

hipError_t radix_histogram(const uint32_t* keys, const SegTable* seg, int n_segments,
                           uint32_t max_len, int passes, uint32_t* hist, hipStream_t stream) {
  if (max_len == 0 || n_segments <= 0) return hipSuccess;
  const uint32_t chunk = 4096;
  const dim3 grid((max_len + chunk - 1) / chunk, uint32_t(n_segments));
  switch (passes) {
    case 1: hipLaunchKernelGGL(radix_hist_kernel<1>, grid, dim3(kThreads), 0, stream, keys, seg, chunk, hist); break;
    case 2: hipLaunchKernelGGL(radix_hist_kernel<2>, grid, dim3(kThreads), 0, stream, keys, seg, chunk, hist); break;
    case 3: hipLaunchKernelGGL(radix_hist_kernel<3>, grid, dim3(kThreads), 0, stream, keys, seg, chunk, hist); break;
    case 4: hipLaunchKernelGGL(radix_hist_kernel<4>, grid, dim3(kThreads), 0, stream, keys, seg, chunk, hist); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t onesweep_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* key_bufs[2],
                         uint32_t* val_bufs[2], const SegTable* seg, uint64_t capacity_elems,
                         int passes, int items, const uint32_t* hist, uint32_t* status,
                         uint32_t* tickets, uint32_t* error, bool keys_needed, int* result_index,
                         hipStream_t stream) {
  *result_index = (passes - 1) & 1;
  if (capacity_elems == 0 || passes <= 0) return hipSuccess;
  const uint64_t tile = uint64_t(kThreads) * items;
  const uint32_t blocks = uint32_t((capacity_elems + tile - 1) / tile);
  const uint32_t words = blocks * 256u;
  for (int p = 0; p < passes; ++p) {
    const uint32_t* ki = p == 0 ? keys_in : key_bufs[(p - 1) & 1];
    const uint32_t* vi = p == 0 ? vals_in : val_bufs[(p - 1) & 1];
    uint32_t* ko = (keys_needed || p + 1 < passes) ? key_bufs[p & 1] : nullptr;
    uint32_t* vo = val_bufs[p & 1];
    const uint32_t* h = hist + size_t(p) * kMaxViews * 256;
    uint32_t* st = status + size_t(p) * words;
    switch (items) {
      case 4:
        hipLaunchKernelGGL(onesweep_kernel<4>, dim3(blocks), dim3(kThreads), 0, stream, ki, vi,
                           ko, vo, seg, h, st, tickets + p, error, 8 * p);
        break;
      case 8:
        hipLaunchKernelGGL(onesweep_kernel<8>, dim3(blocks), dim3(kThreads), 0, stream, ki, vi,
                           ko, vo, seg, h, st, tickets + p, error, 8 * p);
        break;
      case 16:
        hipLaunchKernelGGL(onesweep_kernel<16>, dim3(blocks), dim3(kThreads), 0, stream, ki, vi,
                           ko, vo, seg, h, st, tickets + p, error, 8 * p);
        break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int tile_grid_partials(uint32_t n) {
  const uint32_t b = (n + 8191) / 8192;
  return int(b < 1 ? 1 : (b > 64 ? 64 : b));
}

size_t tile_grid_lds_limit() {
  static const size_t limit = [] {
    int dev = 0, bytes = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
      (void)hipGetLastError();
      bytes = 65536;
    }
    // leave room for the counting kernel's static LDS
    const size_t b = size_t(bytes) > 8192 ? size_t(bytes) - 8192 : 0;
    if (b > 65536) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(tile_grid_kernel<float, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(b));
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(tile_grid_kernel<double, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(b));
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(tile_count_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(b));
      (void)hipGetLastError();
    }
    return b;
  }();
  return limit;
}

template <typename T>
hipError_t tile_grids(const Rect16* rects, const Rec<T>* recs, const ViewSlot* slots,
                      int n_views, uint32_t n, uint64_t max_cells, uint64_t total_cells,
                      int* partials, int* grid, hipStream_t stream) {
  if (n == 0 || n_views <= 0) return hipSuccess;
  const int B = tile_grid_partials(n);
  const dim3 g{uint32_t(B), uint32_t(n_views), 1u};
  const size_t lds = size_t(max_cells) * 4;
  if (lds <= tile_grid_lds_limit()) {
    hipLaunchKernelGGL((tile_grid_kernel<T, true>), g, dim3(kThreads), lds, stream, rects, recs,
                       slots, n, partials, grid);
    hipLaunchKernelGGL(grid_sum_kernel, dim3(uint32_t((total_cells + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, stream, slots, n_views, partials, B,
                       uint32_t(total_cells), grid);
  } else {
    hipLaunchKernelGGL((tile_grid_kernel<T, false>), g, dim3(kThreads), 0, stream, rects, recs,
                       slots, n, partials, grid);
  }
  return hipGetLastError();
}

template hipError_t tile_grids<float>(const Rect16*, const Rec<float>*, const ViewSlot*, int,
                                      uint32_t, uint64_t, uint64_t, int*, int*, hipStream_t);
template hipError_t tile_grids<double>(const Rect16*, const Rec<double>*, const ViewSlot*, int,
                                       uint32_t, uint64_t, uint64_t, int*, int*, hipStream_t);

hipError_t tile_counts(const ViewSlot* slots, int n_views, uint64_t max_cells, int* grid,
                       const unsigned long long* totals, unsigned long long capacity,
                       uint2* ranges, uint32_t* hist, SegTable* seg, hipStream_t stream) {
  const size_t lds = size_t(max_cells) * 4;
  if (lds <= tile_grid_lds_limit())
    hipLaunchKernelGGL(tile_count_kernel<true>, dim3(n_views), dim3(kTcThreads), lds, stream,
                       slots, n_views, grid, totals, capacity, ranges, hist, seg);
  else
    hipLaunchKernelGGL(tile_count_kernel<false>, dim3(n_views), dim3(kTcThreads), 0, stream,
                       slots, n_views, grid, totals, capacity, ranges, hist, seg);
  return hipGetLastError();
}

size_t scan_u32_temp_bytes(uint32_t n) {
  return (scan_temp_elems(uint64_t(n) + 1) + 4) * sizeof(uint32_t);
}

hipError_t scan_u32(const uint32_t* a, uint32_t n, uint32_t* out, void* temp, hipStream_t stream) {
  return device_exclusive_scan<uint32_t, LoadT<uint32_t>>(LoadT<uint32_t>{a, n}, out,
                                                          uint64_t(n) + 1,
                                                          static_cast<uint32_t*>(temp), stream);
}

size_t count_scan_seg_temp_bytes(uint32_t n_pad, int n_views) {
  return (scan_temp_elems(uint64_t(n_pad) * uint64_t(n_views) + 1) + 2) * sizeof(uint64_t);
}

hipError_t count_scan_seg(const uint32_t* order, const uint32_t* counts, uint32_t n,
                          uint32_t n_pad, int n_views, uint64_t* offsets, void* temp,
                          hipStream_t stream) {
  const uint64_t total = uint64_t(n_pad) * uint64_t(n_views);
  return device_exclusive_scan<uint64_t, LoadCountGatherSeg>(
      LoadCountGatherSeg{order, counts, n, n_pad, total}, offsets, total + 1,
      static_cast<uint64_t*>(temp), stream);
}

template <typename T>
hipError_t emit_tile_keys_seg(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                              const Rec<T>* recs, const ViewSlot* slots, const SegTable* seg,
                              uint32_t n, uint32_t n_pad, int n_views, uint32_t* keys,
                              uint32_t* vals, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(emit_kernel<T>, dim3((n + 255) / 256, uint32_t(n_views)), dim3(256), 0,
                     stream, order, offsets, rects, recs, slots, seg, n, n_pad, keys, vals);
  return hipGetLastError();
}

template hipError_t emit_tile_keys_seg<float>(const uint32_t*, const uint64_t*, const Rect16*,
                                              const Rec<float>*, const ViewSlot*, const SegTable*,
                                              uint32_t, uint32_t, int, uint32_t*, uint32_t*,
                                              hipStream_t);
template hipError_t emit_tile_keys_seg<double>(const uint32_t*, const uint64_t*, const Rect16*,
                                               const Rec<double>*, const ViewSlot*,
                                               const SegTable*, uint32_t, uint32_t, int, uint32_t*,
                                               uint32_t*, hipStream_t);

bool packed_tile_sort_ok(uint32_t n, uint32_t max_tiles_per_view) {
  return n <= (1u << 24) && max_tiles_per_view <= 65536u;
}

size_t packed_sort_temp_bytes(uint32_t n_pad, int n_views, uint64_t capacity) {
  (void)n_pad;
  (void)n_views;
  const uint64_t rows = (capacity + kChunk - 1) / kChunk;
  const uint64_t stripes = (rows + kStripe - 1) / kStripe + 1;
  // first[], and per pass: M, P, stripe totals
  return size_t((rows + 64) * 4 + 2 * (rows * 256 + (rows + 1) * 256 + stripes * 256) * 4);
}

namespace {
hipError_t col_scan(const uint32_t* M, uint32_t rows, uint32_t* P, uint32_t* T,
                    hipStream_t stream) {
  const uint32_t stripes = (rows + kStripe - 1) / kStripe;
  if (stripes > 0)
    hipLaunchKernelGGL(col_scan_stripes_kernel, dim3(stripes), dim3(256), 0, stream, M, rows, P,
                       T);
  hipLaunchKernelGGL(col_scan_totals_kernel, dim3(256), dim3(256), 0, stream, T, stripes, P, rows);
  if (stripes > 0)
    hipLaunchKernelGGL(col_scan_add_kernel, dim3(stripes), dim3(256), 0, stream, P, rows, T);
  return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t packed_tile_sort(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                            const Rec<T>* recs, const ViewSlot* slots, const SegTable* seg,
                            uint32_t n, uint32_t n_pad, int n_views, uint32_t max_tiles,
                            uint64_t capacity, void* temp, uint32_t* lo_out, uint32_t* values,
                            hipStream_t stream) {
  const uint32_t rows = uint32_t((capacity + kChunk - 1) / kChunk);
  if (n == 0 || n_views <= 0 || rows == 0) return hipSuccess;
  const uint32_t stripes = (rows + kStripe - 1) / kStripe + 1;
  uint32_t* first = static_cast<uint32_t*>(temp);
  uint32_t* M1 = first + rows + 64;
  uint32_t* P1 = M1 + size_t(rows) * 256;
  uint32_t* T1 = P1 + size_t(rows + 1) * 256;
  uint32_t* M2 = T1 + size_t(stripes) * 256;
  uint32_t* P2 = M2 + size_t(rows) * 256;
  uint32_t* T2 = P2 + size_t(rows + 1) * 256;
  hipLaunchKernelGGL(first_gaussian_kernel, dim3((n + kThreads - 1) / kThreads, uint32_t(n_views)),
                     dim3(kThreads), 0, stream, offsets, seg, n, n_pad, first);
  hipLaunchKernelGGL(lo_count_kernel<T>, dim3(rows), dim3(kThreads), 0, stream, order, offsets,
                     rects, recs, slots, seg, first, n, n_pad, M1);
  hipError_t e = col_scan(M1, rows, P1, T1, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lo_pass_kernel<T>, dim3(rows), dim3(kThreads), 0, stream, order, offsets,
                     rects, recs, slots, seg, first, P1, n, n_pad, lo_out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(hi_count_kernel, dim3(rows), dim3(kThreads), 0, stream, lo_out, seg, M2);
  if ((e = col_scan(M2, rows, P2, T2, stream)) != hipSuccess) return e;
  int nbits = 1;
  while ((1u << nbits) < (max_tiles + 255u) / 256u) ++nbits;
  hipLaunchKernelGGL(hi_pass_kernel, dim3(rows), dim3(kThreads), 0, stream, lo_out, seg, P2,
                     nbits, values);
  return hipGetLastError();
}

template hipError_t packed_tile_sort<float>(const uint32_t*, const uint64_t*, const Rect16*,
                                            const Rec<float>*, const ViewSlot*, const SegTable*,
                                            uint32_t, uint32_t, int, uint32_t, uint64_t, void*,
                                            uint32_t*, uint32_t*, hipStream_t);
template hipError_t packed_tile_sort<double>(const uint32_t*, const uint64_t*, const Rect16*,
                                             const Rec<double>*, const ViewSlot*,
                                             const SegTable*, uint32_t, uint32_t, int, uint32_t,
                                             uint64_t, void*, uint32_t*, uint32_t*, hipStream_t);

}  // namespace r4d
