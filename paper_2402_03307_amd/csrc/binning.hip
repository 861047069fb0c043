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

#include <type_traits>

#include "front.hpp"
#include "r4d_internal.hpp"
#include "rowwalk.hpp"
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
  if constexpr (sizeof(T) == 4) {
    // (32-bit values: lane moves, rowwalk.hpp; two's complement makes it hold
    // for signed values too)
    return T(wave_incl_scan_u32(uint32_t(x), lane));
  } else {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const T y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    return x;
  }
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

// Digit histograms of keys, PASSES digits of 8 bits, per segment (blockIdx.y),
// kHistItems keys per thread, all loaded before the first count.  Same-address
// LDS atomics are serialised, and the top two digits of depths are shared by
// many keys: for those, the lanes of a wavefront whose digit equals the first
// lane's add their number with one atomic.
constexpr uint32_t kHistItems = 8;
constexpr uint32_t kHistChunk = uint32_t(kThreads) * kHistItems;

template <int PASSES>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              const SegTable* __restrict__ seg,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[PASSES][256];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) h[p][threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t s = blockIdx.y;
  if (s < seg->count) {
    const uint32_t s0 = seg->start[s];
    const uint32_t begin = s0 + blockIdx.x * kHistChunk + threadIdx.x;
    const uint32_t send = s0 + seg->len[s];
    const int lane = threadIdx.x & 63;
    uint32_t k[kHistItems];
#pragma unroll
    for (uint32_t i = 0; i < kHistItems; ++i) {
      const uint32_t j = begin + i * kThreads;
      k[i] = j < send ? keys[j] : 0u;
    }
#pragma unroll
    for (uint32_t i = 0; i < kHistItems; ++i) {
      // lane 0 holds the wavefront's first key of the step: when it is past
      // the end, so is every other lane's
      const bool ok = begin + i * kThreads < send;
#pragma unroll
      for (int p = 0; p < PASSES; ++p) {
        const uint32_t d = (k[i] >> (8 * p)) & 255u;
        if (p < 2) {
          if (ok) atomicAdd(&h[p][d], 1u);
          continue;
        }
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const unsigned long long same = __ballot(ok && d == d0);
        if (ok && d != d0) atomicAdd(&h[p][d], 1u);
        if (same && lane == 0) atomicAdd(&h[p][d0], uint32_t(__popcll(same)));
      }
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
  // position in the sort order: the launch order (ticket), or, when every
  // workgroup of the grid is resident at once (ticket null), the block index
  if (tid == 0) s_bid = ticket ? atomicAdd(ticket, 1u) : blockIdx.x;
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
  // past its segment's keys (every later workgroup of the segment is too, and
  // the next segment's look-back stops at its own first workgroup): nothing
  // to publish
  if (e0 >= send) return;
  const uint32_t nvalid = send - e0 < TILE ? send - e0 : TILE;
  // a digit every key of the segment shares (one bin of the segment's
  // histogram holds them all, as the top byte of depths within one binade):
  // the pass keeps the order, so the tile is copied as it is
  if (hist[size_t(s) * 256u + ((keys_in[sstart] >> shift) & 255u)] == send - sstart) {
    for (uint32_t q = uint32_t(tid); q < nvalid; q += kThreads) {
      if (keys_out) keys_out[e0 + q] = keys_in[e0 + q];
      vals_out[e0 + q] = vals_in ? vals_in[e0 + q] : e0 + q - sstart;
    }
    return;
  }

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

// Segment table of the emitted list: render v's entries start at the sum of
// the earlier renders' counts, each rounded up to 4096.  When the entries do
// not fit the capacity (or a render exceeds the per-segment limit) every
// segment is empty and `overflow` is set.
__device__ void write_seg_table(const unsigned long long* __restrict__ totals,
                                const ViewSlot* __restrict__ slots, int n_views,
                                unsigned long long capacity, SegTable* __restrict__ seg,
                                uint32_t* __restrict__ overflow_out) {
  unsigned long long total = 0;
  bool too_long = false;
  for (int v = 0; v < n_views; ++v) {
    const unsigned long long d = totals[2 * v + 1];
    total += seg_extent(d, slots[v]);
    too_long |= d > kStatMask;
  }
  const bool overflow = too_long || total > capacity;
  unsigned long long base = 0;
  for (int v = 0; v < n_views; ++v) {
    const unsigned long long d = totals[2 * v + 1];
    seg->start[v] = overflow ? 0u : uint32_t(base);
    seg->len[v] = overflow ? 0u : uint32_t(d);
    base += seg_extent(d, slots[v]);
  }
  seg->start[n_views] = overflow ? 0u : uint32_t(total);
  seg->count = uint32_t(n_views);
  seg->overflow = overflow ? 1u : 0u;
  if (overflow_out) *overflow_out = overflow ? 1u : 0u;
}

__global__ void seg_table_kernel(const unsigned long long* __restrict__ totals,
                                 const ViewSlot* __restrict__ slots, int n_views,
                                 unsigned long long capacity, SegTable* __restrict__ seg,
                                 uint32_t* __restrict__ overflow_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  write_seg_table(totals, slots, n_views, capacity, seg, overflow_out);
}

struct LoadCountGatherSeg {
  const uint32_t* order;  // [V][n_pad] Gaussian index in depth order
  const uint32_t* counts; // [V][n]
  const unsigned long long* totals;  // totals[2v]: render v's visible Gaussians
  uint32_t n, n_pad;
  uint64_t total;         // V * n_pad
  __device__ uint64_t operator()(uint64_t i) const {
    if (i >= total) return 0;
    const uint32_t v = uint32_t(i / n_pad), k = uint32_t(i % n_pad);
    // only the visible Gaussians are sorted (the rest of a render's order is unset)
    return k < uint32_t(totals[2 * v]) ? uint64_t(counts[size_t(v) * n + order[i]]) : uint64_t(0);
  }
};

template <typename T>
__global__ __launch_bounds__(kThreads) void fill_const_kernel(T* __restrict__ p, size_t count,
                                                              T value) {
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < count; i += stride) p[i] = value;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void add_grads_kernel(GradPtrs<T> out,
                                                             const T* __restrict__ tmp, size_t n,
                                                             size_t k3, uint32_t rm, uint32_t rl,
                                                             uint32_t rr) {
  const size_t e1 = rm * n, e2 = e1 + rl * n, e3 = e2 + rr * n, e4 = e3 + n;
  const size_t total = e4 + k3 * n;
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < total; i += stride) {
    T* dst;
    if (i < e1)
      dst = out.means + i;
    else if (i < e2)
      dst = out.log_scales + (i - e1);
    else if (i < e3)
      dst = out.rotors + (i - e2);
    else if (i < e4)
      dst = out.opacity + (i - e3);
    else
      dst = out.sh + (i - e4);
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
// high 8 bits of the tile id in bits 24..31; the low 8 bits ride along as one
// byte per entry for the first pass.  The entries of a render are numbered in
// emission order (Gaussians in depth order, each one's tiles row by row) and
// cut into blocks of 4096; block b of the render is also block b of its
// segment of the sorted output.  Both passes are reduce-then-scan: per-block
// digit counts, a column scan of those counts, then a stable scatter, so no
// workgroup waits on another.
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

// ---- the count scan: offsets[i] = exclusive prefix of the tile counts in depth
// order (renders back to back, each padded to n_pad), in two launches over
// tiles of kScanTile elements; the first also writes the segment table of the
// emitted list (workgroup 0), the second the first Gaussian of every emission
// block (first_gaussian_kernel's map) and, when the counts are those of front
// lists, each render's front entry count (its segment length) and rest area.
// With at most kCountDirectTiles tiles every tile adds up the sums of the
// tiles before it itself; beyond, the tile sums are scanned in between
// (device_exclusive_scan).
constexpr uint32_t kCountDirectTiles = 2048;

// Per-Gaussian counts as front_counts_kernel wrote them ([V][n_pad]).
struct LoadCountPlain {
  const uint32_t* counts;
  uint64_t total;
  __device__ uint64_t operator()(uint64_t i) const { return i < total ? counts[i] : 0ull; }
};

template <typename Loader>
__global__ __launch_bounds__(kThreads) void count_sums_kernel(
    Loader ld, uint64_t* __restrict__ tile_sums, const unsigned long long* __restrict__ totals,
    const ViewSlot* __restrict__ slots, int n_views, unsigned long long capacity,
    SegTable* __restrict__ seg, uint32_t* __restrict__ overflow_out) {
  __shared__ uint64_t s_w[kThreads / 64];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    write_seg_table(totals, slots, n_views, capacity, seg, overflow_out);
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  uint64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) sum += ld(base + j);
  uint64_t total;
  block_excl_scan<kThreads>(sum, s_w, &total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// scanned: exclusive scan of the tile sums, or null (direct: add them here).
// front (nullable): the counts are front-list counts; the render's last tile
// sets its segment length and rest area.
template <typename Loader>
__global__ __launch_bounds__(kThreads) void count_offsets_kernel(
    Loader ld, uint32_t n, uint32_t n_pad, uint64_t n_elems,
    const uint64_t* __restrict__ tile_sums, const uint64_t* __restrict__ scanned,
    SegTable* __restrict__ seg, FrontTable* __restrict__ front, uint64_t* __restrict__ offsets,
    uint32_t* __restrict__ first) {
  __shared__ uint64_t s_w[kThreads / 64];
  __shared__ uint64_t s_pre[2];
  const uint32_t b = blockIdx.x;
  // the render of this tile (tiles never straddle renders: n_pad is a
  // multiple of kScanTile) and the tile where the render starts
  const uint64_t e_first = uint64_t(b) * kScanTile;
  const uint32_t v = uint32_t(e_first / n_pad);
  const uint64_t row = uint64_t(v) * n_pad;
  const uint32_t rt = uint32_t(row / kScanTile);
  if (scanned) {
    if (threadIdx.x == 0) {
      s_pre[0] = scanned[b];
      s_pre[1] = scanned[rt];
    }
  } else {
    uint64_t pre = 0, pre_row = 0;
    for (uint32_t t = threadIdx.x; t < b; t += kThreads) {
      const uint64_t x = tile_sums[t];
      pre += x;
      pre_row += t < rt ? x : 0ull;
    }
    uint64_t tot;
    block_excl_scan<kThreads>(pre, s_w, &tot);
    if (threadIdx.x == 0) s_pre[0] = tot;
    block_excl_scan<kThreads>(pre_row, s_w, &tot);
    if (threadIdx.x == 0) s_pre[1] = tot;
  }
  const uint64_t base = e_first + uint64_t(threadIdx.x) * kScanItems;
  uint64_t x[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    x[j] = ld(base + j);
    sum += x[j];
  }
  uint64_t total;
  uint64_t run = block_excl_scan<kThreads>(sum, s_w, &total) + s_pre[0];
  const uint64_t o0 = s_pre[1];  // offsets[row]: where the render's entries start
  const bool map = !seg->overflow && v < seg->count;
  const uint32_t sb = map ? seg->start[v] / uint32_t(kChunk) : 0u;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint64_t i = base + j;
    if (i < n_elems) offsets[i] = run;
    // the Gaussian at depth position k holds entries [a, b) of its render;
    // it starts block blk when blk * kChunk lies in [a, b)
    const uint32_t k = uint32_t(i - row);
    if (map && i < n_elems && k < n && x[j] != 0) {
      const uint32_t a = uint32_t(run - o0), e = uint32_t(run + x[j] - o0);
      for (uint32_t blk = (a + kChunk - 1) / kChunk; blk * uint32_t(kChunk) < e; ++blk)
        first[sb + blk] = k;
    }
    run += x[j];
  }
  // front lists: the render's entries are its front entries
  if (front && map && e_first + kScanTile == row + n_pad && threadIdx.x == kThreads - 1) {
    const uint32_t d = uint32_t(run - o0);
    seg->len[v] = d;
    front->n_front[v] = d;
    front->app_base[v] = seg->start[v] + (d + kSegment - 1) / kSegment * kSegment;
    front->app_end[v] = seg->start[v + 1];
  }
}

// ---- front lists (front.hpp)
// Keep bitmap of every render with a depth cut: a tile is kept when at most
// `keep` tile boxes of the render's front Gaussians (depth positions below
// its cut r0) cover it.  Each box is counted as +1 / -1 at its corners into a
// grid whose 2D prefix sums are the cover counts: kKeepGroups workgroups per
// render each take a share of the positions [0, r0) in depth order, count it
// in LDS and add it into the render's grid in memory (cover, zeroed
// beforehand); front_bits_kernel then sums the grid and writes the bits.
// Renders with more than kKeepGrid grid cells get no cut (the host leaves
// front16 at 0 for them).
constexpr int kKeepThreads = 1024;
constexpr int kKeepGroups = 16;
constexpr int kKeepGrid = 16384;
constexpr int kKeepWordsMax = 512;  // keep bitmap words of a render (LDS copies)

// The render's keep bitmap into LDS (the row walks test it for every row).
__device__ __forceinline__ void load_keep(uint64_t* s_keep, const uint64_t* __restrict__ bits,
                                          const ViewSlot& sl) {
  const int nw = int(keep_words(sl.v.tiles_x)) * sl.v.tiles_y;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) s_keep[i] = bits[sl.keep_base + i];
}

__global__ __launch_bounds__(kKeepThreads) void front_keep_kernel(
    const ViewSlot* __restrict__ slots, const Rect16* __restrict__ rects,
    const uint32_t* __restrict__ order, const unsigned long long* __restrict__ totals, uint32_t n,
    uint32_t n_pad, int32_t* __restrict__ cover) {
  __shared__ int32_t s_c[kKeepGrid];
  const uint32_t v = blockIdx.y;
  const ViewSlot& sl = slots[v];
  if (!sl.front16) return;
  const uint32_t r0 = front_cut(uint32_t(totals[2 * v]), sl.front16);
  const uint32_t share = (r0 + kKeepGroups - 1) / kKeepGroups;
  const uint32_t kb = blockIdx.x * share;
  const uint32_t ke = kb + share < r0 ? kb + share : r0;
  if (kb >= ke) return;  // (the whole workgroup)
  const int tx = sl.v.tiles_x, ty = sl.v.tiles_y, w1 = tx + 1, h1 = ty + 1;
  for (int i = threadIdx.x; i < w1 * h1; i += kKeepThreads) s_c[i] = 0;
  __syncthreads();
  for (uint32_t k = kb + threadIdx.x; k < ke; k += kKeepThreads) {
    const Rect16 r = rects[size_t(v) * n + order[size_t(v) * n_pad + k]];
    // (corners on the last row or column change no tile's sum)
    atomicAdd(&s_c[int(r.y0) * w1 + int(r.x0)], 1);
    if (int(r.x1) < tx) atomicAdd(&s_c[int(r.y0) * w1 + int(r.x1)], -1);
    if (int(r.y1) < ty) {
      atomicAdd(&s_c[int(r.y1) * w1 + int(r.x0)], -1);
      if (int(r.x1) < tx) atomicAdd(&s_c[int(r.y1) * w1 + int(r.x1)], 1);
    }
  }
  __syncthreads();
  int32_t* __restrict__ g = cover + sl.cover_base;
  for (int i = threadIdx.x; i < w1 * h1; i += kKeepThreads) {
    const int32_t x = s_c[i];
    if (x) atomicAdd(&g[i], x);
  }
}

// The bits from the summed cover grids: one workgroup per render.
__global__ __launch_bounds__(kKeepThreads) void front_bits_kernel(
    const ViewSlot* __restrict__ slots, const int32_t* __restrict__ cover, int32_t keep,
    uint64_t* __restrict__ bits) {
  __shared__ int32_t s_c[kKeepGrid];
  const uint32_t v = blockIdx.x;
  const ViewSlot& sl = slots[v];
  if (!sl.front16) return;
  const int tx = sl.v.tiles_x, ty = sl.v.tiles_y, w1 = tx + 1, h1 = ty + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = kKeepThreads / 64;
  const int32_t* __restrict__ g = cover + sl.cover_base;
  for (int i = threadIdx.x; i < w1 * h1; i += kKeepThreads) s_c[i] = g[i];
  __syncthreads();
  // prefix sums along the rows, then down the columns: a wavefront per line,
  // four lines interleaved
  for (int r0 = wave * 4; r0 < ty; r0 += NW * 4) {
    int32_t carry[4] = {0, 0, 0, 0};
    for (int c0 = 0; c0 < tx; c0 += 64) {
      const int c = c0 + lane;
      int32_t x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = (r0 + q < ty && c < tx) ? s_c[(r0 + q) * w1 + c] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = wave_incl_scan(x[q], lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (r0 + q < ty && c < tx) s_c[(r0 + q) * w1 + c] = carry[q] + x[q];
        carry[q] += __shfl(x[q], 63, 64);
      }
    }
  }
  __syncthreads();
  for (int c0w = wave * 4; c0w < tx; c0w += NW * 4) {
    int32_t carry[4] = {0, 0, 0, 0};
    for (int rr = 0; rr < ty; rr += 64) {
      const int r = rr + lane;
      int32_t x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = (c0w + q < tx && r < ty) ? s_c[r * w1 + c0w + q] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = wave_incl_scan(x[q], lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (c0w + q < tx && r < ty) s_c[r * w1 + c0w + q] = carry[q] + x[q];
        carry[q] += __shfl(x[q], 63, 64);
      }
    }
  }
  __syncthreads();
  const int words = int(keep_words(tx));
  for (int q = wave; q < ty * words; q += NW) {
    const int y = q / words, x = (q % words) * 64 + lane;
    const unsigned long long m = __ballot(x < tx && s_c[y * w1 + x] <= keep);
    if (lane == 0) bits[sl.keep_base + q] = m;
  }
}

// Per-Gaussian entry counts in depth order for front lists, counts[v][k]
// (k < n_pad): the whole count below the render's depth cut r0, from r0 on the
// kept tiles of the Gaussian's row runs, 0 past the visible Gaussians.  Also
// copies the tile boxes of positions [r0, n_vis) into depth order (srect), for
// the rasteriser's collection of a tile's rest entries.  The rows of a
// wavefront's Gaussians are walked together (rowwalk.hpp).
template <typename T>
__global__ __launch_bounds__(kThreads) void front_counts_kernel(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ whole,
    const Rect16* __restrict__ rects, const Rec<T>* __restrict__ recs,
    const ViewSlot* __restrict__ slots, const unsigned long long* __restrict__ totals,
    const uint64_t* __restrict__ bits, uint32_t n, uint32_t n_pad, uint64_t total,
    uint32_t* __restrict__ counts, Rect16* __restrict__ srect, uint64_t* __restrict__ tile_sums,
    int n_views, unsigned long long capacity, SegTable* __restrict__ seg,
    uint32_t* __restrict__ overflow_out) {
  __shared__ uint32_t s_cnt[kThreads];
  __shared__ uint64_t s_keep[kKeepWordsMax];
  __shared__ uint32_t s_part[kThreads / 64];
  const uint64_t i0 = uint64_t(blockIdx.x) * kThreads;
  if (i0 >= total) return;  // (whole workgroups only)
  if (blockIdx.x == 0 && threadIdx.x == 0)
    write_seg_table(totals, slots, n_views, capacity, seg, overflow_out);
  const uint64_t i = i0 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  // the workgroup's counts into its tile of the count scan (the whole
  // workgroup; a tile holds kScanTile / kThreads workgroups)
  auto add_sum = [&](uint32_t c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t t = 0;
#pragma unroll
      for (int w = 0; w < kThreads / 64; ++w) t += s_part[w];
      if (t) atomicAdd(reinterpret_cast<unsigned long long*>(&tile_sums[i0 / kScanTile]),
                       static_cast<unsigned long long>(t));
    }
  };
  const uint32_t v = uint32_t(i0 / n_pad);  // n_pad % kThreads == 0: one render per workgroup
  const uint32_t k = uint32_t(i - uint64_t(v) * n_pad);
  const ViewSlot& sl = slots[v];
  const uint32_t nvis = uint32_t(totals[2 * v]);
  const uint32_t r0 = front_cut(nvis, sl.front16);
  const uint32_t kfirst = uint32_t(i0 - uint64_t(v) * n_pad);
  if (kfirst >= nvis || kfirst + kThreads <= r0) {
    // no Gaussian of this workgroup is cut: whole counts (0 past the visible ones)
    const uint32_t c = k < nvis ? whole[size_t(v) * n + order[i]] : 0u;
    counts[i] = c;
    add_sum(c);
    return;
  }
  if (sl.front16) load_keep(s_keep, bits, sl);  // (only renders with a cut have a bitmap)
  const uint32_t words = keep_words(sl.v.tiles_x);
  __syncthreads();
  uint32_t c = 0;
  SpanGeom sg = {};
  sg.W = sl.v.W;
  sg.H = sl.v.H;
  sg.sh = __builtin_ctz(unsigned(sl.v.tile_size));
  int y0 = 0, y1 = 0;
  if (k < nvis) {
    const uint32_t gi = order[i];
    if (k < r0) {
      c = whole[size_t(v) * n + gi];
    } else {
      const Rect16 r = rects[size_t(v) * n + gi];
      srect[i] = r;
      // rows walked only where the box holds a kept tile
      if (any_kept_in_box(s_keep, words, r.x0, r.y0, r.x1, r.y1)) {
        sg = geom_of(recs[size_t(v) * n + gi], r, sl.v);
        y0 = r.y0;
        y1 = r.y1;
      }
    }
  }
  s_cnt[threadIdx.x] = c;
  __syncthreads();
  const int wave0 = threadIdx.x & ~63;
  wave_rows(sg, y0, y1, lane, [&](bool ok, int o, int y, int x0, int x1) {
    if (ok && x0 < x1) atomicAdd(&s_cnt[wave0 + o], kept_in_run(s_keep + size_t(y) * words, x0, x1));
  });
  __syncthreads();
  counts[i] = s_cnt[threadIdx.x];
  add_sum(s_cnt[threadIdx.x]);
}

// Entries of the Gaussians from each render's depth cut on (front lists,
// front.hpp): their kept tiles only, at their places in the emitted list
// (offsets; counts from front_counts), row by row and in column order.  The
// rows of a wavefront's Gaussians are walked together (rowwalk.hpp); each row
// finds its place from a wavefront scan of the rows' entry counts within its
// Gaussian's run of rows, plus what the Gaussian's earlier rows took (s_pos).
// Runs before emit_block_kernel, which reads the digits back for its counts.
template <typename T, bool PACKED>
__global__ __launch_bounds__(kThreads) void emit_cut_kernel(
    const uint32_t* __restrict__ order, const uint64_t* __restrict__ offsets,
    const uint32_t* __restrict__ counts, const Rect16* __restrict__ rects,
    const Rec<T>* __restrict__ recs, const ViewSlot* __restrict__ slots,
    const SegTable* __restrict__ seg, const unsigned long long* __restrict__ totals,
    const uint64_t* __restrict__ keep, uint32_t n, uint32_t n_pad, uint64_t total,
    uint32_t* __restrict__ out_a, void* __restrict__ out_b) {
  using BType = typename std::conditional<PACKED, uint8_t, uint32_t>::type;
  __shared__ uint64_t s_keep[kKeepWordsMax];
  __shared__ uint32_t s_pos[kThreads];
  const uint64_t i0 = uint64_t(blockIdx.x) * kThreads;
  if (i0 >= total || seg->overflow) return;
  const uint32_t v = uint32_t(i0 / n_pad);
  if (v >= seg->count) return;
  const ViewSlot& sl = slots[v];
  const uint32_t nvis = uint32_t(totals[2 * v]);
  const uint32_t r0 = front_cut(nvis, sl.front16);
  const uint32_t kfirst = uint32_t(i0 - uint64_t(v) * n_pad);
  if (!sl.front16 || kfirst >= nvis || kfirst + kThreads <= r0) return;
  load_keep(s_keep, keep, sl);
  const uint32_t words = keep_words(sl.v.tiles_x);
  const int lane = threadIdx.x & 63, wave0 = threadIdx.x & ~63;
  const uint64_t i = i0 + threadIdx.x;
  const uint32_t k = kfirst + threadIdx.x;
  const size_t row = size_t(v) * n_pad;
  SpanGeom sg = {};
  sg.W = sl.v.W;
  sg.H = sl.v.H;
  sg.sh = __builtin_ctz(unsigned(sl.v.tile_size));
  int y0 = 0, y1 = 0;
  uint32_t gi = 0;
  if (k >= r0 && k < nvis && counts[i] != 0u) {
    gi = order[i];
    const Rect16 r = rects[size_t(v) * n + gi];
    sg = geom_of(recs[size_t(v) * n + gi], r, sl.v);
    y0 = r.y0;
    y1 = r.y1;
    s_pos[threadIdx.x] = seg->start[v] + uint32_t(offsets[i] - offsets[row]);
  }
  __syncthreads();
  const uint32_t tx = uint32_t(sl.v.tiles_x);
  wave_rows(sg, y0, y1, lane, [&](bool ok, int o, int y, int x0, int x1) {
    const uint64_t* __restrict__ krow = s_keep + size_t(ok ? y : 0) * words;
    const uint32_t c = (ok && x0 < x1) ? kept_in_run(krow, x0, x1) : 0u;
    const uint32_t incl = wave_incl_scan(c, lane), excl = incl - c;
    // the lanes of one Gaussian's rows are consecutive: where its run starts
    const int prev_o = __shfl_up(o, 1, 64);
    const int next_o = __shfl_down(o, 1, 64);
    const bool next_ok = __shfl_down(ok ? 1 : 0, 1, 64) != 0;
    const unsigned long long starts = __ballot(ok && (lane == 0 || prev_o != o));
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int first_lane = 63 - __builtin_clzll(starts & upto | 1ull);
    const uint32_t base_excl = __shfl(excl, first_lane, 64);
    const uint32_t gg = __shfl(gi, o, 64);
    if (ok && c) {
      uint32_t pos = s_pos[wave0 + o] + (excl - base_excl);
      for (int w = x0 >> 6; w <= (x1 - 1) >> 6; ++w) {
        uint64_t m = krow[w];
        const int wl = w << 6;
        if (x0 > wl) m &= ~0ull << (x0 - wl);
        if (x1 - wl < 64) m &= (1ull << (x1 - wl)) - 1ull;
        for (; m; m &= m - 1ull, ++pos) {
          const uint32_t tile = uint32_t(y) * tx + uint32_t(wl + __builtin_ctzll(m));
          if (PACKED) {
            out_a[pos] = gg | ((tile >> 8) << 24);
            static_cast<BType*>(out_b)[pos] = BType(tile & 255u);
          } else {
            out_a[pos] = tile;
            static_cast<BType*>(out_b)[pos] = BType(gg);
          }
        }
      }
    }
    // the last lane of a Gaussian's run carries the run's entries forward
    if (ok && (lane == 63 || next_o != o || !next_ok)) s_pos[wave0 + o] += incl - base_excl;
  });
}

// Emission of the tile entries, one block of 4096 entries (in emission order:
// Gaussians in depth order, each one's tiles row by row) per workgroup, so the
// work is balanced whatever the footprints.  The block's Gaussians are taken
// 256 at a time, one per thread; their tile rows are walked together, one row
// per thread (the holder of a row found by a binary search over the
// Gaussians' first row numbers), each row's run placed by a block scan of the
// run lengths, and its entries inside the block written to LDS; the block is
// then written out coalesced.  PACKED: out_a = Gaussian index | high tile
// byte << 24, out_b = low tile byte (bytes); otherwise out_a = tile id, out_b
// = Gaussian index (words).  With a depth cut (front lists, front.hpp) the
// entries of the Gaussians from the cut on, which emit_cut_kernel has already
// written, are only read back for the digit counts.
template <typename T, bool PACKED>
__global__ __launch_bounds__(kThreads) void emit_block_kernel(
    const uint32_t* __restrict__ order, const uint64_t* __restrict__ offsets,
    const Rect16* __restrict__ rects, const Rec<T>* __restrict__ recs,
    const ViewSlot* __restrict__ slots, const SegTable* __restrict__ seg,
    const unsigned long long* __restrict__ totals, const uint64_t* __restrict__ keep,
    const uint32_t* __restrict__ first, uint32_t n, uint32_t n_pad, uint32_t* __restrict__ out_a,
    void* __restrict__ out_b, uint32_t* __restrict__ lo_counts) {
  // (packed: the low tile bytes as bytes, so that more workgroups fit a CU)
  using BType = typename std::conditional<PACKED, uint8_t, uint32_t>::type;
  __shared__ uint32_t s_a[kChunk];
  __shared__ BType s_b[kChunk];
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_first[kThreads];
  __shared__ float s_geo[6][kThreads];
  __shared__ int s_x0[kThreads], s_x1[kThreads], s_y0[kThreads];
  __shared__ uint32_t s_gi[kThreads];
  __shared__ uint32_t s_w[kThreads / 64];
  __shared__ uint32_t s_ga;
  const int tid = threadIdx.x;
  const uint32_t b = blockIdx.x;
  // packed: the block's low-tile-byte counts, the tile sort's first histogram
  const bool count = PACKED && lo_counts;
  if (count) s_hist[tid] = 0u;
  uint32_t s, sstart, nvalid;
  if (seg->overflow || !block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid) {
    if (count) lo_counts[size_t(b) * 256 + tid] = 0u;
    return;
  }
  const uint32_t lo = b * uint32_t(kChunk) - sstart, hi = lo + nvalid;  // render-local entries
  const size_t row = size_t(s) * n_pad;
  const uint64_t o0 = offsets[row];
  const ViewDev vd = slots[s].v;
  const uint32_t tx = uint32_t(vd.tiles_x);
  // depth positions [0, r0) emitted here, their entries [0, f0) of the render
  // (r0 = n: no cut, every entry)
  const uint32_t r0 =
      (keep && slots[s].front16) ? front_cut(uint32_t(totals[2 * s]), slots[s].front16) : n;
  const uint32_t f0 = r0 < n ? uint32_t(offsets[row + r0] - o0) : 0xffffffffu;
  const uint32_t nf = lo >= f0 ? 0u : (hi <= f0 ? nvalid : f0 - lo);  // block entries emitted here
  for (uint32_t q = tid; q < nf; q += kThreads) {  // (every slot is written below)
    s_a[q] = 0u;
    s_b[q] = 0u;
  }
  for (uint32_t kb = first[b]; nf > 0u; kb += kThreads) {
    const uint32_t k = kb + uint32_t(tid);
    uint32_t a = hi, rows = 0;
    if (k < n) a = uint32_t(offsets[row + k] - o0);
    const bool has = k < r0 && a < hi;
    if (has) {
      const uint32_t gi = order[row + k];
      const Rect16 r = rects[size_t(s) * n + gi];
      const SpanGeom g = geom_of(recs[size_t(s) * n + gi], r, vd);
      rows = uint32_t(r.y1 - r.y0);
      s_geo[0][tid] = g.mx;
      s_geo[1][tid] = g.my;
      s_geo[2][tid] = g.beta;
      s_geo[3][tid] = g.gamma;
      s_geo[4][tid] = g.hy;
      s_geo[5][tid] = g.ds;
      s_x0[tid] = g.x0;
      s_x1[tid] = g.x1;
      s_y0[tid] = r.y0;
      s_gi[tid] = gi;
    }
    if (tid == 0) s_ga = a;  // the group's entries start at its first Gaussian's
    uint32_t total_rows;
    s_first[tid] = block_excl_scan<kThreads>(rows, s_w, &total_rows);
    __syncthreads();
    const uint32_t ga = s_ga;
    uint32_t carry = 0;  // entries of the rows before the current 256
    for (uint32_t c = 0; c < total_rows; c += kThreads) {
      const uint32_t p = c + uint32_t(tid);
      const bool ok = p < total_rows;
      // holder: the last thread whose first row number is <= p
      int o = 0;
#pragma unroll
      for (int step = kThreads / 2; step >= 1; step >>= 1)
        if (s_first[o + step] <= p) o += step;
      int x0 = 0, x1 = 0, y = 0;
      if (ok) {
        SpanGeom g;
        g.mx = s_geo[0][o];
        g.my = s_geo[1][o];
        g.beta = s_geo[2][o];
        g.gamma = s_geo[3][o];
        g.hy = s_geo[4][o];
        g.ds = s_geo[5][o];
        g.x0 = s_x0[o];
        g.x1 = s_x1[o];
        g.W = vd.W;
        g.H = vd.H;
        g.sh = __builtin_ctz(unsigned(vd.tile_size));
        y = s_y0[o] + int(p - s_first[o]);
        row_span(g, y, x0, x1);
      }
      const uint32_t len = uint32_t(x1 - x0);
      uint32_t tot;
      const uint32_t e0 = ga + carry + block_excl_scan<kThreads>(len, s_w, &tot);
      const uint32_t j0 = e0 > lo ? e0 : lo, j1 = e0 + len < hi ? e0 + len : hi;
      if (j0 < j1) {
        const uint32_t gi = s_gi[o];
        const uint32_t t0 = uint32_t(y) * tx + uint32_t(x0) - e0;  // tile of entry j: t0 + j
        for (uint32_t j = j0; j < j1; ++j) {
          const uint32_t tile = t0 + j;
          if (PACKED) {
            s_a[j - lo] = gi | ((tile >> 8) << 24);
            s_b[j - lo] = BType(tile & 255u);
          } else {
            s_a[j - lo] = tile;
            s_b[j - lo] = gi;
          }
        }
      }
      carry += tot;
    }
    // more Gaussians start inside the block only if the group's last one did
    const bool more = __syncthreads_or(tid == kThreads - 1 && has);
    if (!more) break;
  }
  __syncthreads();
  const uint32_t e0 = b * uint32_t(kChunk);
  for (uint32_t q = tid; q < nvalid; q += kThreads) {
    BType d;
    if (q < nf) {
      d = s_b[q];
      out_a[e0 + q] = s_a[q];
      static_cast<BType*>(out_b)[e0 + q] = d;
    } else {
      d = static_cast<const BType*>(out_b)[e0 + q];
    }
    if (count) atomicAdd(&s_hist[uint32_t(d) & 255u], 1u);
  }
  if (count) {
    __syncthreads();
    lo_counts[size_t(b) * 256 + tid] = s_hist[tid];
  }
}

// Tile ranges from the sorted tile ids of every segment: position p starts the
// range of its tile when p is the segment's first position or the previous
// tile differs, and ends it likewise (ranges zeroed beforehand, so tiles
// without entries keep [0, 0)).  Each thread reads 16 bytes of consecutive ids.
template <typename K>
__global__ __launch_bounds__(kThreads) void ranges_kernel(const K* __restrict__ tiles,
                                                          const SegTable* __restrict__ seg,
                                                          const ViewSlot* __restrict__ slots,
                                                          uint2* __restrict__ ranges) {
  constexpr int E = 16 / sizeof(K);
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid;
  if (seg->overflow || !block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid)
    return;
  const uint32_t send = sstart + seg->len[s];
  const uint32_t tb = slots[s].tile_base;
  const uint32_t e0 = b * uint32_t(kChunk);
  for (uint32_t q0 = threadIdx.x * E; q0 < nvalid; q0 += kThreads * E) {
    const uint32_t p0 = e0 + q0;  // a multiple of E: one aligned 16-byte load
    K t[E];
    *reinterpret_cast<uint4*>(t) = *reinterpret_cast<const uint4*>(tiles + p0);
    uint32_t prev = p0 > sstart ? uint32_t(tiles[p0 - 1]) : 0xffffffffu;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t p = p0 + uint32_t(i);
      if (p >= send) break;
      const uint32_t ti = uint32_t(t[i]);
      if (ti != prev) {
        ranges[tb + ti].x = p;
        if (p > sstart) ranges[tb + prev].y = p;
      }
      prev = ti;
    }
    const uint32_t pe = p0 + uint32_t(E) - 1u;  // the last position read
    if (pe + 1u >= send) {
      if (p0 < send) ranges[tb + prev].y = send;  // the segment's last tile
    } else if (uint32_t(tiles[pe + 1u]) != prev) {
      ranges[tb + prev].y = pe + 1u;
    }
  }
}

// Digit histograms hist[p][s][256] of the emitted tile ids for the onesweep
// tile sort (zeroed beforehand).
template <int PASSES>
__global__ __launch_bounds__(kThreads) void tile_hist_kernel(const uint32_t* __restrict__ keys,
                                                             const SegTable* __restrict__ seg,
                                                             uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[PASSES][256];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) h[p][threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t b = blockIdx.x;
  uint32_t s = 0, sstart, nvalid = 0;
  if (!seg->overflow && block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid)) {
    const uint32_t e0 = b * uint32_t(kChunk);
    for (uint32_t q = threadIdx.x; q < nvalid; q += kThreads) {
      const uint32_t key = keys[e0 + q];
#pragma unroll
      for (int p = 0; p < PASSES; ++p) atomicAdd(&h[p][(key >> (8 * p)) & 255u], 1u);
    }
  }
  __syncthreads();
  if (nvalid) {
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const uint32_t c = h[p][threadIdx.x];
      if (c) atomicAdd(&hist[(size_t(p) * kMaxViews + s) * 256 + threadIdx.x], c);
    }
  }
}

// Digit counts per block of entries whose digits are one byte each (the
// digits buffer 16-byte aligned): each thread counts 16 consecutive digits,
// read with one 16-byte load where all 16 lie in the block.
static_assert(kChunk == kThreads * 16, "one 16-byte digit word per thread and block");
__global__ __launch_bounds__(kThreads) void lo_count_kernel(const uint8_t* __restrict__ digits,
                                                            const SegTable* __restrict__ seg,
                                                            uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_h[kThreads / 64][256];
  const int tid = threadIdx.x, wave = tid >> 6;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s_h[w][tid] = 0u;
  __syncthreads();
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid = 0;
  if (!seg->overflow && block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid)) {
    const uint32_t e0 = b * uint32_t(kChunk), q0 = uint32_t(tid) * 16u;
    if (q0 + 16u <= nvalid) {
      const uint4 w4 = *reinterpret_cast<const uint4*>(digits + e0 + q0);
      const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
      for (int j = 0; j < 16; ++j) atomicAdd(&s_h[wave][(w[j >> 2] >> (8 * (j & 3))) & 255u], 1u);
    } else {
      for (uint32_t q = q0; q < nvalid; ++q) atomicAdd(&s_h[wave][digits[e0 + q]], 1u);
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) c += s_h[w][tid];
  cnt[size_t(b) * 256 + tid] = c;
}

// Exclusive prefix of M[rows][256] along rows, per column: sum_{r' < r} M[r'][d]
// for r <= rows, in two launches: per-stripe prefixes P and stripe totals T,
// then a scan of the stripe totals (one workgroup per column, which also
// writes the column totals to P[rows]).  The prefix of row r < rows is then
// P[r][d] + T[r / kStripe][d] (col_prefix), added where it is read.
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

__device__ __forceinline__ uint32_t col_prefix(const uint32_t* __restrict__ P,
                                               const uint32_t* __restrict__ T, uint32_t rows,
                                               uint32_t r, uint32_t d) {
  return r >= rows ? P[size_t(rows) * 256 + d]
                   : P[size_t(r) * 256 + d] + T[size_t(r / kStripe) * 256 + d];
}

// Per-digit output base of block b of the segment [first, end) of blocks:
// segment start + counts of lower digits in the segment + counts of digit d
// in the segment's earlier blocks.
__device__ __forceinline__ uint32_t digit_out_base(const uint32_t* __restrict__ P,
                                                   const uint32_t* __restrict__ T, uint32_t rows,
                                                   uint32_t first, uint32_t end, uint32_t b,
                                                   uint32_t seg_start, uint32_t* s_w) {
  const uint32_t d = threadIdx.x;
  const uint32_t pf = col_prefix(P, T, rows, first, d);
  const uint32_t tot_d = col_prefix(P, T, rows, end, d) - pf;
  uint32_t tot;
  const uint32_t lower = block_excl_scan<kThreads>(tot_d, s_w, &tot);
  return seg_start + lower + (col_prefix(P, T, rows, b, d) - pf);
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

// Low-digit pass: stable scatter of each block's packed entries by the low
// tile byte, in runs of equal digit, to their place in the segment; the
// written word carries the low byte in place of the high one, which goes to
// hi_out.
__global__ __launch_bounds__(kThreads) void lo_pass_kernel(const uint32_t* __restrict__ in,
                                                           const uint8_t* __restrict__ digits,
                                                           const SegTable* __restrict__ seg,
                                                           const uint32_t* __restrict__ P,
                                                           const uint32_t* __restrict__ T,
                                                           uint32_t* __restrict__ out,
                                                           uint8_t* __restrict__ hi_out) {
  constexpr int ITEMS = kChunk / kThreads;
  __shared__ uint32_t s_sorted[kChunk];
  __shared__ uint8_t s_dsorted[kChunk];
  __shared__ uint32_t s_base[256], s_start[256];
  __shared__ uint32_t s_wh[kThreads / 64][256];
  __shared__ uint32_t s_w[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid;
  if (seg->overflow || !block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid)
    return;
  const uint32_t send = sstart + seg->len[s];
  const uint32_t e0 = b * uint32_t(kChunk);
  uint32_t x[ITEMS], dg[ITEMS], pos[ITEMS];
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    x[i] = q < nvalid ? in[e0 + q] : 0u;
    dg[i] = q < nvalid ? uint32_t(digits[e0 + q]) : 0u;
  }
  s_base[tid] = digit_out_base(P, T, gridDim.x, sstart / uint32_t(kChunk),
                               (send + uint32_t(kChunk) - 1) / uint32_t(kChunk), b, sstart, s_w);
  rank_block<ITEMS>(dg, nvalid, 8, s_wh, s_start, s_w, pos);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    if (q < nvalid) {
      s_sorted[pos[i]] = x[i];
      s_dsorted[pos[i]] = uint8_t(dg[i]);
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < nvalid; p += kThreads) {
    const uint32_t d = s_dsorted[p];
    const uint32_t x = s_sorted[p];
    const uint32_t pos = s_base[d] + (p - s_start[d]);
    out[pos] = (x & 0xffffffu) | (d << 24);
    hi_out[pos] = uint8_t(x >> 24);
  }
}

// High-digit pass: stable scatter of each block's entries by the high tile
// byte (nbits significant bits, from hi_in); writes the Gaussian index and the
// 16-bit tile id of every sorted entry.
__global__ __launch_bounds__(kThreads) void hi_pass_kernel(const uint32_t* __restrict__ in,
                                                           const uint8_t* __restrict__ hi_in,
                                                           const SegTable* __restrict__ seg,
                                                           const uint32_t* __restrict__ P,
                                                           const uint32_t* __restrict__ T,
                                                           int nbits,
                                                           uint32_t* __restrict__ values,
                                                           uint16_t* __restrict__ tiles) {
  constexpr int ITEMS = kChunk / kThreads;
  __shared__ uint32_t s_sorted[kChunk];
  __shared__ uint8_t s_dsorted[kChunk];
  __shared__ uint32_t s_base[256], s_start[256];
  __shared__ uint32_t s_wh[kThreads / 64][256];
  __shared__ uint32_t s_w[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t b = blockIdx.x;
  uint32_t s, sstart, nvalid;
  if (seg->overflow || !block_span(seg, b * uint32_t(kChunk), s, sstart, nvalid) || !nvalid)
    return;
  const uint32_t send = sstart + seg->len[s];
  const uint32_t e0 = b * uint32_t(kChunk);
  uint32_t x[ITEMS], dg[ITEMS], pos[ITEMS];
  const uint32_t wbase = uint32_t(wave) * ITEMS * 64u;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    x[i] = q < nvalid ? in[e0 + q] : 0u;
    dg[i] = q < nvalid ? uint32_t(hi_in[e0 + q]) : 0u;
  }
  s_base[tid] = digit_out_base(P, T, gridDim.x, sstart / uint32_t(kChunk),
                               (send + uint32_t(kChunk) - 1) / uint32_t(kChunk), b, sstart, s_w);
  rank_block<ITEMS>(dg, nvalid, nbits, s_wh, s_start, s_w, pos);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t q = wbase + uint32_t(i) * 64u + uint32_t(lane);
    if (q < nvalid) {
      s_sorted[pos[i]] = x[i];
      s_dsorted[pos[i]] = uint8_t(dg[i]);
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < nvalid; p += kThreads) {
    const uint32_t d = s_dsorted[p];
    const uint32_t y = s_sorted[p];
    const uint32_t o = s_base[d] + (p - s_start[d]);
    values[o] = y & 0xffffffu;
    tiles[o] = uint16_t((d << 8) | (y >> 24));
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
hipError_t add_grads(const GradPtrs<T>& out, const T* tmp, size_t n, size_t k3, bool static3d,
                     hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t rm = static3d ? 3 : 4, rl = static3d ? 3 : 4, rr = static3d ? 4 : 8;
  hipLaunchKernelGGL(add_grads_kernel<T>, dim3(grid_for((rm + rl + rr + 1 + k3) * n)),
                     dim3(kThreads), 0, stream, out, tmp, n, k3, rm, rl, rr);
  return hipGetLastError();
}
template hipError_t add_grads<float>(const GradPtrs<float>&, const float*, size_t, size_t, bool,
                                     hipStream_t);
template hipError_t add_grads<double>(const GradPtrs<double>&, const double*, size_t, size_t,
                                      bool, hipStream_t);

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
  const dim3 grid((max_len + kHistChunk - 1) / kHistChunk, uint32_t(n_segments));
  switch (passes) {
    case 1: hipLaunchKernelGGL(radix_hist_kernel<1>, grid, dim3(kThreads), 0, stream, keys, seg, hist); break;
    case 2: hipLaunchKernelGGL(radix_hist_kernel<2>, grid, dim3(kThreads), 0, stream, keys, seg, hist); break;
    case 3: hipLaunchKernelGGL(radix_hist_kernel<3>, grid, dim3(kThreads), 0, stream, keys, seg, hist); break;
    case 4: hipLaunchKernelGGL(radix_hist_kernel<4>, grid, dim3(kThreads), 0, stream, keys, seg, hist); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Workgroups of `kernel` (kThreads each) resident on the whole device at once;
// 0 when unknown (then every launch takes tickets).
template <typename K>
uint32_t resident_blocks(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
      per_cu < 1 || cus < 1) {
    (void)hipGetLastError();
    return 0u;
  }
  return uint32_t(per_cu) * uint32_t(cus);
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
  // launch-order tickets are needed only when the grid does not fit the
  // device at once (a workgroup must never wait on one that cannot start)
  static const uint32_t resident[3] = {resident_blocks(onesweep_kernel<4>),
                                       resident_blocks(onesweep_kernel<8>),
                                       resident_blocks(onesweep_kernel<16>)};
  const int which = items == 4 ? 0 : (items == 8 ? 1 : 2);
  const bool ticketed = blocks > resident[which];
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
                           ko, vo, seg, h, st, ticketed ? tickets + p : nullptr, error, 8 * p);
        break;
      case 8:
        hipLaunchKernelGGL(onesweep_kernel<8>, dim3(blocks), dim3(kThreads), 0, stream, ki, vi,
                           ko, vo, seg, h, st, ticketed ? tickets + p : nullptr, error, 8 * p);
        break;
      case 16:
        hipLaunchKernelGGL(onesweep_kernel<16>, dim3(blocks), dim3(kThreads), 0, stream, ki, vi,
                           ko, vo, seg, h, st, ticketed ? tickets + p : nullptr, error, 8 * p);
        break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t seg_table(const unsigned long long* totals, const ViewSlot* slots, int n_views,
                     unsigned long long capacity, SegTable* seg, uint32_t* overflow_out,
                     hipStream_t stream) {
  hipLaunchKernelGGL(seg_table_kernel, dim3(1), dim3(64), 0, stream, totals, slots, n_views,
                     capacity, seg, overflow_out);
  return hipGetLastError();
}

size_t emit_temp_bytes(uint64_t capacity) {
  return size_t((capacity + kChunk - 1) / kChunk + 64) * 4;
}

template <typename T>
hipError_t emit_blocks(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                       const Rec<T>* recs, const ViewSlot* slots, const SegTable* seg,
                       const unsigned long long* totals, const uint64_t* keep,
                       const uint32_t* counts, uint32_t n,
                       uint32_t n_pad, int n_views, uint64_t capacity, bool packed, void* temp,
                       uint32_t* out_a, void* out_b, void* sort_temp, hipStream_t stream) {
  const uint32_t blocks = uint32_t((capacity + kChunk - 1) / kChunk);
  if (n == 0 || n_views <= 0 || blocks == 0) return hipSuccess;
  const uint32_t* first = static_cast<const uint32_t*>(temp);  // written by the count scan
  if (keep) {
    const uint64_t total = uint64_t(n_pad) * uint64_t(n_views);
    const dim3 grid(uint32_t((total + kThreads - 1) / kThreads));
    if (packed)
      hipLaunchKernelGGL((emit_cut_kernel<T, true>), grid, dim3(kThreads), 0, stream, order,
                         offsets, counts, rects, recs, slots, seg, totals, keep, n, n_pad, total,
                         out_a, out_b);
    else
      hipLaunchKernelGGL((emit_cut_kernel<T, false>), grid, dim3(kThreads), 0, stream, order,
                         offsets, counts, rects, recs, slots, seg, totals, keep, n, n_pad, total,
                         out_a, out_b);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (packed)
    hipLaunchKernelGGL((emit_block_kernel<T, true>), dim3(blocks), dim3(kThreads), 0, stream,
                       order, offsets, rects, recs, slots, seg, totals, keep, first, n, n_pad,
                       out_a, out_b, static_cast<uint32_t*>(sort_temp));
  else
    hipLaunchKernelGGL((emit_block_kernel<T, false>), dim3(blocks), dim3(kThreads), 0, stream,
                       order, offsets, rects, recs, slots, seg, totals, keep, first, n, n_pad,
                       out_a, out_b, (uint32_t*)nullptr);
  return hipGetLastError();
}

template hipError_t emit_blocks<float>(const uint32_t*, const uint64_t*, const Rect16*,
                                       const Rec<float>*, const ViewSlot*, const SegTable*,
                                       const unsigned long long*, const uint64_t*,
                                       const uint32_t*, uint32_t,
                                       uint32_t, int, uint64_t, bool, void*, uint32_t*, void*,
                                       void*, hipStream_t);
template hipError_t emit_blocks<double>(const uint32_t*, const uint64_t*, const Rect16*,
                                        const Rec<double>*, const ViewSlot*, const SegTable*,
                                        const unsigned long long*, const uint64_t*,
                                        const uint32_t*, uint32_t,
                                        uint32_t, int, uint64_t, bool, void*, uint32_t*, void*,
                                        void*, hipStream_t);

hipError_t tile_ranges(const void* sorted_tiles, bool tiles16, const SegTable* seg,
                       const ViewSlot* slots, uint32_t total_tiles, uint64_t capacity,
                       uint2* ranges, hipStream_t stream) {
  const uint32_t blocks = uint32_t((capacity + kChunk - 1) / kChunk);
  if (blocks == 0) return hipSuccess;
  if (tiles16)
    hipLaunchKernelGGL(ranges_kernel<uint16_t>, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const uint16_t*>(sorted_tiles), seg, slots, ranges);
  else
    hipLaunchKernelGGL(ranges_kernel<uint32_t>, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const uint32_t*>(sorted_tiles), seg, slots, ranges);
  return hipGetLastError();
}

hipError_t tile_key_histogram(const uint32_t* keys, const SegTable* seg, uint64_t capacity,
                              int passes, uint32_t* hist, hipStream_t stream) {
  hipError_t e = fill_zero(hist, size_t(passes) * kMaxViews * 256 * 4, stream);
  if (e != hipSuccess) return e;
  const uint32_t blocks = uint32_t((capacity + kChunk - 1) / kChunk);
  if (blocks == 0) return hipSuccess;
  switch (passes) {
    case 1: hipLaunchKernelGGL(tile_hist_kernel<1>, dim3(blocks), dim3(kThreads), 0, stream, keys, seg, hist); break;
    case 2: hipLaunchKernelGGL(tile_hist_kernel<2>, dim3(blocks), dim3(kThreads), 0, stream, keys, seg, hist); break;
    case 3: hipLaunchKernelGGL(tile_hist_kernel<3>, dim3(blocks), dim3(kThreads), 0, stream, keys, seg, hist); break;
    default: return hipErrorInvalidValue;
  }
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

size_t count_tile_sums_bytes(uint32_t n_pad, int n_views) {
  const uint64_t tiles = (uint64_t(n_pad) * uint64_t(n_views) + 1 + kScanTile - 1) / kScanTile;
  return tiles * sizeof(uint64_t);
}

size_t count_scan_seg_temp_bytes(uint32_t n_pad, int n_views) {
  const uint64_t tiles = (uint64_t(n_pad) * uint64_t(n_views) + 1 + kScanTile - 1) / kScanTile;
  return (2 * tiles + scan_temp_elems(tiles) + 2) * sizeof(uint64_t);
}

hipError_t count_scan_seg(const uint32_t* order, const uint32_t* counts,
                          const uint32_t* front_counts, const unsigned long long* totals,
                          const ViewSlot* slots, uint32_t n, uint32_t n_pad, int n_views,
                          uint64_t* offsets, void* temp, unsigned long long capacity,
                          SegTable* seg, FrontTable* front, uint32_t* overflow_out,
                          uint32_t* first, uint64_t* tile_sums, hipStream_t stream) {
  const uint64_t total = uint64_t(n_pad) * uint64_t(n_views);
  const uint64_t n_elems = total + 1;
  const uint64_t tiles = (n_elems + kScanTile - 1) / kScanTile;
  // (front lists: front_counts added up the tile sums and wrote the table)
  const bool summed = front_counts != nullptr;
  uint64_t* sums = summed ? tile_sums : static_cast<uint64_t*>(temp);
  uint64_t* scanned = static_cast<uint64_t*>(temp) + tiles;
  const bool direct = tiles <= kCountDirectTiles;
  auto run = [&](auto ld, FrontTable* ft) -> hipError_t {
    hipError_t e = hipSuccess;
    if (!summed) {
      hipLaunchKernelGGL(count_sums_kernel<decltype(ld)>, dim3(uint32_t(tiles)), dim3(kThreads),
                         0, stream, ld, sums, totals, slots, n_views, capacity, seg, overflow_out);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (!direct) {
      e = device_exclusive_scan<uint64_t, LoadT<uint64_t>>(LoadT<uint64_t>{sums, tiles}, scanned,
                                                           tiles, scanned + tiles, stream);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(count_offsets_kernel<decltype(ld)>, dim3(uint32_t(tiles)), dim3(kThreads),
                       0, stream, ld, n, n_pad, n_elems, sums, direct ? nullptr : scanned, seg, ft,
                       offsets, first);
    return hipGetLastError();
  };
  if (front_counts) return run(LoadCountPlain{front_counts, total}, front);
  return run(LoadCountGatherSeg{order, counts, totals, n, n_pad, total}, nullptr);
}

hipError_t front_keep(const ViewSlot* slots, int n_views, const Rect16* rects,
                      const uint32_t* order, const unsigned long long* totals, uint32_t n,
                      uint32_t n_pad, int32_t keep, int32_t* cover, uint64_t* bits,
                      hipStream_t stream) {
  if (n_views <= 0) return hipSuccess;
  hipLaunchKernelGGL(front_keep_kernel, dim3(uint32_t(kKeepGroups), uint32_t(n_views)),
                     dim3(kKeepThreads), 0, stream, slots, rects, order, totals, n, n_pad, cover);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(front_bits_kernel, dim3(uint32_t(n_views)), dim3(kKeepThreads), 0, stream,
                     slots, cover, keep, bits);
  return hipGetLastError();
}

bool front_grid_ok(int tiles_x, int tiles_y) {
  return int64_t(tiles_x + 1) * int64_t(tiles_y + 1) <= int64_t(kKeepGrid) &&
         int64_t(keep_words(tiles_x)) * int64_t(tiles_y) <= int64_t(kKeepWordsMax);
}

template <typename T>
hipError_t front_counts(const uint32_t* order, const uint32_t* whole, const Rect16* rects,
                        const Rec<T>* recs, const ViewSlot* slots,
                        const unsigned long long* totals, const uint64_t* bits, uint32_t n,
                        uint32_t n_pad, int n_views, uint32_t* counts, Rect16* srect,
                        uint64_t* tile_sums, unsigned long long capacity, SegTable* seg,
                        uint32_t* overflow_out, hipStream_t stream) {
  const uint64_t total = uint64_t(n_pad) * uint64_t(n_views);
  if (total == 0) return hipSuccess;
  static_assert(kScanTile % kThreads == 0, "a scan tile holds whole workgroups");
  hipLaunchKernelGGL(front_counts_kernel<T>, dim3(uint32_t((total + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, stream, order, whole, rects, recs, slots, totals, bits, n,
                     n_pad, total, counts, srect, tile_sums, n_views, capacity, seg,
                     overflow_out);
  return hipGetLastError();
}

template hipError_t front_counts<float>(const uint32_t*, const uint32_t*, const Rect16*,
                                        const Rec<float>*, const ViewSlot*,
                                        const unsigned long long*, const uint64_t*, uint32_t,
                                        uint32_t, int, uint32_t*, Rect16*, uint64_t*,
                                        unsigned long long, SegTable*, uint32_t*, hipStream_t);
template hipError_t front_counts<double>(const uint32_t*, const uint32_t*, const Rect16*,
                                         const Rec<double>*, const ViewSlot*,
                                         const unsigned long long*, const uint64_t*, uint32_t,
                                         uint32_t, int, uint32_t*, Rect16*, uint64_t*,
                                         unsigned long long, SegTable*, uint32_t*, hipStream_t);

bool packed_tile_sort_ok(uint32_t n, uint32_t max_tiles_per_view) {
  return n <= (1u << 24) && max_tiles_per_view <= 65536u;
}

size_t packed_sort_temp_bytes(uint64_t capacity) {
  const uint64_t rows = (capacity + kChunk - 1) / kChunk;
  const uint64_t stripes = (rows + kStripe - 1) / kStripe + 1;
  // per pass: block digit counts M, their column prefix P, stripe totals
  return size_t(2 * (rows * 256 + (rows + 1) * 256 + stripes * 256) * 4);
}

namespace {
hipError_t col_scan(const uint32_t* M, uint32_t rows, uint32_t* P, uint32_t* T,
                    hipStream_t stream) {
  const uint32_t stripes = (rows + kStripe - 1) / kStripe;
  if (stripes > 0)
    hipLaunchKernelGGL(col_scan_stripes_kernel, dim3(stripes), dim3(256), 0, stream, M, rows, P,
                       T);
  hipLaunchKernelGGL(col_scan_totals_kernel, dim3(256), dim3(256), 0, stream, T, stripes, P, rows);
  return hipGetLastError();
}
}  // namespace

hipError_t packed_tile_sort(const uint32_t* packed, const uint8_t* digits, const SegTable* seg,
                            uint32_t max_tiles, uint64_t capacity, void* temp, uint32_t* mid,
                            uint8_t* mid_hi, uint32_t* values, uint16_t* tiles,
                            hipStream_t stream) {
  const uint32_t rows = uint32_t((capacity + kChunk - 1) / kChunk);
  if (rows == 0) return hipSuccess;
  const uint32_t stripes = (rows + kStripe - 1) / kStripe + 1;
  uint32_t* M1 = static_cast<uint32_t*>(temp);
  uint32_t* P1 = M1 + size_t(rows) * 256;
  uint32_t* T1 = P1 + size_t(rows + 1) * 256;
  uint32_t* M2 = T1 + size_t(stripes) * 256;
  uint32_t* P2 = M2 + size_t(rows) * 256;
  uint32_t* T2 = P2 + size_t(rows + 1) * 256;
  // (the emission wrote M1, the low-byte counts of its blocks)
  hipError_t e = col_scan(M1, rows, P1, T1, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lo_pass_kernel, dim3(rows), dim3(kThreads), 0, stream, packed, digits, seg,
                     P1, T1, mid, mid_hi);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(lo_count_kernel, dim3(rows), dim3(kThreads), 0, stream, mid_hi, seg, M2);
  if ((e = col_scan(M2, rows, P2, T2, stream)) != hipSuccess) return e;
  int nbits = 1;
  while ((1u << nbits) < (max_tiles + 255u) / 256u) ++nbits;
  hipLaunchKernelGGL(hi_pass_kernel, dim3(rows), dim3(kThreads), 0, stream, mid, mid_hi, seg, P2,
                     T2, nbits, values, tiles);
  return hipGetLastError();
}

}  // namespace r4d
