// Device-wide scans, stable LSD radix sort of (u32 key, u32 value) pairs, tile-key
// emission and tile ranges.
//
// The (tile, depth) order the rasteriser needs is produced in two stable
// stages: the Gaussians are first sorted by the float32 bit pattern of their
// depth (positive floats order like their bit patterns; culled Gaussians carry
// 0xffffffff and sort last), each Gaussian's tiles are then emitted in that
// depth order, and the emitted list is stably sorted by tile id.  The result is
// ordered by (tile, depth, Gaussian index) -- a radix sort of that composite key
// whose low 32 bits are sorted once per Gaussian instead of once per tile entry.
//
// Radix sort: 8-bit digits, one pass per digit, each pass = per-block digit
// histogram, exclusive scan of the [digit][block] table, and a scatter in which
// every block ranks its 4096 keys stably in LDS (wave64 ballots find the lanes
// holding the same digit) and writes each digit run with consecutive lanes on
// consecutive addresses.
#include <hip/hip_runtime.h>

#include "r4d_internal.hpp"

namespace r4d {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadix = 256;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive block scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* s_wave, T* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(x, lane);
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  T wave_off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const T s = s_wave[w];
    wave_off += w < wave ? s : T(0);
    tot += s;
  }
  *total = tot;
  return wave_off + inc - x;
}

struct LoadU32 {
  const uint32_t* p;
  uint64_t n;
  __device__ uint32_t operator()(uint64_t i) const { return i < n ? p[i] : 0u; }
};

template <typename T>
struct LoadT {
  const T* p;
  uint64_t n;
  __device__ T operator()(uint64_t i) const { return i < n ? p[i] : T(0); }
};

struct LoadCountGather {
  const uint32_t* order;
  const uint32_t* counts;
  uint64_t n;
  __device__ uint64_t operator()(uint64_t i) const {
    return i < n ? uint64_t(counts[order[i]]) : uint64_t(0);
  }
};

template <typename T, typename Loader>
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(Loader ld, T* out, T* tile_sums,
                                                                  uint64_t n) {
  __shared__ T s_wave[kScanThreads / 64];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = ld(base + j);
    sum += v[j];
  }
  T total;
  T run = block_exclusive_scan(sum, s_wave, &total);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(T* out, const T* tile_offsets,
                                                                uint64_t n) {
  const T add = tile_offsets[blockIdx.x];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint64_t i = base + uint64_t(j) * kScanThreads + threadIdx.x;
    if (i < n) out[i] += add;
  }
}

template <typename T>
size_t scan_temp_elems(uint64_t n) {
  size_t total = 0;
  uint64_t m = n;
  while (m > uint64_t(kScanTile)) {
    m = (m + kScanTile - 1) / kScanTile;
    total += m;
  }
  return total;
}

// Exclusive scan of ld(0..n-1) into out[0..n-1]; temp holds scan_temp_elems<T>(n).
template <typename T, typename Loader>
hipError_t device_exclusive_scan(Loader ld, T* out, uint64_t n, T* temp, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    hipLaunchKernelGGL((scan_tiles_kernel<T, Loader>), dim3(1), dim3(kScanThreads), 0, stream, ld,
                       out, (T*)nullptr, n);
    return hipGetLastError();
  }
  T* sums = temp;
  hipLaunchKernelGGL((scan_tiles_kernel<T, Loader>), dim3(tiles), dim3(kScanThreads), 0, stream,
                     ld, out, sums, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_exclusive_scan<T, LoadT<T>>(LoadT<T>{sums, tiles}, sums, tiles, temp + tiles, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_add_kernel<T>, dim3(tiles), dim3(kScanThreads), 0, stream, out,
                     (const T*)sums, n);
  return hipGetLastError();
}

// ---- radix sort

__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                                     uint32_t n, int shift,
                                                                     uint32_t* __restrict__ hist,
                                                                     uint32_t nblocks) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kSortTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = base + i * kSortThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ hist_scan, uint32_t n, int shift, uint32_t nblocks) {
  __shared__ uint32_t s_keys[kSortTile];
  __shared__ uint32_t s_vals[kSortTile];
  __shared__ uint32_t s_cnt[kSortThreads / 64][kRadix];
  __shared__ uint32_t s_run[kRadix];
  __shared__ uint32_t s_start[kRadix];
  __shared__ uint32_t s_gofs[kRadix];
  __shared__ uint32_t s_wave[kSortThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t base = blockIdx.x * kSortTile;
  s_run[tid] = 0;
  s_gofs[tid] = hist_scan[tid * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kSortThreads / 64; ++w) s_cnt[w][tid] = 0;
  uint32_t k[kSortItems], v[kSortItems], rank[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const uint32_t idx = base + i * kSortThreads + tid;
    const bool valid = idx < n;
    k[i] = valid ? keys_in[idx] : 0u;
    v[i] = valid ? vals_in[idx] : 0u;
  }
  __syncthreads();
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const bool valid = base + i * kSortThreads + tid < n;
    const uint32_t d = (k[i] >> shift) & (kRadix - 1);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const unsigned long long before = peers & lt_mask;
    const uint32_t r_w = __popcll(before);
    const uint32_t c_w = __popcll(peers);
    const bool leader = valid && before == 0ull;
    const uint32_t tag = uint32_t(i + 1) << 16;
    if (leader) s_cnt[wave][d] = tag | c_w;
    __syncthreads();
    if (valid) {
      uint32_t prefix = 0;
      for (int w = 0; w < wave; ++w) {
        const uint32_t val = s_cnt[w][d];
        prefix += (val & 0xffff0000u) == tag ? (val & 0xffffu) : 0u;
      }
      rank[i] = s_run[d] + prefix + r_w;
    }
    __syncthreads();
    if (leader) atomicAdd(&s_run[d], c_w);
  }
  __syncthreads();
  // exclusive scan of the block's digit counts
  {
    const uint32_t x = s_run[tid];
    const uint32_t inc = wave_inclusive_scan(x, lane);
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += s_wave[w];
    s_start[tid] = off + inc - x;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const bool valid = base + i * kSortThreads + tid < n;
    if (valid) {
      const uint32_t d = (k[i] >> shift) & (kRadix - 1);
      const uint32_t pos = s_start[d] + rank[i];
      s_keys[pos] = k[i];
      s_vals[pos] = v[i];
    }
  }
  __syncthreads();
  const uint32_t cnt = n - base < uint32_t(kSortTile) ? n - base : uint32_t(kSortTile);
  for (uint32_t p = tid; p < cnt; p += kSortThreads) {
    const uint32_t key = s_keys[p];
    const uint32_t d = (key >> shift) & (kRadix - 1);
    const uint32_t gpos = s_gofs[d] + (p - s_start[d]);
    keys_out[gpos] = key;
    vals_out[gpos] = s_vals[p];
  }
}

// ---- tile-key emission: each wavefront takes 64 consecutive Gaussians of the
// depth order and writes their tile entries one Gaussian at a time, lanes on
// consecutive entries, so the stores are coalesced whatever the rectangle size.
__global__ __launch_bounds__(256) void emit_kernel(const uint32_t* __restrict__ order,
                                                   const uint64_t* __restrict__ offsets,
                                                   const Rect16* __restrict__ rects, uint32_t n,
                                                   int tiles_x, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const uint32_t k = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t idx = 0, cnt = 0, off = 0;
  Rect16 rc = {0, 0, 0, 0};
  if (k < n) {
    idx = order[k];
    rc = rects[idx];
    cnt = uint32_t(rc.x1 - rc.x0) * uint32_t(rc.y1 - rc.y0);
    off = uint32_t(offsets[k]);
  }
  unsigned long long todo = __ballot(cnt > 0);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1ull;
    const uint32_t s_idx = __shfl(idx, src, 64);
    const uint32_t s_cnt = __shfl(cnt, src, 64);
    const uint32_t s_off = __shfl(off, src, 64);
    const uint32_t x0 = __shfl(uint32_t(rc.x0), src, 64);
    const uint32_t y0 = __shfl(uint32_t(rc.y0), src, 64);
    const uint32_t w = __shfl(uint32_t(rc.x1 - rc.x0), src, 64);
    for (uint32_t j = lane; j < s_cnt; j += 64) {
      const uint32_t ty = y0 + j / w, tx = x0 + j % w;
      keys[s_off + j] = ty * uint32_t(tiles_x) + tx;
      vals[s_off + j] = s_idx;
    }
  }
}

__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* __restrict__ keys, uint32_t d,
                                                     uint2* __restrict__ ranges) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d) return;
  const uint32_t t = keys[i];
  if (i == 0 || keys[i - 1] != t) ranges[t].x = i;
  if (i == d - 1 || keys[i + 1] != t) ranges[t].y = i + 1;
}

}  // namespace

size_t sort_pairs_temp_bytes(uint32_t n) {
  const uint64_t nblocks = (uint64_t(n) + kSortTile - 1) / kSortTile;
  const uint64_t h = nblocks * kRadix;
  return (h + scan_temp_elems<uint32_t>(h) + 64) * sizeof(uint32_t);
}

hipError_t sort_pairs_u32(uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int end_bit,
                          SortTemp temp, int* result_index, hipStream_t stream) {
  int cur = 0;
  *result_index = 0;
  if (n <= 1) return hipSuccess;
  const uint32_t nblocks = (n + kSortTile - 1) / kSortTile;
  const uint64_t h = uint64_t(nblocks) * kRadix;
  if (temp.bytes < sort_pairs_temp_bytes(n)) return hipErrorInvalidValue;
  uint32_t* hist = static_cast<uint32_t*>(temp.ptr);
  uint32_t* scan_tmp = hist + h;
  for (int shift = 0; shift < end_bit; shift += 8) {
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(nblocks), dim3(kSortThreads), 0, stream,
                       keys[cur], n, shift, hist, nblocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = device_exclusive_scan<uint32_t, LoadU32>(LoadU32{hist, h}, hist, h, scan_tmp, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_downsweep_kernel, dim3(nblocks), dim3(kSortThreads), 0, stream,
                       keys[cur], vals[cur], keys[1 - cur], vals[1 - cur], hist, n, shift,
                       nblocks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = 1 - cur;
  }
  *result_index = cur;
  return hipSuccess;
}

size_t count_scan_temp_bytes(uint32_t n) {
  return (scan_temp_elems<uint64_t>(uint64_t(n) + 1) + 8) * sizeof(uint64_t);
}

hipError_t count_scan(const uint32_t* order, const uint32_t* tiles_touched, uint32_t n,
                      uint64_t* offsets, SortTemp temp, hipStream_t stream) {
  return device_exclusive_scan<uint64_t, LoadCountGather>(
      LoadCountGather{order, tiles_touched, n}, offsets, uint64_t(n) + 1,
      static_cast<uint64_t*>(temp.ptr), stream);
}

hipError_t emit_tile_keys(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                          uint32_t n, int tiles_x, uint32_t* keys, uint32_t* vals,
                          hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(emit_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, order, offsets,
                     rects, n, tiles_x, keys, vals);
  return hipGetLastError();
}

hipError_t tile_ranges(const uint32_t* sorted_keys, uint32_t d, uint32_t n_tiles, uint2* ranges,
                       hipStream_t stream) {
  hipError_t e = hipMemsetAsync(ranges, 0, size_t(n_tiles) * sizeof(uint2), stream);
  if (e != hipSuccess || d == 0) return e;
  hipLaunchKernelGGL(ranges_kernel, dim3((d + 255) / 256), dim3(256), 0, stream, sorted_keys, d,
                     ranges);
  return hipGetLastError();
}

}  // namespace r4d
