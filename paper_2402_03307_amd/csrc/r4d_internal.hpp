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

// Tile rectangle of a Gaussian: tile x0, y0, x1, y1 (x1, y1 exclusive).
struct Rect16 {
  uint16_t x0, y0, x1, y1;
};

// ---- preprocess (per Gaussian)
// totals[0] += number of visible Gaussians, totals[1] += number of tile entries
// (the caller zeroes them first).
template <typename T>
hipError_t launch_preprocess_fwd(const GaussPtrs<T>& g, const ViewDev& v, const SettingsDev& st,
                                 Rec<T>* recs, Rect16* rects, uint32_t* tiles_touched,
                                 uint32_t* depth_keys, uint32_t* values_iota,
                                 unsigned long long* totals, hipStream_t stream);

// grad2d: [9][n] double (mean2 x, y, conic a, b, c, opacity_t, r, g, b).
// accumulate=false overwrites `out`, true adds to it.
template <typename T>
hipError_t launch_preprocess_bwd(const GaussPtrs<T>& g, const ViewDev& v, const SettingsDev& st,
                                 const double* grad2d, const GradPtrs<T>& out, bool accumulate,
                                 hipStream_t stream);

// ---- sorting and binning
struct SortTemp {
  void* ptr;
  size_t bytes;
};

// Bytes of temporary storage that sort_pairs_u32 needs for n elements.
size_t sort_pairs_temp_bytes(uint32_t n);
// Stable LSD radix sort of (key, value) pairs on key bits [0, end_bit).
// keys/vals: in/out double buffers; on return *result_index says which of the two
// buffers (0 or 1) holds the sorted data.
hipError_t sort_pairs_u32(uint32_t* keys[2], uint32_t* vals[2], uint32_t n, int end_bit,
                          SortTemp temp, int* result_index, hipStream_t stream);

size_t count_scan_temp_bytes(uint32_t n);
// offsets[k] = sum_{j<k} tiles_touched[order[j]] for k in [0, n]; offsets[n] = total.
hipError_t count_scan(const uint32_t* order, const uint32_t* tiles_touched, uint32_t n,
                      uint64_t* offsets, SortTemp temp, hipStream_t stream);

// Writes, for each Gaussian in `order` (first n entries), its tiles in row-major
// order: keys = tile id, vals = Gaussian index, at offsets[k].
hipError_t emit_tile_keys(const uint32_t* order, const uint64_t* offsets, const Rect16* rects,
                          uint32_t n, int tiles_x, uint32_t* keys, uint32_t* vals,
                          hipStream_t stream);

// ranges[t] = [start, end) of tile t in the sorted keys; tiles without entries [0,0).
hipError_t tile_ranges(const uint32_t* sorted_keys, uint32_t d, uint32_t n_tiles, uint2* ranges,
                       hipStream_t stream);

// ---- rasterisation
// (tile size, pixels per lane) pairs the rasteriser is compiled for.
bool raster_config_supported(int tile_size, int ppt);
int raster_default_ppt(int tile_size, bool backward);

// n_eval (nullable): per pixel, the number of list entries evaluated.
template <typename T>
hipError_t launch_raster_fwd(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                             const ViewDev& v, const SettingsDev& st, int ppt, T* image,
                             T* T_final, uint32_t* n_contrib, uint32_t* n_eval,
                             hipStream_t stream);

// grad2d: [9][n] double accumulators (see launch_preprocess_bwd), added to.
template <typename T>
hipError_t launch_raster_bwd(const Rec<T>* recs, const uint32_t* values, const uint2* ranges,
                             const ViewDev& v, const SettingsDev& st, int ppt, const T* T_final,
                             const uint32_t* n_contrib, const T* dL_dimage, double* grad2d,
                             uint32_t n_gaussians, hipStream_t stream);

hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, float* grad,
                          float* loss, hipStream_t stream);

}  // namespace r4d
