// Launchers of the bin views (views.hip): per-bin histograms, line raster,
// brushing mask.
#pragma once

#include "common.hpp"

namespace dvl {

constexpr int kRasterPolyline = 0;   // column b spans the rows of heights b and b + 1
constexpr int kRasterBars = 1;       // column b spans rows 0 .. the row of height b

// counts[b * H + k]: cells first[b]..last[b] of the sorted field whose
// entry under the quantiser (s, b) of H buckets is k
dvl_status launch_bin_histograms(int dtype, const void* field, int32_t W, const uint32_t* first,
                                 const uint32_t* last, int32_t H, float s, float b, uint32_t* counts,
                                 int n_cu, hipStream_t st);
// img[l][r][b] for `lines` lines of W heights each, H rows
dvl_status launch_rasterize(const float* y, int32_t W, int32_t H, int32_t lines, int32_t mode, uint8_t* img,
                            hipStream_t st);
// mask[perm[h]] = keys_sorted[h] inside one of the ranges [ranges[2i], ranges[2i+1]]
// (host array, n_ranges <= kMaxSelectRanges)
constexpr int kMaxSelectRanges = 128;
dvl_status launch_select_mask(int64_t n, const uint64_t* keys_sorted, const uint32_t* perm, int32_t n_ranges,
                              const uint64_t* ranges, uint8_t* mask, hipStream_t st);
// out[i] = i
dvl_status launch_iota(int64_t n, uint32_t* out, hipStream_t st);

}  // namespace dvl
