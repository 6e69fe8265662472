// Views of an update's bins beyond the lines themselves:
//
//   k_bin_histograms  per bin, the histogram of one field's values over its
//                     cells (the histogram heatmap of volume-line plots;
//                     paper section Prototypical User Interface)
//   k_rasterize       the lines drawn as polylines or bar charts into an
//                     image (the paper's RasterizeLines kernel, GPU section)
//   k_select_mask     brushing and linking: which cells (original order) have
//                     a Hilbert key inside one of the selected key ranges
//                     (paper section Brushing and Linking: regions of
//                     interest travel to the 3D view as Hilbert-code ranges)
#include "views.hpp"

#include <algorithm>

namespace dvl {

// ------------------------------------------------------------------ histograms

// One workgroup per bin (grid-stride over bins): the bin's sorted cells
// first..last are streamed with coalesced loads and counted into an LDS
// histogram of H buckets; the bucket of a value is its entry under the
// quantiser of [lo, hi] for H entries (the TF entry rule), so the counts are
// exact integers independent of the order of the additions.
template <typename S>
__global__ __launch_bounds__(256) void k_bin_histograms(const typename S::raw* __restrict__ v, int32_t W,
                                                        const uint32_t* __restrict__ first,
                                                        const uint32_t* __restrict__ last, int32_t H,
                                                        float s, float b, uint32_t* __restrict__ counts) {
    extern __shared__ uint32_t hist[];
    const float nmax = (float)(H - 1);
    for (int32_t bin = blockIdx.x; bin < W; bin += gridDim.x) {
        for (int32_t k = threadIdx.x; k < H; k += blockDim.x) hist[k] = 0u;
        __syncthreads();
        const uint32_t f = first[bin], l = last[bin];
        if (f <= l) {
            for (uint64_t h = (uint64_t)f + threadIdx.x; h <= (uint64_t)l; h += blockDim.x) {
                float t = fmaf(to_f32(S{}, v[h]), s, b);
                t = fminf(fmaxf(t, 0.0f), nmax);
                atomicAdd(&hist[(int)t], 1u);
            }
        }
        __syncthreads();
        for (int32_t k = threadIdx.x; k < H; k += blockDim.x) counts[(int64_t)bin * H + k] = hist[k];
        __syncthreads();
    }
}

dvl_status launch_bin_histograms(int dtype, const void* field, int32_t W, const uint32_t* first,
                                 const uint32_t* last, int32_t H, float s, float b, uint32_t* counts,
                                 int n_cu, hipStream_t st) {
    const unsigned grid = (unsigned)std::max(1, std::min(W, n_cu * 16));
    const size_t lds = (size_t)H * sizeof(uint32_t);
    if (dtype == DVL_F16)
        hipLaunchKernelGGL(k_bin_histograms<F16>, dim3(grid), dim3(256), lds, st, (const uint16_t*)field, W,
                           first, last, H, s, b, counts);
    else if (dtype == DVL_BF16)
        hipLaunchKernelGGL(k_bin_histograms<BF16>, dim3(grid), dim3(256), lds, st, (const uint16_t*)field, W,
                           first, last, H, s, b, counts);
    else
        hipLaunchKernelGGL(k_bin_histograms<F32>, dim3(grid), dim3(256), lds, st, (const float*)field, W, first,
                           last, H, s, b, counts);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ raster

// the row of a height y in [0, 1] on H rows (row 0 at the bottom)
__device__ __forceinline__ int raster_row(float y, int H) {
    const float t = y * (float)H;
    if (!(t >= 0.0f)) return 0;
    return min((int)floorf(t), H - 1);
}

// One thread per pixel (row-major image, rows of W pixels, coalesced along
// a row).  Polyline: column b spans the rows between its height's row and
// the next column's; bars: rows 0 .. its height's row.  `y` holds the
// heights of `lines` lines, one after another (W each); image l is at
// img + l * H * W.
__global__ __launch_bounds__(256) void k_rasterize(const float* __restrict__ y, int32_t W, int32_t H,
                                                   int32_t lines, int32_t mode, uint8_t* __restrict__ img) {
    const int64_t total = (int64_t)lines * H * W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t l = i / ((int64_t)H * W);
        const int64_t p = i - l * H * W;
        const int r = (int)(p / W), b = (int)(p - (int64_t)r * W);
        const float* yl = y + l * W;
        const int r0 = raster_row(yl[b], H);
        int lo, hi;
        if (mode == kRasterBars) {
            lo = 0;
            hi = r0;
        } else {
            const int r1 = b + 1 < W ? raster_row(yl[b + 1], H) : r0;
            lo = min(r0, r1);
            hi = max(r0, r1);
        }
        img[i] = (r >= lo && r <= hi) ? 1 : 0;
    }
}

dvl_status launch_rasterize(const float* y, int32_t W, int32_t H, int32_t lines, int32_t mode, uint8_t* img,
                            hipStream_t st) {
    const int64_t total = (int64_t)lines * H * W;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(k_rasterize, dim3(grid), dim3(256), 0, st, y, W, H, lines, mode, img);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ brushing

// For every sorted cell h: 1 at its original index if its key lies in one of
// the n_ranges closed ranges [lo[i], hi[i]] (held in LDS), else 0.
// (the ranges travel as a kernel argument: no device buffer is needed)
struct KeyRanges {
    int32_t n;
    uint64_t lohi[2 * kMaxSelectRanges];
};

__global__ __launch_bounds__(256) void k_select_mask(int64_t n, const uint64_t* __restrict__ keys_sorted,
                                                     const uint32_t* __restrict__ perm, KeyRanges rg,
                                                     uint8_t* __restrict__ mask) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n; h += stride) {
        const uint64_t k = keys_sorted[h];
        uint8_t in = 0;
        for (int i = 0; i < rg.n; ++i) in |= (k >= rg.lohi[2 * i] && k <= rg.lohi[2 * i + 1]) ? 1 : 0;
        const uint32_t o = perm[h];
        if (o < (uint64_t)n) mask[o] = in;
    }
}

dvl_status launch_select_mask(int64_t n, const uint64_t* keys_sorted, const uint32_t* perm, int32_t n_ranges,
                              const uint64_t* ranges, uint8_t* mask, hipStream_t st) {
    if (n_ranges < 0 || n_ranges > kMaxSelectRanges) return DVL_E_INVALID;
    KeyRanges rg;
    rg.n = n_ranges;
    for (int i = 0; i < 2 * kMaxSelectRanges; ++i) rg.lohi[i] = i < 2 * n_ranges ? ranges[i] : 0;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
    hipLaunchKernelGGL(k_select_mask, dim3(grid), dim3(256), 0, st, n, keys_sorted, perm, rg, mask);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ zoom

__global__ __launch_bounds__(256) void k_iota(int64_t n, uint32_t* __restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = (uint32_t)i;
}

dvl_status launch_iota(int64_t n, uint32_t* out, hipStream_t st) {
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
    hipLaunchKernelGGL(k_iota, dim3(grid), dim3(256), 0, st, n, out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

}  // namespace dvl
