// Internal helpers of the DVL library (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dvl.h"

namespace dvl {

constexpr int kWave = 64;
constexpr int kMaxFields = 16;
constexpr int kMaxTfEntries = 4096;
constexpr int kMaxTfTotal = 16384;          // M * n_tf, lives in LDS (64 KB)

// ---------------------------------------------------------------- lanes

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T readlane(T v, int l);

template <>
__device__ __forceinline__ float readlane<float>(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ int readlane<int>(int v, int l) {
    return __builtin_amdgcn_readlane(v, l);
}
template <>
__device__ __forceinline__ uint32_t readlane<uint32_t>(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
template <>
__device__ __forceinline__ double readlane<double>(double v, int l) {
    uint64_t u = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// DPP controls (GFX9): row_shr:n shifts within rows of 16 lanes
#define DVL_DPP_ROW_SHR(n) (0x110 + (n))

// move from lane - n of the same row; lanes whose source is outside the row get 0
__device__ __forceinline__ float dpp_row_shr_f(float v, int n) {
    int r;
    switch (n) {
        case 1: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), DVL_DPP_ROW_SHR(1), 0xF, 0xF, false); break;
        case 2: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), DVL_DPP_ROW_SHR(2), 0xF, 0xF, false); break;
        case 4: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), DVL_DPP_ROW_SHR(4), 0xF, 0xF, false); break;
        default: r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), DVL_DPP_ROW_SHR(8), 0xF, 0xF, false); break;
    }
    return __int_as_float(r);
}

// Inclusive wave64 sum scan: Hillis-Steele inside each row of 16 lanes via
// DPP row shifts, then row totals combined through readlane.  The result is
// NOT guaranteed monotone under rounding; callers that need monotone
// prefixes follow it with wave_max_scan.
__device__ __forceinline__ float wave_incl_sum(float v) {
    v += dpp_row_shr_f(v, 1);
    v += dpp_row_shr_f(v, 2);
    v += dpp_row_shr_f(v, 4);
    v += dpp_row_shr_f(v, 8);
    const float r0 = readlane(v, 15), r1 = readlane(v, 31), r2 = readlane(v, 47);
    const int row = lane_id() >> 4;
    const float o1 = r0, o2 = r0 + r1, o3 = o2 + r2;
    const float off = row == 0 ? 0.0f : (row == 1 ? o1 : (row == 2 ? o2 : o3));
    return v + off;
}

__device__ __forceinline__ float dpp_row_shr_max(float v, int n) {
    // source outside the row yields -0.0f-free neutral element: use the lane's own value
    int r;
    switch (n) {
        case 1: r = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), DVL_DPP_ROW_SHR(1), 0xF, 0xF, false); break;
        case 2: r = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), DVL_DPP_ROW_SHR(2), 0xF, 0xF, false); break;
        case 4: r = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), DVL_DPP_ROW_SHR(4), 0xF, 0xF, false); break;
        default: r = __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), DVL_DPP_ROW_SHR(8), 0xF, 0xF, false); break;
    }
    return __int_as_float(r);
}

// Inclusive wave64 running maximum.
__device__ __forceinline__ float wave_incl_max(float v) {
    v = fmaxf(v, dpp_row_shr_max(v, 1));
    v = fmaxf(v, dpp_row_shr_max(v, 2));
    v = fmaxf(v, dpp_row_shr_max(v, 4));
    v = fmaxf(v, dpp_row_shr_max(v, 8));
    const float r0 = readlane(v, 15), r1 = readlane(v, 31), r2 = readlane(v, 47);
    const int row = lane_id() >> 4;
    const float o2 = fmaxf(r0, r1), o3 = fmaxf(o2, r2);
    const float off = row == 0 ? v : (row == 1 ? r0 : (row == 2 ? o2 : o3));
    return fmaxf(v, off);
}

// value of lane - 1 (lane 0 gets `first`)
__device__ __forceinline__ float shfl_up1(float v, float first) {
    const int l = lane_id();
    int r = __builtin_amdgcn_ds_bpermute((l == 0 ? 0 : l - 1) << 2, __float_as_int(v));
    return l == 0 ? first : __int_as_float(r);
}

__device__ __forceinline__ int shfl_up_i(int v, int d) {
    const int l = lane_id();
    return __builtin_amdgcn_ds_bpermute((l >= d ? l - d : l) << 2, v);
}
__device__ __forceinline__ float shfl_up_f(float v, int d) {
    return __int_as_float(shfl_up_i(__float_as_int(v), d));
}
__device__ __forceinline__ double shfl_up_d(double v, int d) {
    uint64_t u = __double_as_longlong(v);
    int lo = shfl_up_i((int)(uint32_t)u, d), hi = shfl_up_i((int)(uint32_t)(u >> 32), d);
    return __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int shfl_i(int v, int src) {
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

// wave64 butterfly reductions (result in every lane)
__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t u = __double_as_longlong(v);
        const int l = lane_id() ^ o;
        int lo = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)u);
        int hi = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)(u >> 32));
        v += __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    return v;
}
__device__ __forceinline__ float wave_min_f(float v) {
    for (int o = 32; o > 0; o >>= 1)
        v = fminf(v, __int_as_float(__builtin_amdgcn_ds_bpermute((lane_id() ^ o) << 2, __float_as_int(v))));
    return v;
}
__device__ __forceinline__ float wave_max_f(float v) {
    for (int o = 32; o > 0; o >>= 1)
        v = fmaxf(v, __int_as_float(__builtin_amdgcn_ds_bpermute((lane_id() ^ o) << 2, __float_as_int(v))));
    return v;
}

// ---------------------------------------------------------------- storage types

struct F32 { using raw = float; static constexpr int bytes = 4; };
struct F16 { using raw = uint16_t; static constexpr int bytes = 2; };
struct BF16 { using raw = uint16_t; static constexpr int bytes = 2; };

__device__ __forceinline__ float to_f32(F32, float v) { return v; }
__device__ __forceinline__ float to_f32(F16, uint16_t v) {
    return (float)__builtin_bit_cast(_Float16, v);
}
__device__ __forceinline__ float to_f32(BF16, uint16_t v) {
    return __uint_as_float((uint32_t)v << 16);
}

// Loads and stores through pointers known to address global memory.  The
// kernels receive their buffers inside descriptor tables in memory, so the
// compiler cannot infer the address space and would emit flat instructions,
// which share the LDS counter: every wait for an LDS result would then also
// wait for the outstanding prefetch loads.
#define DVL_GLOBAL __attribute__((address_space(1)))

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ T gload(const void* base, int64_t i) {
    return ((const DVL_GLOBAL T*)base)[i];
}
template <typename T>
__device__ __forceinline__ void gstore(void* base, int64_t i, T v) {
    ((DVL_GLOBAL T*)base)[i] = v;
}
// scalar base + 32-bit byte offset: one global load with a scalar address
template <typename T>
__device__ __forceinline__ T gload_at(const char* base, uint32_t byte_off) {
    const DVL_GLOBAL char* g = (const DVL_GLOBAL char*)base;
    return *(const DVL_GLOBAL T*)(g + byte_off);
}

// The constant address space (the dispatch packet is read through it).
#define DVL_CONST __attribute__((address_space(4)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Work-item and work-group indices from the hardware and the dispatch packet.
// The kernels of the update run in non-IEEE float mode, which keeps the
// device library's functions from being inlined into them; an out-of-line
// call waits for every memory operation in flight on entry, so the hot
// kernels use these instead of threadIdx / blockIdx / blockDim / gridDim.
__device__ __forceinline__ int thread_x() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int block_x() { return (int)__builtin_amdgcn_workgroup_id_x(); }
__device__ __forceinline__ int block_dim_x() {
    const DVL_CONST uint16_t* pk = (const DVL_CONST uint16_t*)__builtin_amdgcn_dispatch_ptr();
    return (int)pk[2];                        // workgroup_size_x
}
__device__ __forceinline__ int grid_dim_x() {
    const DVL_CONST uint32_t* pk = (const DVL_CONST uint32_t*)__builtin_amdgcn_dispatch_ptr();
    const uint32_t wg = (uint32_t)block_dim_x();
    return (int)((pk[3] + wg - 1) / wg);      // grid_size_x in work-items
}

// Values that are the same in every lane (descriptor fields) moved to scalar
// registers, so that branches on them are scalar branches and addresses built
// from them use scalar bases.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
    return reinterpret_cast<T*>(uni((int64_t)reinterpret_cast<uintptr_t>(p)));
}

// four consecutive values starting at a 4-aligned index
template <typename S>
struct Quad;
template <>
struct Quad<F32> {
    static constexpr uint32_t kBytes = 16;
    f32x4 v;
    __device__ __forceinline__ void load(const void* base, int64_t i4) { v = gload<f32x4>(base, i4); }
    __device__ __forceinline__ void load_at(const char* base, uint32_t off) { v = gload_at<f32x4>(base, off); }
    __device__ __forceinline__ float get(int k) const {
        return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
    }
};
template <typename S16>
struct Quad16 {
    static constexpr uint32_t kBytes = 8;
    u32x2 v;
    __device__ __forceinline__ void load(const void* base, int64_t i4) { v = gload<u32x2>(base, i4); }
    __device__ __forceinline__ void load_at(const char* base, uint32_t off) { v = gload_at<u32x2>(base, off); }
    __device__ __forceinline__ float get(int k) const {
        const uint32_t w = k < 2 ? v.x : v.y;
        const uint16_t h = (uint16_t)((k & 1) ? (w >> 16) : (w & 0xFFFF));
        return to_f32(S16{}, h);
    }
};
template <>
struct Quad<F16> : Quad16<F16> {};
template <>
struct Quad<BF16> : Quad16<BF16> {};

// ---------------------------------------------------------------- host side

struct Status {
    dvl_status code = DVL_OK;
};

void set_error(const char* fmt, ...);
dvl_status hip_fail(hipError_t e, const char* what);

}  // namespace dvl

#define DVL_HIP(call)                                                 \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ::dvl::hip_fail(e_, #call);      \
    } while (0)
