// Launchers of the one-time ordering kernels (order.hip).
#pragma once

#include "common.hpp"

namespace dvl {

dvl_status launch_extent(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                         const uint8_t* level, unsigned long long* out, hipStream_t s);
dvl_status launch_keys(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                       const uint8_t* level, int bits, uint64_t* keys, uint32_t* idx, hipStream_t s);
// stable LSD sort of (keys, vals) on the low key_bits bits; ping-pongs between the
// two buffer pairs and reports which holds the result
dvl_status radix_sort(int64_t n, int key_bits, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                      uint32_t* vals_tmp, uint32_t* counts, uint32_t* partial, hipStream_t s,
                      uint64_t** keys_out, uint32_t** vals_out);
int64_t sort_tile_count(int64_t n);        // sort tiles rounded up to a group of 16; counts needs 256 * that
int64_t scan_partial_count(int64_t n);     // partial sums the count scan needs for n entries
dvl_status launch_dup(int64_t n, const uint64_t* keys, unsigned long long* flag, hipStream_t s);
dvl_status launch_gather(int64_t n, const uint32_t* perm, const void* src, void* dst, int elem_bytes,
                         hipStream_t s);
dvl_status launch_scatter_back(int64_t n, const uint32_t* perm, const void* sorted, void* orig,
                               int elem_bytes, hipStream_t s);
// out[0] = min, out[1] = max as order-preserving uint keys, out[2] = NaN seen
dvl_status launch_range(int64_t n, int dtype, const void* v, unsigned int* out, hipStream_t s);
// dst[i] = src[perm[i]] for a field of storage `dtype`, with the range of the values as launch_range
dvl_status launch_gather_range(int64_t n, const uint32_t* perm, int dtype, const void* src, void* dst,
                               unsigned int* out, hipStream_t s);

}  // namespace dvl
