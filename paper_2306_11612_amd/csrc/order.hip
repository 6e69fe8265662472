// One-time ordering: Hilbert keys at finest-level resolution, LSD radix
// sort of (key, original index), gather of levels and fields into sorted
// order, and per-field data ranges.
//
// Paper: Background (AMR cells snapped to the logical grid: lower corner +
// level, width 2^L), Dynamic Volume Lines (cells represented by quantised
// centroids, ordered along a Hilbert curve), GPU section (the order is
// established once; only the spacing changes afterwards).
#include "order.hpp"

#include <algorithm>

namespace dvl {

// ===================================================================
// extent: max(corner + 2^level) over all cells and axes, plus range checks
// ===================================================================
__global__ __launch_bounds__(256) void k_extent(int64_t n, const int32_t* __restrict__ x,
                                                const int32_t* __restrict__ y,
                                                const int32_t* __restrict__ z,
                                                const uint8_t* __restrict__ level,
                                                unsigned long long* __restrict__ out /* [0] max upper corner, [1] bad, [2] max level */) {
    int64_t mx = 0;
    uint32_t bad = 0, lmax = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t cx = x[i], cy = y[i], cz = z[i];
        const uint32_t L = level[i];
        bad |= (cx < 0) | (cy < 0) | (cz < 0) | (L > 20u);
        lmax = max(lmax, L);
        const int64_t w = (int64_t)1 << (L & 31u);
        const int64_t m = max(max((int64_t)cx, (int64_t)cy), (int64_t)cz) + w;
        mx = max(mx, m);
    }
    // wave reduce then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
        const int l = lane_id() ^ o;
        int lo = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)mx);
        int hi = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)((uint64_t)mx >> 32));
        mx = max(mx, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
        bad |= (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)bad);
        lmax = max(lmax, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)lmax));
    }
    if (lane_id() == 0) {
        atomicMax(&out[0], (unsigned long long)mx);
        if (bad) atomicOr(&out[1], 1ull);
        atomicMax(&out[2], (unsigned long long)lmax);
    }
}

// ===================================================================
// Hilbert index (Skilling 2004, "Programming the Hilbert curve"): the
// axes are turned into the transposed index by undoing the recursive
// construction's excess work plane by plane from the top, then Gray-coded;
// the bits are interleaved with axis x most significant in every 3-bit
// digit.  The final Gray correction is computed in closed form: its bit j is
// the parity of the bits of the last axis above j.
// ===================================================================
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t hilbert3(uint32_t a, uint32_t b, uint32_t c, int bits) {
    for (int j = bits - 1; j >= 1; --j) {
        const uint32_t Q = 1u << j, P = Q - 1u;
        // axis 0 against itself: invert when set, exchanging with itself is a no-op
        a ^= (a & Q) ? P : 0u;
        if (b & Q) {
            a ^= P;
        } else {
            const uint32_t t = (a ^ b) & P;
            a ^= t;
            b ^= t;
        }
        if (c & Q) {
            a ^= P;
        } else {
            const uint32_t t = (a ^ c) & P;
            a ^= t;
            c ^= t;
        }
    }
    b ^= a;
    c ^= b;
    uint32_t t = c >> 1;          // bit j of t = xor of bits > j of c
    t ^= t >> 1;
    t ^= t >> 2;
    t ^= t >> 4;
    t ^= t >> 8;
    t ^= t >> 16;
    const uint32_t mask = (bits >= 32) ? 0xFFFFFFFFu : ((1u << bits) - 1u);
    t &= mask;
    a ^= t;
    b ^= t;
    c ^= t;
    return (spread3(a) << 2) | (spread3(b) << 1) | spread3(c);
}

__global__ __launch_bounds__(256) void k_keys(int64_t n, const int32_t* __restrict__ x,
                                              const int32_t* __restrict__ y,
                                              const int32_t* __restrict__ z,
                                              const uint8_t* __restrict__ level, int bits,
                                              uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t half = (1u << level[i]) >> 1;
        keys[i] = hilbert3((uint32_t)x[i] + half, (uint32_t)y[i] + half, (uint32_t)z[i] + half, bits);
        idx[i] = (uint32_t)i;
    }
}

// The same two passes over four consecutive cells per thread and iteration
// (x, y, z 16-byte aligned and level 4-byte aligned, checked by the
// launchers): vector loads of the coordinates and levels, vector stores of
// the keys and indices; the last n % 4 cells one by one.
__device__ __forceinline__ void extent_add(int32_t cx, int32_t cy, int32_t cz, uint32_t L, int64_t& mx,
                                           uint32_t& bad, uint32_t& lmax) {
    bad |= (cx < 0) | (cy < 0) | (cz < 0) | (L > 20u);
    lmax = max(lmax, L);
    const int64_t w = (int64_t)1 << (L & 31u);
    mx = max(mx, max(max((int64_t)cx, (int64_t)cy), (int64_t)cz) + w);
}

__global__ __launch_bounds__(256) void k_extent4(int64_t n, const int32_t* __restrict__ x,
                                                 const int32_t* __restrict__ y,
                                                 const int32_t* __restrict__ z,
                                                 const uint8_t* __restrict__ level,
                                                 unsigned long long* __restrict__ out) {
    int64_t mx = 0;
    uint32_t bad = 0, lmax = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = n >> 2;
    for (int64_t q = tid; q < nq; q += stride) {
        const int4 cx = reinterpret_cast<const int4*>(x)[q];
        const int4 cy = reinterpret_cast<const int4*>(y)[q];
        const int4 cz = reinterpret_cast<const int4*>(z)[q];
        const uint32_t lw = reinterpret_cast<const uint32_t*>(level)[q];
        extent_add(cx.x, cy.x, cz.x, lw & 0xFFu, mx, bad, lmax);
        extent_add(cx.y, cy.y, cz.y, (lw >> 8) & 0xFFu, mx, bad, lmax);
        extent_add(cx.z, cy.z, cz.z, (lw >> 16) & 0xFFu, mx, bad, lmax);
        extent_add(cx.w, cy.w, cz.w, lw >> 24, mx, bad, lmax);
    }
    for (int64_t i = 4 * nq + tid; i < n; i += stride) extent_add(x[i], y[i], z[i], level[i], mx, bad, lmax);
    for (int o = 32; o > 0; o >>= 1) {
        const int l = lane_id() ^ o;
        int lo = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)mx);
        int hi = __builtin_amdgcn_ds_bpermute(l << 2, (int)(uint32_t)((uint64_t)mx >> 32));
        mx = max(mx, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
        bad |= (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)bad);
        lmax = max(lmax, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)lmax));
    }
    if (lane_id() == 0) {
        atomicMax(&out[0], (unsigned long long)mx);
        if (bad) atomicOr(&out[1], 1ull);
        atomicMax(&out[2], (unsigned long long)lmax);
    }
}

__global__ __launch_bounds__(256) void k_keys4(int64_t n, const int32_t* __restrict__ x,
                                               const int32_t* __restrict__ y,
                                               const int32_t* __restrict__ z,
                                               const uint8_t* __restrict__ level, int bits,
                                               uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = n >> 2;
    for (int64_t q = tid; q < nq; q += stride) {
        const int4 cx = reinterpret_cast<const int4*>(x)[q];
        const int4 cy = reinterpret_cast<const int4*>(y)[q];
        const int4 cz = reinterpret_cast<const int4*>(z)[q];
        const uint32_t lw = reinterpret_cast<const uint32_t*>(level)[q];
        const int32_t xs[4] = {cx.x, cx.y, cx.z, cx.w}, ys[4] = {cy.x, cy.y, cy.z, cy.w},
                      zs[4] = {cz.x, cz.y, cz.z, cz.w};
        uint64_t k4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t half = (1u << ((lw >> (8 * k)) & 0xFFu)) >> 1;
            k4[k] = hilbert3((uint32_t)xs[k] + half, (uint32_t)ys[k] + half, (uint32_t)zs[k] + half, bits);
        }
        u64x2* kd = reinterpret_cast<u64x2*>(keys + 4 * q);
        kd[0] = u64x2{k4[0], k4[1]};
        kd[1] = u64x2{k4[2], k4[3]};
        const uint32_t i0 = (uint32_t)(4 * q);
        reinterpret_cast<u32x4*>(idx)[q] = u32x4{i0, i0 + 1, i0 + 2, i0 + 3};
    }
    for (int64_t i = 4 * nq + tid; i < n; i += stride) {
        const uint32_t half = (1u << level[i]) >> 1;
        keys[i] = hilbert3((uint32_t)x[i] + half, (uint32_t)y[i] + half, (uint32_t)z[i] + half, bits);
        idx[i] = (uint32_t)i;
    }
}

// ===================================================================
// LSD radix sort, 8-bit digits.  Per pass:
//   k_digit_hist   per-tile digit counts, stored digit-major [256][T_pad]
//                  (T_pad: tiles rounded up to a group of 16); one workgroup
//                  counts 16 consecutive tiles and writes each digit's 16
//                  counts as one contiguous 64-byte run
//   scan_u32       exclusive scan of that array (global bucket offsets)
//   k_scatter      stable in-tile ranking (wave match of equal digits),
//                  staging of the tile in digit order in LDS, then writes of
//                  contiguous runs to the global offsets
// ===================================================================
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                       // per thread
constexpr int kSortTile = kSortThreads * kSortItems; // 4096 keys
constexpr int kWavesPerSortTile = kSortThreads / kWave;
constexpr int kRadix = 256;
constexpr int kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2

constexpr int kHistGroup = 16;   // tiles per k_digit_hist workgroup (64 B of counts per digit)

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(int64_t n, const uint64_t* __restrict__ keys,
                                                             int shift, int64_t t_pad,
                                                             uint32_t* __restrict__ counts) {
    __shared__ uint32_t hist[kWavesPerSortTile][kRadix];
    __shared__ uint32_t out[kRadix][kHistGroup];
    const int w = threadIdx.x / kWave;
    const int64_t tile0 = (int64_t)blockIdx.x * kHistGroup;
    for (int g = 0; g < kHistGroup; ++g) {
        for (int i = threadIdx.x; i < kWavesPerSortTile * kRadix; i += kSortThreads)
            (&hist[0][0])[i] = 0;
        __syncthreads();
        const int64_t base = (tile0 + g) * kSortTile;
#pragma unroll 4
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
            if (i < n) {
                const uint32_t d = (uint32_t)(keys[i] >> shift) & 0xFFu;
                atomicAdd(&hist[w][d], 1u);
            }
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < kWavesPerSortTile; ++q) c += hist[q][d];
            out[d][g] = c;
        }
        __syncthreads();
    }
    // digit d's counts of the group's 16 tiles: one 64-byte run
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
        uint4* dst = reinterpret_cast<uint4*>(counts + (int64_t)d * t_pad + tile0);
#pragma unroll
        for (int q = 0; q < kHistGroup / 4; ++q)
            dst[q] = make_uint4(out[d][4 * q], out[d][4 * q + 1], out[d][4 * q + 2], out[d][4 * q + 3]);
    }
}

// exclusive scan of uint32 (values and totals fit 32 bits: n_cells < 2^32)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanBlock = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* sh /* [kScanThreads/64] */,
                                                        uint32_t* total) {
    // wave inclusive scan (shuffles), then wave totals through LDS
    uint32_t x = v;
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = (uint32_t)shfl_up_i((int)x, d);
        if (lane_id() >= d) x += t;
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) sh[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
        if (q < w) off += sh[q];
        tot += sh[q];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(int64_t n, const uint32_t* __restrict__ in,
                                                              uint32_t* __restrict__ partial) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan_u32(s, sh, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(int64_t n_part, uint32_t* __restrict__ partial) {
    __shared__ uint32_t sh[1024 / kWave];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < n_part; b0 += blockDim.x) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < n_part ? partial[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32(v, sh, &tot);
        if (i < n_part) partial[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(int64_t n, const uint32_t* __restrict__ in,
                                                            const uint32_t* __restrict__ partial,
                                                            uint32_t* __restrict__ out) {
    __shared__ uint32_t sh[kScanThreads / kWave];
    // blocked arrangement: thread t owns items [t*kScanItems, (t+1)*kScanItems)
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + r;
        v[r] = i < n ? in[i] : 0u;
        s += v[r];
    }
    uint32_t tot;
    uint32_t run = partial[blockIdx.x] + block_excl_scan_u32(s, sh, &tot);
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + r;
        if (i < n) out[i] = run;
        run += v[r];
    }
}

static dvl_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partial,
                           hipStream_t s) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, n, in, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, nb, partial);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, n, in, partial, out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

int64_t scan_partial_count(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

__global__ __launch_bounds__(kSortThreads) void k_scatter(int64_t n, const uint64_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, int shift,
                                                          int64_t t_pad, const uint32_t* __restrict__ offs,
                                                          uint64_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout) {
    __shared__ uint32_t whist[kWavesPerSortTile][kRadix];   // per-wave digit counts, then bases
    __shared__ uint32_t tbase[kRadix];                      // tile-local start of each digit
    __shared__ uint32_t gbase[kRadix];                      // global start of each digit for this tile
    __shared__ uint32_t wsum[kSortThreads / kWave];
    // the tile in digit order: keys first, then (in the same space) values,
    // so that four workgroups fit a compute unit's LDS
    __shared__ uint64_t stage[kSortTile];
    uint32_t* sval = reinterpret_cast<uint32_t*>(stage);

    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    // Workgroups go to the 8 XCDs in turn; consecutive tiles on one XCD share
    // the L2 lines of their digit offsets (16 tiles per 64-byte run), so XCD x
    // takes the x-th contiguous eighth of the tiles.
    const int64_t nb = gridDim.x, bid = blockIdx.x;
    const int64_t xcd = bid % kXcds, per = nb / kXcds, rem = nb % kXcds;
    const int64_t tile = xcd * per + min(xcd, rem) + bid / kXcds;
    const int64_t tbeg = tile * kSortTile;
    const int n_here = (int)min((int64_t)kSortTile, n - tbeg);

    for (int i = threadIdx.x; i < kWavesPerSortTile * kRadix; i += kSortThreads) (&whist[0][0])[i] = 0;
    __syncthreads();

    // each wave owns a contiguous quarter of the tile; round r covers 64 keys
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int li = w * (kWave * kSortItems) + r * kWave + lane;   // tile-local index
        const bool ok = li < n_here;
        key[r] = ok ? kin[tbeg + li] : 0ull;
        val[r] = ok ? vin[tbeg + li] : 0u;
        const uint32_t d = ok ? ((uint32_t)(key[r] >> shift) & 0xFFu) : 0u;
        // lanes holding the same digit
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t b = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? b : ~b;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        const uint32_t old = ok ? whist[w][d] : 0u;
        rank[r] = old + before;
        // the lowest peer bumps the counter by the group size
        if (ok && before == 0) whist[w][d] = old + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: wave bases inside the tile and the tile's digit start
    if (threadIdx.x < kRadix) {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kWavesPerSortTile; ++q) {
            const uint32_t c = whist[q][d];
            whist[q][d] = run;
            run += c;
        }
        tbase[d] = run;   // tile count of digit d for now
        gbase[d] = offs[(int64_t)d * t_pad + tile];
    }
    __syncthreads();
    // exclusive scan of the 256 tile counts (threads 0..255 hold one each)
    {
        const uint32_t c = threadIdx.x < kRadix ? tbase[threadIdx.x] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32(c, wsum, &tot);
        __syncthreads();
        if (threadIdx.x < kRadix) tbase[threadIdx.x] = ex;
    }
    __syncthreads();

    // positions in digit order, kept for the value pass
    uint32_t pos[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int li = w * (kWave * kSortItems) + r * kWave + lane;
        pos[r] = 0xFFFFFFFFu;
        if (li < n_here) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
            const uint32_t p = tbase[d] + whist[w][d] + rank[r];
            if (p < (uint32_t)kSortTile) {
                pos[r] = p;
                stage[p] = key[r];
            }
        }
    }
    __syncthreads();
    // keys out (contiguous runs per digit); remember each slot's destination
    uint32_t dest[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = r * kSortThreads + threadIdx.x;
        dest[r] = 0xFFFFFFFFu;
        if (i < n_here) {
            const uint64_t k = stage[i];
            const uint32_t d = (uint32_t)(k >> shift) & 0xFFu;
            const int64_t g = (int64_t)gbase[d] + (i - (int64_t)tbase[d]);
            if (g >= 0 && g < n) {
                kout[g] = k;
                dest[r] = (uint32_t)g;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (pos[r] != 0xFFFFFFFFu) sval[pos[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int i = r * kSortThreads + threadIdx.x;
        if (i < n_here && dest[r] != 0xFFFFFFFFu) vout[dest[r]] = sval[i];
    }
}

// flag adjacent equal keys
__global__ __launch_bounds__(256) void k_dup(int64_t n, const uint64_t* __restrict__ k,
                                             unsigned long long* __restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t d = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride)
        d |= (k[i] == k[i - 1]);
    if (__ballot(d) != 0ull && lane_id() == 0) atomicOr(flag, 1ull);
}

dvl_status radix_sort(int64_t n, int key_bits, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                      uint32_t* vals_tmp, uint32_t* counts, uint32_t* partial, hipStream_t s,
                      uint64_t** keys_out, uint32_t** vals_out) {
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t t_pad = sort_tile_count(n);
    const int passes = std::max(1, (key_bits + 7) / 8);
    uint64_t* ka = keys; uint64_t* kb = keys_tmp;
    uint32_t* va = vals; uint32_t* vb = vals_tmp;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)(t_pad / kHistGroup)), dim3(kSortThreads), 0, s, n, ka,
                           shift, t_pad, counts);
        DVL_HIP(hipGetLastError());
        dvl_status st = scan_u32(counts, counts, (int64_t)kRadix * t_pad, partial, s);
        if (st != DVL_OK) return st;
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)n_tiles), dim3(kSortThreads), 0, s, n, ka, va, shift,
                           t_pad, counts, kb, vb);
        DVL_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *keys_out = ka;
    *vals_out = va;
    return DVL_OK;
}

int64_t sort_tile_count(int64_t n) {
    const int64_t t = (n + kSortTile - 1) / kSortTile;
    return (t + kHistGroup - 1) / kHistGroup * kHistGroup;
}

// ===================================================================
// gather into sorted order; data ranges
// ===================================================================
template <typename T>
struct alignas(4 * sizeof(T)) Four {
    T v[4];
};

// dst[i] = src[perm[i]]; four consecutive i per thread and iteration (perm and
// dst are the volume's own, 256-byte aligned): one 16-byte load of perm, four
// scattered loads in flight together, one vector store
template <typename T>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const uint32_t* __restrict__ perm,
                                                const T* __restrict__ src, T* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = n >> 2;
    for (int64_t q = tid; q < nq; q += stride) {
        const u32x4 p = *reinterpret_cast<const u32x4*>(perm + 4 * q);
        const uint32_t pk[4] = {p.x, p.y, p.z, p.w};
        Four<T> o;
#pragma unroll
        for (int k = 0; k < 4; ++k) o.v[k] = pk[k] < (uint64_t)n ? src[pk[k]] : T(0);
        reinterpret_cast<Four<T>*>(dst)[q] = o;
    }
    for (int64_t i = 4 * nq + tid; i < n; i += stride) {
        const uint32_t p = perm[i];
        if (p < (uint64_t)n) dst[i] = src[p];
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_range(int64_t n, const typename S::raw* __restrict__ v,
                                               unsigned int* __restrict__ out /* [0] min key, [1] max key, [2] nan */) {
    // order-preserving map of floats to unsigned ints
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, nan = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float f = to_f32(S{}, v[i]);
        if (f != f) { nan = 1u; continue; }
        uint32_t u = __float_as_uint(f);
        u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        lo = min(lo, u);
        hi = max(hi, u);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int l = lane_id() ^ o;
        lo = min(lo, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)lo));
        hi = max(hi, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)hi));
        nan |= (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)nan);
    }
    if (lane_id() == 0) {
        atomicMin(&out[0], lo);
        atomicMax(&out[1], hi);
        if (nan) atomicOr(&out[2], 1u);
    }
}

// gather of one field into sorted order fused with its data range (the
// order-preserving uint map of k_range; out[0] min, out[1] max, out[2] NaN)
template <typename S>
__device__ __forceinline__ void range_add(float f, uint32_t& lo, uint32_t& hi, uint32_t& nan) {
    if (f != f) {
        nan = 1u;
        return;
    }
    uint32_t u = __float_as_uint(f);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    lo = min(lo, u);
    hi = max(hi, u);
}

// Four consecutive sorted cells per thread and iteration: one 16-byte load of
// their permutation entries, then the four (scattered) value loads in flight
// together, one vector store; the last n % 4 cells one by one.
template <typename S>
__global__ __launch_bounds__(256) void k_gather_range(int64_t n, const uint32_t* __restrict__ perm,
                                                      const typename S::raw* __restrict__ src,
                                                      typename S::raw* __restrict__ dst,
                                                      unsigned int* __restrict__ out) {
    using raw = typename S::raw;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, nan = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = n >> 2;
    for (int64_t q = tid; q < nq; q += stride) {
        const u32x4 p = *reinterpret_cast<const u32x4*>(perm + 4 * q);
        const uint32_t pk[4] = {p.x, p.y, p.z, p.w};
        raw r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = pk[k] < (uint64_t)n ? src[pk[k]] : raw(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            dst[4 * q + k] = r[k];
            if (pk[k] < (uint64_t)n) range_add<S>(to_f32(S{}, r[k]), lo, hi, nan);
        }
    }
    for (int64_t i = 4 * nq + tid; i < n; i += stride) {
        const uint32_t p = perm[i];
        if (p >= (uint64_t)n) continue;
        const raw r = src[p];
        dst[i] = r;
        range_add<S>(to_f32(S{}, r), lo, hi, nan);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const int l = lane_id() ^ o;
        lo = min(lo, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)lo));
        hi = max(hi, (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)hi));
        nan |= (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)nan);
    }
    if (lane_id() == 0) {
        atomicMin(&out[0], lo);
        atomicMax(&out[1], hi);
        if (nan) atomicOr(&out[2], 1u);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scatter_back(int64_t n, const uint32_t* __restrict__ perm,
                                                      const T* __restrict__ sorted, T* __restrict__ orig) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t p = perm[i];
        if (p < (uint64_t)n) orig[p] = sorted[i];
    }
}

static unsigned grid_for(int64_t n, int per_block = 256, int max_blocks = 8192) {
    int64_t g = (n + per_block - 1) / per_block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, max_blocks));
}

// the caller's coordinate and level arrays allow the 4-cell loads
static bool vec4_inputs(const int32_t* x, const int32_t* y, const int32_t* z, const uint8_t* level) {
    return ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(z)) & 15u) == 0 &&
           (reinterpret_cast<uintptr_t>(level) & 3u) == 0;
}

dvl_status launch_extent(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                         const uint8_t* level, unsigned long long* out, hipStream_t s) {
    if (vec4_inputs(x, y, z, level))
        hipLaunchKernelGGL(k_extent4, dim3(grid_for((n + 3) / 4)), dim3(256), 0, s, n, x, y, z, level, out);
    else
        hipLaunchKernelGGL(k_extent, dim3(grid_for(n)), dim3(256), 0, s, n, x, y, z, level, out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_keys(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                       const uint8_t* level, int bits, uint64_t* keys, uint32_t* idx, hipStream_t s) {
    if (vec4_inputs(x, y, z, level))
        hipLaunchKernelGGL(k_keys4, dim3(grid_for((n + 3) / 4)), dim3(256), 0, s, n, x, y, z, level, bits, keys, idx);
    else
        hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(256), 0, s, n, x, y, z, level, bits, keys, idx);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_dup(int64_t n, const uint64_t* keys, unsigned long long* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_dup, dim3(grid_for(n)), dim3(256), 0, s, n, keys, flag);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_gather(int64_t n, const uint32_t* perm, const void* src, void* dst, int elem_bytes,
                         hipStream_t s) {
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_gather<uint32_t>, dim3(grid_for(n)), dim3(256), 0, s, n, perm,
                           (const uint32_t*)src, (uint32_t*)dst);
    else if (elem_bytes == 2)
        hipLaunchKernelGGL(k_gather<uint16_t>, dim3(grid_for(n)), dim3(256), 0, s, n, perm,
                           (const uint16_t*)src, (uint16_t*)dst);
    else
        hipLaunchKernelGGL(k_gather<uint8_t>, dim3(grid_for(n)), dim3(256), 0, s, n, perm,
                           (const uint8_t*)src, (uint8_t*)dst);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_scatter_back(int64_t n, const uint32_t* perm, const void* sorted, void* orig,
                               int elem_bytes, hipStream_t s) {
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_scatter_back<uint64_t>, dim3(grid_for(n)), dim3(256), 0, s, n, perm,
                           (const uint64_t*)sorted, (uint64_t*)orig);
    else
        return DVL_E_INVALID;
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_gather_range(int64_t n, const uint32_t* perm, int dtype, const void* src, void* dst,
                               unsigned int* out, hipStream_t s) {
    if (dtype == DVL_F32)
        hipLaunchKernelGGL(k_gather_range<F32>, dim3(grid_for(n)), dim3(256), 0, s, n, perm, (const float*)src,
                           (float*)dst, out);
    else if (dtype == DVL_F16)
        hipLaunchKernelGGL(k_gather_range<F16>, dim3(grid_for(n)), dim3(256), 0, s, n, perm, (const uint16_t*)src,
                           (uint16_t*)dst, out);
    else
        hipLaunchKernelGGL(k_gather_range<BF16>, dim3(grid_for(n)), dim3(256), 0, s, n, perm, (const uint16_t*)src,
                           (uint16_t*)dst, out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_range(int64_t n, int dtype, const void* v, unsigned int* out, hipStream_t s) {
    if (dtype == DVL_F32)
        hipLaunchKernelGGL(k_range<F32>, dim3(grid_for(n)), dim3(256), 0, s, n, (const float*)v, out);
    else if (dtype == DVL_F16)
        hipLaunchKernelGGL(k_range<F16>, dim3(grid_for(n)), dim3(256), 0, s, n, (const uint16_t*)v, out);
    else
        hipLaunchKernelGGL(k_range<BF16>, dim3(grid_for(n)), dim3(256), 0, s, n, (const uint16_t*)v, out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

}  // namespace dvl
