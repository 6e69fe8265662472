// Device code of the per-update kernels that depend on the field storage
// type (K0 exact max V, K1 importance and tile sums, K3b rescan), their
// helpers, and the templated launcher.  Each storage type is instantiated in
// its own translation unit (update_f32.hip, update_f16.hip, update_bf16.hip);
// the storage-independent kernels and the per-kernel commentary are in
// update.hip.
#pragma once

#include "update.hpp"

#include <algorithm>
#include <atomic>
#include <climits>
#include <type_traits>

namespace dvl {

// ------------------------------------------------------------------ unit lookup

// last job whose first importance-pass unit is <= u
__device__ __forceinline__ int find_job_k1(const BatchDev& b, int64_t u) {
    int lo = 0, hi = b.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.jobs[mid].k1_unit0 <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_req_k3(const BatchDev& b, int64_t u) {
    int lo = 0, hi = b.n_reqs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.reqs[mid].k3_unit0 <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_req_k4(const BatchDev& b, int64_t u) {
    int lo = 0, hi = b.n_reqs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.reqs[mid].k4_unit0 <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ per-cell math

struct ImpCtx {
    float inv_vmax;
    float fmin;
    float p;
    int exp_is_one;
    int clamp_mode;
    int lshift;
};

__device__ __forceinline__ ImpCtx make_ctx(const ReqDev& q) {
    ImpCtx c;
    const float vm = uni(gload<float>(q.vmax_dev, 0));
    c.inv_vmax = vm > 0.0f ? 1.0f / vm : 0.0f;
    c.fmin = uni(q.fmin);
    c.p = uni(q.exponent);
    c.exp_is_one = uni(q.exp_is_one);
    c.clamp_mode = uni(q.clamp_mode);
    c.lshift = uni(q.level_shift);
    return c;
}

// TF entry: clamp(floor(fma(x, s, b)), 0, n_tf - 1); the clamp is one
// median-of-three (nmax >= 1), the floor the truncation of a value >= 0
__device__ __forceinline__ int tf_entry(float x, float s, float b, float nmax) {
    return (int)__builtin_amdgcn_fmed3f(fmaf(x, s, b), 0.0f, nmax);
}

// Eq. 1: V = max_m alpha_m(x_m) - min_m alpha_m(x_m); `tf` is the request's block
template <int MT>
__device__ __forceinline__ float variation(const float (&x)[MT], int M, const float* __restrict__ tf,
                                           const ReqDev& q) {
    float amax = -INFINITY, amin = INFINITY;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const int e = tf_entry(x[m], q.s[m], q.b[m], q.nmax[m]);
            const float al = tf[q.tf_off[m] + e];
            amax = fmaxf(amax, al);
            amin = fminf(amin, al);
        }
    }
    return amax - amin;
}

// Eq. 3 with the minimum importance
__device__ __forceinline__ float importance_from_v(float v, uint32_t L, const ImpCtx& c) {
    const float r = v * c.inv_vmax;
    const int e = (int)(((uint32_t)c.lshift & 0xFFu) * (L & 0xFFu));   // 8 x 8 bits: a 24-bit multiply
    float f;
    if (c.clamp_mode == 0) {
        const float g = ldexpf(r, e);
        f = c.exp_is_one ? g : powf(g, c.p);
        f = fmaxf(f, c.fmin);
    } else {
        const float g = ldexpf(fmaxf(r, c.fmin), e);
        f = c.exp_is_one ? g : powf(g, c.p);
    }
    return f;
}

// Field count of a job: the variants MT = 1, 2, 4, 8 run batches whose jobs
// all have exactly MT fields (a compile-time count); MT = 16 reads it per job.
// Eq. 3 for P = 1 with the minimum importance on f (the paper's setting):
// the same operations as importance_from_v takes for it
__device__ __forceinline__ float importance_p1(float v, uint32_t L, const ImpCtx& c) {
    const float r = v * c.inv_vmax;
    const int e = (int)(((uint32_t)c.lshift & 0xFFu) * (L & 0xFFu));   // 8 x 8 bits: a 24-bit multiply
    return fmaxf(ldexpf(r, e), c.fmin);
}

template <int MT>
__device__ __forceinline__ int fields_of(int M) {
    return MT <= 8 ? MT : M;
}

// A wave's streams over one run of a job: scalar base pointers advanced to
// the run's first cell, so every load is a scalar base plus a 32-bit lane
// offset (a run holds at most 1/64 of a volume, well below 2^32 bytes), and
// the level codes of the run's steps.
template <int MT>
struct RunView {
    const char* base[MT];
    const char* lev;
    const uint32_t* lcode;
};

// Levels of the 4 cells of a lane.  The per-step level code says for every
// 64 cells whether they share one level; lanes in such a segment take it from
// the code and point their level load at the run's first word (a cached
// line), so only segments of mixed levels fetch level bytes.
struct LaneLevels {
    uint32_t lv;   // loaded levels (meaningful for code 0xFF only)
    uint32_t lc;   // the lane's segment code
    __device__ __forceinline__ void load(const char* lev, uint32_t qd, uint32_t code) {
        lc = (code >> ((lane_id() >> 4) << 3)) & 0xFFu;
        lv = gload_at<uint32_t>(lev, lc == 0xFFu ? qd * 4u : 0u);
    }
    // the 4 levels as the bytes of one word: the loaded ones, or the code's
    // level in every byte (one select per step instead of one per cell)
    __device__ __forceinline__ uint32_t word() const {
        return lc == 0xFFu ? lv : __builtin_amdgcn_perm(0u, lc, 0u);
    }
    __device__ __forceinline__ uint32_t get(int k) const { return (word() >> (8 * k)) & 0xFFu; }
};

// values of the 4 cells of this lane in the given step
template <int MT, typename S>
struct StepData {
    static constexpr uint32_t kQuadBytes = Quad<S>::kBytes;
    Quad<S> q[MT];
    LaneLevels lv;
    __device__ static const void* source(const JobDev& j, int m) { return j.fields[m]; }
    // step: index from the run's first step; code: its level code
    __device__ __forceinline__ void load(const RunView<MT>& v, int M, int step, uint32_t code) {
        const uint32_t qd = (uint32_t)(step * kWave + lane_id());
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (m < M) q[m].load_at(v.base[m], qd * kQuadBytes);
        lv.load(v.lev, qd, code);
    }
};

// TF entries of the 4 cells of this lane in the given step, from the
// volume's entry cache (one byte per cell and field)
template <int MT>
struct StepIdx {
    static constexpr uint32_t kQuadBytes = 4;
    uint32_t e[MT];
    LaneLevels lv;
    __device__ static const void* source(const JobDev& j, int m) { return j.idx[m]; }
    __device__ __forceinline__ void load(const RunView<MT>& v, int M, int step, uint32_t code) {
        const uint32_t qd = (uint32_t)(step * kWave + lane_id());
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (m < M) e[m] = gload_at<uint32_t>(v.base[m], qd * 4u);
        lv.load(v.lev, qd, code);
    }
};

// the importance of the 4 cells of this lane, as the importance pass stored
// it (view.base[0]: the request's stored f)
template <int MT>
struct StepF {
    static constexpr uint32_t kQuadBytes = 16;
    f32x4 fv;
    __device__ __forceinline__ void load(const RunView<MT>& v, int M, int step, uint32_t code) {
        fv = gload_at<f32x4>(v.base[0], (uint32_t)(step * kWave + lane_id()) * kQuadBytes);
    }
};

template <int MT, typename D>
__device__ __forceinline__ RunView<MT> run_view(const JobDev& j, int M, int64_t c_begin) {
    RunView<MT> v;
    const int64_t quad0 = c_begin >> 2;
#pragma unroll
    for (int m = 0; m < MT; ++m)
        v.base[m] = m < M ? uni(reinterpret_cast<const char*>(D::source(j, m))) + quad0 * D::kQuadBytes : nullptr;
    v.lev = uni(reinterpret_cast<const char*>(j.level)) + quad0 * 4;
    v.lcode = uni(j.lcode) + (c_begin >> 8);
    return v;
}

// V of cell k of this lane for request q, from values or from cached
// entries; off[m]: start of field m's table in `tf` (the request's block)
template <int MT, typename S>
__device__ __forceinline__ float cell_v(const StepData<MT, S>& d, int k, int M, const float* lds0, const float* tf,
                                        const ReqDev& q, const int (&off)[MT]) {
    float xk[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) xk[m] = m < M ? d.q[m].get(k) : 0.0f;
    return variation<MT>(xk, M, tf, q);
}
// 4 x byte k of w (the byte offset of an entry in its table), one
// instruction through the byte operand select of the SDWA encoding
__device__ __forceinline__ uint32_t entry_x4(uint32_t w, int k) {
    uint32_t a;
    switch (k) {
    case 0:
        asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
            : "=v"(a) : "v"(w));
        break;
    case 1:
        asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
            : "=v"(a) : "v"(w));
        break;
    case 2:
        asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
            : "=v"(a) : "v"(w));
        break;
    default:
        asm("v_lshlrev_b32_sdwa %0, 2, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
            : "=v"(a) : "v"(w));
        break;
    }
    return a;
}

typedef __attribute__((address_space(3))) const float lds_f32;

// lds0: the kernel's dynamic LDS array, which starts at LDS address 0 (the
// kernels that take this path have no static LDS; their launcher checks), so
// an entry's LDS address is its byte offset in the table plus the table's
// compile-time offset, and the table offset lands in the instruction's
// immediate.
template <int MT>
__device__ __forceinline__ float cell_v(const StepIdx<MT>& d, int k, int M, const float* lds0, const float* tf,
                                        const ReqDev& q, const int (&off)[MT]) {
    const uint32_t tb = (uint32_t)(tf - lds0) * (uint32_t)sizeof(float);
    float amax = -INFINITY, amin = INFINITY;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const uint32_t a = entry_x4(d.e[m], k) + tb + (uint32_t)(m * kIdxTable * sizeof(float));
            const float al = *reinterpret_cast<lds_f32*>((uintptr_t)a);
            amax = fmaxf(amax, al);
            amin = fminf(amin, al);
        }
    }
    return amax - amin;
}

// the start of request q's tables in LDS for step type D
template <int MT, typename D> struct TableBase {
    __device__ static int of(int q, int toff) { return toff; }
};
template <int MT> struct TableBase<MT, StepIdx<MT>> {
    __device__ static int of(int q, int toff) { return q * MT * kIdxTable; }
};

// a request's table offsets, in scalar registers
template <int MT>
__device__ __forceinline__ void table_offsets(const ReqDev& q, int M, int (&off)[MT]) {
#pragma unroll
    for (int m = 0; m < MT; ++m) off[m] = m < M ? uni(q.tf_off[m]) : 0;
}

// How many steps one loop iteration loads ahead: one 4-vector per field is
// enough to keep HBM busy; 16-bit values are half of that and cached entries
// a quarter, so two or four steps go together (tiles hold a multiple of four
// steps and are padded, so the loads of a group stay inside the volume's
// buffers).
template <typename D> struct Group { static constexpr int n = 1; };
#ifndef DVL_ENTRY_GROUP
#define DVL_ENTRY_GROUP 4
#endif
template <int MT> struct Group<StepIdx<MT>> { static constexpr int n = DVL_ENTRY_GROUP; };
#ifndef DVL_HALF_GROUP
#define DVL_HALF_GROUP 2
#endif
template <int MT> struct Group<StepData<MT, F16>> { static constexpr int n = DVL_HALF_GROUP; };
template <int MT> struct Group<StepData<MT, BF16>> { static constexpr int n = DVL_HALF_GROUP; };

// level codes of the G steps of a group (step: its first, a multiple of G),
// through vector loads (every lane the same words): they are waited for in
// order with the stream loads (a scalar load would be waited for with the
// LDS lookups, and all outstanding scalar loads at once)
template <int G>
struct StepCodes {
    uint32_t c[G];
};
template <int G>
__device__ __forceinline__ StepCodes<G> load_codes(const uint32_t* lcode, int step) {
    StepCodes<G> r;
    if constexpr (G == 4) {
        const u32x4 w = gload<u32x4>(lcode + step, 0);
        r.c[0] = w.x;
        r.c[1] = w.y;
        r.c[2] = w.z;
        r.c[3] = w.w;
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) r.c[g] = gload<uint32_t>(lcode, step + g);
    }
    return r;
}

// ------------------------------------------------------------------ K0

template <int MT, int KR, typename D>
__device__ __forceinline__ void vmax_run(const BatchDev& b, const JobDev& j, int64_t r, const float* tf_lds) {
    constexpr int G = Group<D>::n;
    const int lane = lane_id();
    const int M = uni(fields_of<MT>(j.M));
    const int64_t n = uni(j.n);
    const int64_t tile_cells = (int64_t)uni(j.tile_steps) * kStepCells;
    const int64_t c_begin = r * uni(j.tiles_per_run) * tile_cells;
    const int64_t c_end = min(n, (r + 1) * uni(j.tiles_per_run) * tile_cells);
    const int nsteps = (int)((c_end - c_begin + kStepCells - 1) / kStepCells);
    const ReqDev* rq = b.reqs + uni(j.req0);
    float vmax[KR];
    int toff[KR], off[KR][MT];
#pragma unroll
    for (int q = 0; q < KR; ++q) {
        vmax[q] = 0.0f;
        if (q < j.n_req) {
            toff[q] = uni(rq[q].tf_job_off);
            table_offsets<MT>(rq[q], M, off[q]);
        }
    }
    const RunView<MT> view = run_view<MT, D>(j, M, c_begin);
    for (int s = 0; s < nsteps; s += G) {
        D d[G];
#pragma unroll
        for (int g = 0; g < G; ++g) d[g].load(view, M, s + g, 0u);   // levels unused
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (s + g >= nsteps) break;
            const int64_t quad = ((c_begin + (int64_t)(s + g) * kStepCells) >> 2) + lane;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((quad << 2) + k >= n) continue;
#pragma unroll
                for (int q = 0; q < KR; ++q)
                    if (q < j.n_req && rq[q].vmax_exact)
                        vmax[q] = fmaxf(vmax[q], cell_v<MT>(d[g], k, M, tf_lds, tf_lds + TableBase<MT, D>::of(q, toff[q]), rq[q], off[q]));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KR; ++q) {
        if (q < j.n_req && rq[q].vmax_exact) {
            const float v = wave_max_f(vmax[q]);
            if (lane == 0 && v > 0.0f) atomicMax(reinterpret_cast<unsigned int*>(rq[q].vmax_dev), __float_as_uint(v));
        }
    }
}

// Jobs that read values keep the requests' blocks as uploaded; jobs that read
// cached entries (tables of <= 256 entries) place table (request q, field m)
// at (q * MT + m) * 256 floats, so that every lookup address is the entry
// times 4 plus a compile-time offset.
// n LDS floats dst[i] = value(i), i < n, by the whole workgroup: each thread
// issues the loads of four of its elements before it stores any, so a round
// costs one memory latency instead of four (a load-store loop waits for each
// load alone)
template <typename F>
__device__ __forceinline__ void stage_lds(float* dst, int n, F value) {
    const int tid = thread_x(), nthr = block_dim_x();
    for (int i0 = tid; i0 < n; i0 += 4 * nthr) {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k * nthr < n ? value(i0 + k * nthr) : 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k * nthr < n) dst[i0 + k * nthr] = v[k];
    }
}

template <int MT, bool IDX>
__device__ __forceinline__ void load_job_tables(const BatchDev& b, const JobDev& j, int ji, int& loaded,
                                                float* tf_lds) {
    if (ji != loaded) {
        __syncthreads();
        if constexpr (IDX) {
            const int M = uni(fields_of<MT>(j.M)), nq = uni(j.n_req);
            const ReqDev* rq = b.reqs + uni(j.req0);
            stage_lds(tf_lds, nq * MT * kIdxTable, [&](int i) {
                const int q = i / (MT * kIdxTable), m = (i / kIdxTable) % MT, e = i % kIdxTable;
                float v = 0.0f;
                if (m < M && e < (int)rq[q].nmax[m] + 1) v = gload<float>(rq[q].tf, rq[q].tf_off[m] + e);
                return v;
            });
        } else {
            const float* src = j.tf_all;
            stage_lds(tf_lds, j.tf_total_all, [&](int i) { return gload<float>(src, i); });
        }
        __syncthreads();
        loaded = ji;
    }
}

// IDX: this instance serves the jobs that read cached entries (1) or values (0)
template <int MT, typename S, int KR, int IDX>
__global__ __launch_bounds__(kUpdThreads) void k_vmax_exact(BatchDev b) {
    extern __shared__ float tf_lds[];
    const int wv = uni((int)(thread_x() / kWave));
    int loaded = -1;
    for (int64_t u = block_x(); u < b.k1_units; u += grid_dim_x()) {
        const int ji = find_job_k1(b, u);
        const JobDev& j = b.jobs[ji];
        if ((j.idx[0] != nullptr) != (IDX != 0)) continue;
        load_job_tables<MT, IDX != 0>(b, j, ji, loaded, tf_lds);
        const int64_t r = uni((u - j.k1_unit0) * (kUpdThreads / kWave) + wv);
        if (r >= j.n_runs) continue;
        if constexpr (IDX != 0)
            vmax_run<MT, KR, StepIdx<MT>>(b, j, r, tf_lds);
        else
            vmax_run<MT, KR, StepData<MT, S>>(b, j, r, tf_lds);
    }
}

// ------------------------------------------------------------------ K1

// Error-free sum of two floats: s + e == a + b exactly (Knuth's TwoSum).
__device__ __forceinline__ void two_sum_f(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// A sum kept in the arithmetic of the scan mode: fp64 (d), compensated fp32
// (the unevaluated pair hi + lo) or plain fp32 (hi).  Used for the per-lane
// tile partials and the running sum of tile sums along a run; the mode is
// the same in every lane (a scalar branch).
struct ModeSum {
    double d;
    float hi, lo;
    __device__ void init() { d = 0.0; hi = 0.0f; lo = 0.0f; }
    __device__ double value(int mode) const {
        return mode == DVL_SCAN_FP64 ? d : (mode == DVL_SCAN_KAHAN_FP32 ? (double)hi + (double)lo : (double)hi);
    }
    __device__ void add_f(int mode, float x) {
        if (mode == DVL_SCAN_FP64) {
            d += (double)x;
        } else if (mode == DVL_SCAN_KAHAN_FP32) {
            float s, e;
            two_sum_f(hi, x, s, e);
            const float l = lo + e;
            hi = s + l;
            lo = l - (hi - s);
        } else {
            hi += x;
        }
    }
    // add another sum of the same mode
    __device__ void add(int mode, const ModeSum& o) {
        if (mode == DVL_SCAN_FP64) {
            d += o.d;
        } else if (mode == DVL_SCAN_KAHAN_FP32) {
            float s, e;
            two_sum_f(hi, o.hi, s, e);
            const float l = (lo + o.lo) + e;
            hi = s + l;
            lo = l - (hi - s);
        } else {
            hi += o.hi;
        }
    }
    // the same total in every lane (butterfly; each combine is symmetric in
    // its two operands, so every lane computes the same bits)
    __device__ void wave_total(int mode) {
        if (mode == DVL_SCAN_FP64) {
            d = wave_sum_d(d);
            return;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const int src = (lane_id() ^ o) << 2;
            ModeSum x;
            x.hi = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(hi)));
            x.lo = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(lo)));
            add(mode, x);
        }
    }
};

// One wave's run r of job j: stream its cells once (values, or cached
// entries), evaluate f for every request of the job, sum f over each tile
// (per lane, 4 cells per step as (f0 + f1) + (f2 + f3) in fp32, accumulated
// over the tile's steps and then over the wave in the request's scan
// arithmetic: fp64, compensated fp32 or plain fp32) and record, per request
// and tile, the non-decreasing sum of the earlier tiles of the run.  Both
// sources give the same f bit for bit.
template <int MT, int KR, typename D, bool P1>
__device__ __forceinline__ void tile_sums_run(const BatchDev& b, const JobDev& j, int64_t r, const float* tf_lds) {
    constexpr int G = Group<D>::n;
    const int lane = lane_id();
    const int M = uni(fields_of<MT>(j.M));
    const int nreq = KR == 1 ? 1 : uni(j.n_req);
    const ReqDev* rq = b.reqs + uni(j.req0);
    const int tile_steps = uni(j.tile_steps);
    const int64_t n = uni(j.n);
    const int64_t tile_cells = (int64_t)tile_steps * kStepCells;
    const int64_t t_begin = r * uni(j.tiles_per_run);
    const int64_t t_end = min(uni(j.n_tiles), t_begin + uni(j.tiles_per_run));
    const int64_t c_begin = t_begin * tile_cells;
    const int64_t c_end = min(n, t_end * tile_cells);
    const int nsteps = (int)((c_end - c_begin + kStepCells - 1) / kStepCells);

    ImpCtx ctx[KR];
    ModeSum run[KR], tacc[KR];
    double prev[KR];
    int toff[KR], off[KR][MT], mode[KR];
    float* fst[KR];                   // where f of every cell is kept for the projection, or NULL
    double* lpre[KR];                 // the requests' in-run tile prefixes
    // every descriptor field the loop reads is held in registers: a load
    // inside the loop would be the youngest in flight, and waiting for it
    // would drain the prefetched steps
#pragma unroll
    for (int q = 0; q < KR; ++q) {
        fst[q] = nullptr;
        lpre[q] = nullptr;
        mode[q] = DVL_SCAN_FP64;
        if (q < nreq) {
            ctx[q] = make_ctx(rq[q]);
            toff[q] = uni(rq[q].tf_job_off);
            table_offsets<MT>(rq[q], M, off[q]);
            fst[q] = uni(rq[q].ws.fstore);
            lpre[q] = uni(rq[q].ws.local_prefix);
            mode[q] = uni(rq[q].scan_mode);
        }
        run[q].init();
        prev[q] = 0.0;
        tacc[q].init();
    }
    int64_t t = t_begin;
    int in_tile = 0;
    const RunView<MT> view = run_view<MT, D>(j, M, c_begin);
    const int last_group = (nsteps - 1) / G * G;

    // the steps s .. s + G - 1 of the run, loaded into `cur`
    auto process = [&](const D (&cur)[G], int s) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (s + g >= nsteps) break;
            const int64_t quad = ((c_begin + (int64_t)(s + g) * kStepCells) >> 2) + lane;
            const bool full = c_begin + (int64_t)(s + g + 1) * kStepCells <= n;   // no cell past the end
#pragma unroll
            for (int q = 0; q < KR; ++q) {
                if (q < nreq) {
                    float f[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float v = cell_v<MT>(cur[g], k, M, tf_lds, tf_lds + TableBase<MT, D>::of(q, toff[q]), rq[q], off[q]);
                        const uint32_t L = cur[g].lv.get(k);
                        f[k] = P1 ? importance_p1(v, L, ctx[q]) : importance_from_v(v, L, ctx[q]);
                    }
                    if (!full) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) f[k] = ((quad << 2) + k < n) ? f[k] : 0.0f;
                    }
                    if (fst[q]) {
                        f32x4 fv;
                        fv.x = f[0];
                        fv.y = f[1];
                        fv.z = f[2];
                        fv.w = f[3];
                        gstore<f32x4>(fst[q], quad, fv);
                    }
                    tacc[q].add_f(mode[q], (f[0] + f[1]) + (f[2] + f[3]));
                }
            }
            if (++in_tile == tile_steps || s + g + 1 == nsteps) {
#pragma unroll
                for (int q = 0; q < KR; ++q) {
                    if (q < nreq) {
                        tacc[q].wave_total(mode[q]);
                        prev[q] = fmax(prev[q], run[q].value(mode[q]));
                        if (lane == 0) gstore<double>(lpre[q], t, prev[q]);
                        run[q].add(mode[q], tacc[q]);
                        tacc[q].init();
                    }
                }
                ++t;
                in_tile = 0;
            }
        }
    };

    // Two groups in flight, in buffers A and B that take turns: a buffer is
    // loaded again (unconditionally; past the run's end the last step is
    // reloaded) right after its group was used, so no loaded value is ever
    // moved and every wait is for the older of the two groups only.  The
    // level codes a reload needs were fetched before the buffer's previous
    // load, so they have arrived.
    D A[G], B[G];
    StepCodes<G> cA, cB;
    {
        const StepCodes<G> c0 = load_codes<G>(view.lcode, 0);
        const StepCodes<G> c1 = load_codes<G>(view.lcode, min(G, last_group));
        cA = load_codes<G>(view.lcode, min(2 * G, last_group));
#pragma unroll
        for (int g = 0; g < G; ++g) A[g].load(view, M, g, c0.c[g]);
        cB = load_codes<G>(view.lcode, min(3 * G, last_group));
#pragma unroll
        for (int g = 0; g < G; ++g) B[g].load(view, M, min(G + g, nsteps - 1), c1.c[g]);
    }
    for (int s = 0; s < nsteps; s += 2 * G) {
        process(A, s);
        {
            const StepCodes<G> c2 = load_codes<G>(view.lcode, min(s + 4 * G, last_group));
#pragma unroll
            for (int g = 0; g < G; ++g) A[g].load(view, M, min(s + 2 * G + g, nsteps - 1), cA.c[g]);
            cA = c2;
        }
        if (s + G >= nsteps) break;
        process(B, s + G);
        {
            const StepCodes<G> c3 = load_codes<G>(view.lcode, min(s + 5 * G, last_group));
#pragma unroll
            for (int g = 0; g < G; ++g) B[g].load(view, M, min(s + 3 * G + g, nsteps - 1), cB.c[g]);
            cB = c3;
        }
    }
#pragma unroll
    for (int q = 0; q < KR; ++q)
        if (q < nreq && lane == 0) gstore<double>(rq[q].ws.run_total, r, fmax(prev[q], run[q].value(mode[q])));
}

// A workgroup takes 4 consecutive runs of one job; wave r of the job owns the
// tiles [r k, (r + 1) k).
template <int MT, typename S, int KR, int IDX>
#ifdef DVL_K1_WAVES_PER_EU
#define DVL_K1_OCCUPANCY __attribute__((amdgpu_waves_per_eu(DVL_K1_WAVES_PER_EU)))
#else
#define DVL_K1_OCCUPANCY
#endif
__global__ __launch_bounds__(kUpdThreads) DVL_K1_OCCUPANCY void k_tile_sums(BatchDev b) {
    extern __shared__ float tf_lds[];
    const int wv = uni((int)(thread_x() / kWave));
    int loaded = -1;
    for (int64_t u = block_x(); u < b.k1_units; u += grid_dim_x()) {
        const int ji = find_job_k1(b, u);
        const JobDev& j = b.jobs[ji];
        if ((j.idx[0] != nullptr) != (IDX != 0)) continue;
        load_job_tables<MT, IDX != 0>(b, j, ji, loaded, tf_lds);
        const int64_t r = uni((u - j.k1_unit0) * (kUpdThreads / kWave) + wv);
        if (r >= j.n_runs) continue;
        // P = 1 with the importance clamp in every request of the job: no pow
        bool p1 = true;
        for (int q = 0; q < (KR == 1 ? 1 : j.n_req); ++q) {
            const ReqDev& rq = b.reqs[j.req0 + q];
            p1 = p1 && rq.exp_is_one && rq.clamp_mode == 0;
        }
        p1 = uni((int)p1) != 0;
        if constexpr (IDX != 0) {
            if (p1)
                tile_sums_run<MT, KR, StepIdx<MT>, true>(b, j, r, tf_lds);
            else
                tile_sums_run<MT, KR, StepIdx<MT>, false>(b, j, r, tf_lds);
        } else {
            if (p1)
                tile_sums_run<MT, KR, StepData<MT, S>, true>(b, j, r, tf_lds);
            else
                tile_sums_run<MT, KR, StepData<MT, S>, false>(b, j, r, tf_lds);
        }
    }
}

// ------------------------------------------------------------------ K3 helpers

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ o) << 2, (int)v));
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1)
        v = max(v, (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ o) << 2, (int)v));
    return v;
}
__device__ __forceinline__ int wave_min_i32(int v) {
    for (int o = 32; o > 0; o >>= 1)
        v = min(v, __builtin_amdgcn_ds_bpermute((lane_id() ^ o) << 2, v));
    return v;
}

// Sum of the importance of all tiles before tile t (t = T gives F_tot): the
// run's base plus the tile's prefix inside its run, never above the next
// run's base.  One definition serves both neighbours of every tile boundary,
// and the offsets never decrease.
__device__ __forceinline__ double tile_offset(const JobDev& j, const UpdWorkspace& ws, int64_t t,
                                              bool degenerate) {
    const int64_t tile_cells = (int64_t)j.tile_steps * kStepCells;
    if (degenerate) return t >= j.n_tiles ? (double)j.n : (double)(t * tile_cells);
    if (t >= j.n_tiles) return gload<double>(ws.run_base, j.n_runs);
    const int64_t r = t / j.tiles_per_run;
    const double lo = gload<double>(ws.run_base, r), hi = gload<double>(ws.run_base, r + 1);
    return fmin(fmax(lo + gload<double>(ws.local_prefix, t), lo), hi);
}

// Cell range [first, last] of bin `key` found in tile t: a bin that starts
// and ends inside the tile (dest 0) is stored as the request's output; the
// tile's first bin (dest 1) and last bin (dest 2) go to the tile's head and
// tail records, merged across tiles by K4.  Called by the whole wave.
__device__ __forceinline__ void close_bin(const ReqDev& q, int64_t T, int dest, int64_t t, int key,
                                          uint32_t first, uint32_t last) {
    if (lane_id() != 0) return;
    if (dest == 0) {
        gstore<uint32_t>(q.first_cell, key, first);
        gstore<uint32_t>(q.last_cell, key, last);
    } else {
        gstore<uint32_t>(q.ws.rec_first, (dest - 1) * T + t, first);
        gstore<uint32_t>(q.ws.rec_last, (dest - 1) * T + t, last);
    }
}

// ------------------------------------------------------------------ K3

constexpr int kBinThreads = 192;  // one workgroup of three waves per queued (request, tile)

// Pixel interval [X0, X1] of tile t of request q, and its first and last bin.
struct TileSpan {
    double scale_d;
    float scale_f, X0, X1;
    int b0, b1;
};

__device__ __forceinline__ TileSpan tile_span(const ReqDev& q, const JobDev& j, int64_t t) {
    TileSpan sp;
    const bool degenerate = gload<double>(q.ws.scal, 1) != 0.0;
    sp.scale_d = (double)q.W / gload<double>(q.ws.scal, 0);
    sp.scale_f = (float)sp.scale_d;
    sp.X0 = (float)(tile_offset(j, q.ws, t, degenerate) * sp.scale_d);
    sp.X1 = (float)(tile_offset(j, q.ws, t + 1, degenerate) * sp.scale_d);
    const int W1 = q.W - 1;
    sp.b0 = max(0, min((int)floorf(sp.X0), W1));
    sp.b1 = max(0, min((int)floorf(sp.X1), W1));
    return sp;
}

// V of cell k of this lane (request q, tables in the request's block layout)
template <int MT, typename S>
__device__ __forceinline__ float rescan_v(const StepData<MT, S>& d, int k, int M, const float* tf,
                                          const ReqDev& q, const int (&off)[MT]) {
    float xk[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) xk[m] = m < M ? d.q[m].get(k) : 0.0f;
    return variation<MT>(xk, M, tf, q);
}
template <int MT>
__device__ __forceinline__ float rescan_v(const StepIdx<MT>& d, int k, int M, const float* tf, const ReqDev& q,
                                          const int (&off)[MT]) {
    float amax = -INFINITY, amin = INFINITY;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const float al = tf[off[m] + (int)((d.e[m] >> (8 * k)) & 0xFFu)];
            amax = fmaxf(amax, al);
            amin = fminf(amin, al);
        }
    }
    return amax - amin;
}

// The in-step prefix of one 256-cell step, per lane (4 cells): the wave's
// exclusive prefix before the lane (Bex), the lane's own partial sums p1..p3
// and the inclusive prefix B through the lane (running maximum: never
// decreasing).
struct StepPrefix {
    f32x4 ex_p;   // Bex, p1, p2, p3
    float B;
};

// LDS of the staged prefixes of one tile: [steps][64] (Bex, p1, p2, p3).
// B is not stored: B of a lane is Bex of the next lane, and B of the last
// lane (the step total) is kept in the Bex slot of lane 0, whose Bex is 0 by
// definition.  16 bytes per lane and step.
struct Stage {
    f32x4* ex_p;
    __device__ void put(int s, const StepPrefix& p) {
        f32x4 v = p.ex_p;
        const float total = readlane(p.B, kWave - 1);
        if (lane_id() == 0) v.x = total;
        ex_p[s * kWave + lane_id()] = v;
    }
    __device__ StepPrefix get(int s) const {
        StepPrefix p;
        p.ex_p = ex_p[s * kWave + lane_id()];
        p.B = __int_as_float(
            __builtin_amdgcn_ds_bpermute(((lane_id() + 1) & (kWave - 1)) << 2, __float_as_int(p.ex_p.x)));
        if (lane_id() == 0) p.ex_p.x = 0.0f;
        return p;
    }
};

constexpr int kBinWaves = kBinThreads / kWave;
constexpr int kMaxTileSteps = 32;
constexpr size_t kStageBytesPerStep = (size_t)kWave * sizeof(f32x4);

// Phase 1 of the rescan, for the steps s = w, w + kBinWaves, ... of tile t
// taken by wave w: f of every cell again (from values, cached entries or the
// stored f, bit for bit as in K1; 1 when the total importance is 0) and the
// step's monotone prefix, into LDS.
template <int MT, typename S, typename D>
__device__ __forceinline__ void rescan_stage(const ReqDev& q, const JobDev& j, int64_t t, const float* tf_lds,
                                             Stage stage) {
    const int lane = lane_id();
    const int w = uni((int)(thread_x() / kWave));
    const int M = uni(fields_of<MT>(j.M));
    const int64_t n = uni(j.n);
    const bool degenerate = uni((int)(gload<double>(q.ws.scal, 1) != 0.0)) != 0;
    const int tile_steps = uni(j.tile_steps);
    const int64_t tbase = t * (int64_t)tile_steps * kStepCells;
    const int nsteps = (int)((min(tbase + (int64_t)tile_steps * kStepCells, n) - tbase + kStepCells - 1) / kStepCells);
    RunView<MT> view;
    if constexpr (std::is_same<D, StepF<MT>>::value) {
        view = run_view<MT, StepData<MT, S>>(j, M, tbase);
        view.base[0] = reinterpret_cast<const char*>(uni(q.ws.fstore)) + tbase * 4;
    } else {
        view = run_view<MT, D>(j, M, tbase);
    }
    const ImpCtx c = make_ctx(q);
    int off[MT];
    table_offsets<MT>(q, M, off);
    if (w >= nsteps) return;
    auto process = [&](const D& cur, int s) {
        const int64_t quad = ((tbase + (int64_t)s * kStepCells) >> 2) + lane;
        float f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float fk = 1.0f;
            if constexpr (std::is_same<D, StepF<MT>>::value) {
                if (!degenerate) fk = k == 0 ? cur.fv.x : (k == 1 ? cur.fv.y : (k == 2 ? cur.fv.z : cur.fv.w));
            } else {
                if (!degenerate) fk = importance_from_v(rescan_v<MT>(cur, k, M, tf_lds, q, off), cur.lv.get(k), c);
            }
            f[k] = ((quad << 2) + k < n) ? fk : 0.0f;
        }
        // monotone in-tile prefix: lane-serial over 4 cells, wave sum scan,
        // running max to undo rounding steps back
        const float p1 = f[0], p2 = p1 + f[1], p3 = p2 + f[2], tl = p3 + f[3];
        const float B = wave_incl_max(wave_incl_sum(tl));
        StepPrefix sp;
        sp.ex_p.x = shfl_up1(B, 0.0f);
        sp.ex_p.y = p1;
        sp.ex_p.z = p2;
        sp.ex_p.w = p3;
        sp.B = B;
        stage.put(s, sp);
    };
    if constexpr (!std::is_same<D, StepData<MT, S>>::value) {
        // cached entries or stored f (a few registers per step): the level
        // codes of all of this wave's steps first (uniform: scalar registers;
        // a lane's level load address depends on its code), then the steps
        // two at a time, loaded together and then processed (two keep the
        // rescan within 64 VGPRs, eight waves per SIMD)
        constexpr int kAhead = 2;
        constexpr int kMaxPer = (kMaxTileSteps + kBinWaves - 1) / kBinWaves;
        const int cnt = (nsteps - w + kBinWaves - 1) / kBinWaves;
        uint32_t code[kMaxPer];
#pragma unroll
        for (int k = 0; k < kMaxPer; ++k) {
            code[k] = 0u;
            if constexpr (std::is_same<D, StepIdx<MT>>::value)
                if (k < cnt) code[k] = uni(gload<uint32_t>(view.lcode, w + k * kBinWaves));
        }
#pragma unroll
        for (int k0 = 0; k0 < kMaxPer; k0 += kAhead) {
            if (k0 >= cnt) break;
            D buf[kAhead];
#pragma unroll
            for (int k = 0; k < kAhead; ++k)
                if (k0 + k < cnt) buf[k].load(view, M, w + (k0 + k) * kBinWaves, code[k0 + k]);
#pragma unroll
            for (int k = 0; k < kAhead; ++k)
                if (k0 + k < cnt) process(buf[k], w + (k0 + k) * kBinWaves);
        }
    } else {
        // values: two steps in flight in buffers that take turns (no loaded
        // register is copied, so each wait is for the older step only)
        D A, B;
        A.load(view, M, w, gload<uint32_t>(view.lcode, w));
        const int s1 = min(w + kBinWaves, nsteps - 1);
        B.load(view, M, s1, gload<uint32_t>(view.lcode, s1));
        for (int s = w; s < nsteps; s += 2 * kBinWaves) {
            process(A, s);
            const int s2 = min(s + 2 * kBinWaves, nsteps - 1);
            A.load(view, M, s2, gload<uint32_t>(view.lcode, s2));
            if (s + kBinWaves >= nsteps) break;
            process(B, s + kBinWaves);
            const int s3 = min(s + 3 * kBinWaves, nsteps - 1);
            B.load(view, M, s3, gload<uint32_t>(view.lcode, s3));
        }
    }
}

// Phase 2, by one wave: the cells' pixel intervals and bins from the staged
// prefixes, step after step (the running base of a step is the fp32 sum of
// the earlier steps' totals, in order).  Each bin's cell range is closed as
// soon as it is known: bins inside the tile are written as outputs, the
// tile's first and last bin as its head and tail records.
__device__ __forceinline__ void rescan_walk(const ReqDev& q, const JobDev& j, int64_t t, const Stage stage) {
    const int lane = lane_id();
    const int64_t T = uni(j.n_tiles);
    const int64_t n = uni(j.n);
    const TileSpan sp = tile_span(q, j, t);
    const float scale_f = uni(sp.scale_f), X0 = uni(sp.X0), X1 = uni(sp.X1);
    const int W1 = uni(q.W) - 1;
    const int tile_steps = uni(j.tile_steps);
    const int64_t tile_cells = (int64_t)tile_steps * kStepCells;
    const int64_t tbase = t * tile_cells;
    const int64_t tend = min(tbase + tile_cells, n);
    const uint32_t last_valid = (uint32_t)(tend - 1);
    const int nsteps = (int)((tend - tbase + kStepCells - 1) / kStepCells);

    // The per-step quantities of the sequential walk, for every step at once
    // (lane s: step s): the running base (the fp32 sum of the earlier steps'
    // totals, added in step order as the walk would), the bins of the step's
    // first and last cell, and whether it lies inside one bin.  Lanes past
    // the last step repeat it.
    float run_v = 0.0f;
    int key0_v, key_end_v, fast_v = 0;
    {
        const int ls = min(lane, nsteps - 1);
        for (int k = 0; k < nsteps; ++k) {
            const float st_k = stage.ex_p[k * kWave].x;   // step k's total (lane 0's Bex slot)
            if (k < ls) run_v = run_v + st_k;
        }
        const int64_t c0 = tbase + (int64_t)ls * kStepCells;
        const float B63 = stage.ex_p[ls * kWave].x;       // the step total: B of lane 63
        const float B0 = stage.ex_p[ls * kWave + 1].x;    // B of lane 0: Bex of lane 1
        const f32x4 e63 = stage.ex_p[ls * kWave + kWave - 1];
        const float x_first = fminf(fmaf(run_v + fminf(0.0f, B0), scale_f, X0), X1);
        key0_v = max(0, min((int)floorf(x_first), W1));
        key_end_v = INT_MAX;
        if (c0 + kStepCells <= n) {
            const float x3 = fminf(fmaf(run_v + fminf(e63.x + e63.w, B63), scale_f, X0), X1);
            const float x4 = (uint32_t)(c0 + kStepCells - 1) == last_valid ? X1
                                                                          : fminf(fmaf(run_v + B63, scale_f, X0), X1);
            const int lo3 = max(0, min((int)floorf(x3), W1));
            key_end_v = max(lo3, min((int)ceilf(x4) - 1, W1));
            fast_v = key0_v == key_end_v;
        }
    }

    bool o_valid = false;
    int O = -1, Bh = -1;
    uint32_t O_first = 0;

    for (int s = 0; s < nsteps; ++s) {
        const int64_t c0 = tbase + (int64_t)s * kStepCells;
        const int key0 = readlane(key0_v, s);
        if (s == 0) Bh = key0;
        if (readlane(fast_v, s) && (!o_valid || key0 == O)) {
            // the whole step lies in the open bin
            if (!o_valid) {
                o_valid = true;
                O = key0;
                O_first = (uint32_t)c0;
            }
            continue;
        }
        const int key_end = readlane(key_end_v, s);
        const float run = readlane(run_v, s);
        const int64_t quad = (c0 >> 2) + lane;
        const StepPrefix pr = stage.get(s);
        const float Bex = pr.ex_p.x, p1 = pr.ex_p.y, p2 = pr.ex_p.z, p3 = pr.ex_p.w, B = pr.B;
        const bool full = c0 + kStepCells <= n;

        uint32_t g[4];
        bool valid[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            g[k] = (uint32_t)((quad << 2) + k);
            valid[k] = (int64_t)g[k] < n;
        }
        float xs[5];
        xs[0] = fminf(fmaf(run + fminf(Bex, B), scale_f, X0), X1);
        xs[1] = fminf(fmaf(run + fminf(Bex + p1, B), scale_f, X0), X1);
        xs[2] = fminf(fmaf(run + fminf(Bex + p2, B), scale_f, X0), X1);
        xs[3] = fminf(fmaf(run + fminf(Bex + p3, B), scale_f, X0), X1);
        xs[4] = fminf(fmaf(run + B, scale_f, X0), X1);

        // pixel bins of each cell: [floor(x1), ceil(x2) - 1], clamped
        int blo[4], bhi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float en = (g[k] == last_valid) ? X1 : xs[k + 1];
            blo[k] = max(0, min((int)floorf(xs[k]), W1));
            bhi[k] = max(blo[k], min((int)ceilf(en) - 1, W1));
        }

        // ---- bin boundary inside the step ----
        const int last_lane = full ? kWave - 1 : (int)((n - 1 - c0) >> 2);
        const int kl = (int)((n - 1 - c0) & 3);
        const int bhi_last = kl == 0 ? bhi[0] : (kl == 1 ? bhi[1] : (kl == 2 ? bhi[2] : bhi[3]));
        const int key_last = full ? key_end : readlane(bhi_last, last_lane);
        // (1) the open bin ended with the previous step
        if (o_valid && key0 != O) {
            close_bin(q, T, O == Bh ? 1 : 0, t, O, O_first, (uint32_t)(c0 - 1));
            o_valid = false;
        }
        // (2) bins strictly inside a wide cell hold that cell alone
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (valid[k] && bhi[k] > blo[k] + 1)
                for (int bb = blo[k] + 1; bb < bhi[k]; ++bb) {
                    gstore<uint32_t>(q.first_cell, bb, g[k]);
                    gstore<uint32_t>(q.last_cell, bb, g[k]);
                }
        // (3) every bin that is the first or last bin of some cell of this
        //     step, in increasing order; all but the step's last one close
        int b = key0;
        while (true) {
            uint32_t gmin = 0xFFFFFFFFu, gmax = 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (valid[k] && (blo[k] == b || bhi[k] == b)) {
                    gmin = min(gmin, g[k]);
                    gmax = max(gmax, g[k]);
                }
            }
            const uint32_t bfirst = (o_valid && b == O) ? O_first : wave_min_u32(gmin);
            if (b == key_last) {
                // stays open into the next step
                O = b;
                O_first = bfirst;
                o_valid = true;
                break;
            }
            close_bin(q, T, b == Bh ? 1 : 0, t, b, bfirst, wave_max_u32(gmax));
            o_valid = false;
            int nk = INT_MAX;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (valid[k]) {
                    if (blo[k] > b) nk = min(nk, blo[k]);
                    if (bhi[k] > b) nk = min(nk, bhi[k]);
                }
            }
            b = wave_min_i32(nk);
            if (b == INT_MAX) break;   // cannot happen: key_last is above
        }
    }

    // tile end: the open bin is the tile's last bin
    if (o_valid) {
        close_bin(q, T, O == Bh ? 1 : 2, t, O, O_first, last_valid);
        if (lane == 0) {
            gstore<int32_t>(q.ws.head_bin, t, Bh);
            gstore<int32_t>(q.ws.tail_bin, t, O);
        }
    }
}

// K3b: the queued tiles, one workgroup each.  Its waves stage the prefixes
// of the tile's steps in LDS together (phase 1; the loads of three waves in
// flight instead of one), then the first wave walks the bins (phase 2).
// Three waves, not four: at 62 VGPRs a compute unit holds seven waves per
// SIMD, so seven workgroups of four waves (1792 on the chip) would leave some
// of the ~1900 tiles of W = 1920 to a second round, while eight workgroups of
// three fit (LDS: 20 KB each); measured 36 instead of 41 us.
// IDX: this instance serves the requests whose projection reads values (0),
// cached entries (1) or the f the importance pass stored (2); each skips the
// others' tiles.  LDS: the request's tables, then the staged prefixes.
template <int MT, typename S, int IDX>
__global__ __launch_bounds__(kBinThreads) void k_bin(BatchDev bd) {
    extern __shared__ float tf_lds[];
    int loaded = -1;
    const int64_t n_queued = gload<uint32_t>(bd.rescan_count, IDX);
    const uint64_t* queue = bd.rescan_queue + IDX * bd.k3_units;
    Stage stage;
    stage.ex_p = reinterpret_cast<f32x4*>(tf_lds + ((bd.max_req_tf + 3) & ~3));

    for (int64_t i = block_x(); i < n_queued; i += grid_dim_x()) {
        const int64_t u = uni((int64_t)gload<uint64_t>(queue, i));
        const int qi = uni(find_req_k3(bd, u));
        const ReqDev& q = bd.reqs[qi];
        const JobDev& j = bd.jobs[uni(q.job)];
        const int64_t t = u - uni(q.k3_unit0);
        // the tile is rescanned: this request's tables in LDS
        if (qi != loaded) {
            const float* src = q.tf;
            stage_lds(tf_lds, q.tf_total, [&](int k) { return gload<float>(src, k); });
            loaded = qi;
        }
        __syncthreads();
        if constexpr (IDX == 2)
            rescan_stage<MT, S, StepF<MT>>(q, j, t, tf_lds, stage);
        else if constexpr (IDX == 1)
            rescan_stage<MT, S, StepIdx<MT>>(q, j, t, tf_lds, stage);
        else
            rescan_stage<MT, S, StepData<MT, S>>(q, j, t, tf_lds, stage);
        __syncthreads();
        if (thread_x() < kWave) rescan_walk(q, j, t, stage);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ K4

// Field statistics of the sorted cells [first, last], by one wave: the stored
// values of the partial 256-cell steps at the two ends, the per-step
// statistics of the whole steps next to them and the per-tile statistics of
// the whole tiles in between (a step or tile is whole when the range holds
// all of its cells below n).  Sums are fp64; every lane ends with the result.
template <int MT, typename S>
__device__ __forceinline__ void bin_range_stats(const JobDev& j, int M, uint32_t first, uint32_t last,
                                                double (&sum)[MT], float (&mn)[MT], float (&mx)[MT]) {
    const int lane = lane_id();
    const int64_t n = uni(j.n);
    const int ts = uni(j.tile_steps);
    const int64_t T = uni(j.n_tiles);
    const int64_t S_all = T * ts;
    const int64_t f = first, l = last;
    auto whole_step = [&](int64_t st) { return f <= st * kStepCells && l >= min(n, st * kStepCells + kStepCells) - 1; };
    const int64_t sf = f / kStepCells, sl = l / kStepCells;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        sum[m] = 0.0;
        mn[m] = INFINITY;
        mx[m] = -INFINITY;
    }
    // partial end steps: each lane its 4 cells
    const bool wf = whole_step(sf), wl = whole_step(sl);
#pragma unroll
    for (int end = 0; end < 2; ++end) {
        if (end == 0 && wf) continue;
        if (end == 1 && (sl == sf || wl)) break;
        const int64_t st = end == 0 ? sf : sl;
        const int64_t c = st * kStepCells + 4 * lane;
        const bool need = c + 3 >= f && c <= l;     // lanes with no cell of the range fetch nothing
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (m < M && need) {
                Quad<S> qd;
                qd.load(j.fields[m], st * kWave + lane);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (c + k >= f && c + k <= l) {
                        const float v = qd.get(k);
                        sum[m] += (double)v;
                        mn[m] = fminf(mn[m], v);
                        mx[m] = fmaxf(mx[m], v);
                    }
                }
            }
        }
    }
    // whole steps [a, b]; whole tiles [ta, tb] among them
    const int64_t a = wf ? sf : sf + 1, b = wl ? sl : sl - 1;
    if (a <= b) {
        const int64_t ta = (a + ts - 1) / ts, tb = (b + 1) / ts - 1;
        int64_t s0 = a, s1 = b, s2 = 1, s3 = 0;       // step ranges [s0, s1] and [s2, s3] outside whole tiles
        if (ta <= tb) {
            s1 = ta * ts - 1;
            s2 = (tb + 1) * ts;
            s3 = b;
            for (int64_t t = ta + lane; t <= tb; t += kWave) {
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if (m < M) {
                        const int64_t o = (int64_t)m * T + t;
                        sum[m] += gload<double>(j.agg_sum, o);
                        mn[m] = fminf(mn[m], gload<float>(j.agg_min, o));
                        mx[m] = fmaxf(mx[m], gload<float>(j.agg_max, o));
                    }
                }
            }
        }
        const int64_t n0 = s1 >= s0 ? s1 - s0 + 1 : 0, n1 = s3 >= s2 ? s3 - s2 + 1 : 0;
        for (int64_t i = lane; i < n0 + n1; i += kWave) {
            const int64_t st = i < n0 ? s0 + i : s2 + (i - n0);
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (m < M) {
                    const int64_t o = (int64_t)m * S_all + st;
                    sum[m] += gload<double>(j.step_sum, o);
                    mn[m] = fminf(mn[m], gload<float>(j.step_min, o));
                    mx[m] = fmaxf(mx[m], gload<float>(j.step_max, o));
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            sum[m] = wave_sum_d(sum[m]);
            mn[m] = wave_min_f(mn[m]);
            mx[m] = wave_max_f(mx[m]);
        }
    }
}

// K4: one wave per (request, bin).  The bin's cell range: written by the
// rescan when the bin starts and ends inside one rescanned tile; else the
// smallest first and largest last cell over the records of the tiles it
// touches (a tile inside one bin is that bin's record whole, a rescanned
// tile holds records of its first and last bin).  Then the statistics of the
// range and the height of the mean.
template <int MT, typename S>
__global__ __launch_bounds__(256) void k_bin_stats(BatchDev bd) {
    const int lane = lane_id();
    const int64_t u = (int64_t)block_x() * (256 / kWave) + thread_x() / kWave;
    if (u >= bd.k4_units) return;   // the whole wave
    const int qi = uni(find_req_k4(bd, u));
    const ReqDev& q = bd.reqs[qi];
    const JobDev& j = bd.jobs[uni(q.job)];
    const int M = uni(fields_of<MT>(j.M));
    const int b = (int)(u - uni(q.k4_unit0));
    if (b == 0 && lane == 0) {
        gstore<double>(q.f_total, 0, gload<double>(q.ws.scal, 0));
        gstore<float>(q.vmax_used, 0, gload<float>(q.vmax_dev, 0));
    }
    const int64_t T = uni(j.n_tiles);
    const int32_t* hb = q.ws.head_bin;
    const int32_t* tb = q.ws.tail_bin;
    // tiles touching bin b: t0 = first with tail >= b, t1 = last with head <= b
    // (K3a wrote both per bin; t0 is its candidate ta or the next tile)
    const int64_t t1 = uni(gload<int32_t>(q.ws.bin_t1, b));
    const int64_t ta = uni(gload<int32_t>(q.ws.bin_ta, b));
    // then one round of loads: the candidate's tail bin, the last tile's head
    // and tail bins, the bin's own outputs (written by the rescan when the
    // bin starts and ends inside one tile) and, per lane, the head and tail
    // bins and both records of the tiles [ta, t1].  When t0 = ta + 1, tile
    // ta's bins are all below b and it adds nothing.
    const int ea = gload<int32_t>(tb, ta);
    const int h1 = gload<int32_t>(hb, t1), e1 = gload<int32_t>(tb, t1);
    const uint32_t in_first = gload<uint32_t>(q.first_cell, b), in_last = gload<uint32_t>(q.last_cell, b);
    uint32_t first = 0xFFFFFFFFu, last = 0u;
    for (int64_t t = ta + lane; t <= t1; t += kWave) {
        const int h = gload<int32_t>(hb, t), e = gload<int32_t>(tb, t);
        const uint32_t f0 = gload<uint32_t>(q.ws.rec_first, t), l0 = gload<uint32_t>(q.ws.rec_last, t);
        const uint32_t f1 = gload<uint32_t>(q.ws.rec_first, T + t), l1 = gload<uint32_t>(q.ws.rec_last, T + t);
        if (h == b) {
            first = min(first, f0);
            last = max(last, l0);
        } else if (e == b) {
            first = min(first, f1);
            last = max(last, l1);
        }
    }
    const int64_t t0 = (ea >= b || ta + 1 >= T) ? ta : ta + 1;
    const bool inside = t0 == t1 && h1 < b && b < e1;
    if (inside) {
        first = in_first;
        last = in_last;
    } else {
        first = wave_min_u32(first);
        last = wave_max_u32(last);
    }
    // no cell (cannot happen with a positive total width); a range outside
    // the volume is treated the same way, so no statistic reads past it
    if (first == 0xFFFFFFFFu || first > last || (int64_t)last >= uni(j.n)) {
        if (lane == 0) {
            gstore<uint32_t>(q.first_cell, b, 0xFFFFFFFFu);
            gstore<uint32_t>(q.last_cell, b, 0xFFFFFFFEu);
        }
        if (lane < M) {
            const int64_t o = (int64_t)lane * q.W + b;
            gstore<float>(q.mean, o, 0.0f);
            gstore<float>(q.vmin, o, INFINITY);
            gstore<float>(q.vmax, o, -INFINITY);
            gstore<float>(q.y, o, 0.0f);
        }
        return;
    }
    double sm[MT];
    float mn[MT], mx[MT];
    bin_range_stats<MT, S>(j, M, first, last, sm, mn, mx);
    if (lane == 0 && !inside) {
        gstore<uint32_t>(q.first_cell, b, first);
        gstore<uint32_t>(q.last_cell, b, last);
    }
    const uint32_t cnt = last - first + 1u;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M && lane == m) {
            const float mean = (float)(sm[m] / (double)cnt);
            const int e = tf_entry(mean, q.s[m], q.b[m], q.nmax[m]);
            const int64_t o = (int64_t)m * q.W + b;
            gstore<float>(q.mean, o, mean);
            gstore<float>(q.vmin, o, mn[m]);
            gstore<float>(q.vmax, o, mx[m]);
            gstore<float>(q.y, o, gload<float>(q.tf, q.tf_off[m] + e));
        }
    }
}

// ------------------------------------------------------------------ launcher

// launchers of the kernels that do not depend on the storage type (update.hip)
dvl_status launch_carry_classify(const BatchDev& b, hipStream_t s);

// The cached-entry importance kernels address their tables from LDS address
// 0 (the start of the dynamic LDS array): they must hold no static LDS.
template <void (*Kernel)(BatchDev)>
static dvl_status check_no_static_lds(const char* name) {
    static int checked = 0;   // one flag per kernel instance
    if (checked == 1) return DVL_OK;
    hipFuncAttributes fa;
    DVL_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(Kernel)));
    if (fa.sharedSizeBytes != 0) {
        set_error("%s holds %zu bytes of static LDS; its table addressing needs none", name, (size_t)fa.sharedSizeBytes);
        return DVL_E_HIP;
    }
    checked = 1;
    return DVL_OK;
}

// Grid of the importance pass.  When the units split evenly over the
// workgroups that fit the chip at once with `lds` bytes of LDS each (or
// number no more than them), or belong to several volumes (units of unequal
// length: the 32-volume batch's pass took 612 instead of 735 us), one round
// of that many: a workgroup that finishes its unit takes the next one with
// its tables already in LDS, instead of a second round of workgroups
// starting cold (descriptors,
// tables, the first loads: a few dependent memory round trips each), 5 %
// faster for the 501 M-cell cached-entry pass.  Otherwise 8 workgroups per
// compute unit, whose later rounds the hardware hands to whichever compute
// unit frees a slot (a fixed uneven split, 2048 units over 1280 resident
// workgroups of the value path, was 3 % slower).  The occupancy is queried
// once per kernel and LDS size; any grid gives the same results.
template <void (*Kernel)(BatchDev)>
static int64_t resident_grid(size_t lds, int n_cu, int64_t units, int n_jobs) {
    static std::atomic<uint64_t> cache{0};   // (lds << 8) | blocks per compute unit, 0: none
    uint64_t c = cache.load(std::memory_order_relaxed);
    int nb = (c >> 8) == (uint64_t)lds && c != 0 ? (int)(c & 0xFF) : 0;
    if (nb == 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(Kernel), kUpdThreads,
                                                         lds) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = 8;
        }
        nb = std::min(nb, 255);
        cache.store(((uint64_t)lds << 8) | (uint64_t)nb, std::memory_order_relaxed);
    }
    const int64_t resident = (int64_t)n_cu * nb;
    if (units <= resident) return std::max<int64_t>(1, units);
    return units % resident == 0 || n_jobs > 1 ? resident : std::min<int64_t>(units, (int64_t)n_cu * 8);
}

template <int MT, typename S, int KR>
static dvl_status launch_typed(const BatchDev& b, int n_cu, hipStream_t s, hipEvent_t* ev) {
    if (b.paths & kPathEntries) {
        if (dvl_status st = check_no_static_lds<k_tile_sums<MT, S, KR, 1>>("k_tile_sums")) return st;
        if (dvl_status st = check_no_static_lds<k_vmax_exact<MT, S, KR, 1>>("k_vmax_exact")) return st;
    }
    auto mark = [&](int i) -> dvl_status {
        if (ev && ev[i]) DVL_HIP(hipEventRecord(ev[i], s));
        return DVL_OK;
    };
    const size_t lds1 = (size_t)b.max_job_tf * sizeof(float);
    const size_t lds1i = (size_t)std::max(1, b.max_req_job) * MT * kIdxTable * sizeof(float);
    const unsigned g1 = (unsigned)std::max<int64_t>(1, std::min<int64_t>(b.k1_units, (int64_t)n_cu * 8));
    if (dvl_status st = mark(0)) return st;
    if (b.any_exact) {
        if (b.paths & kPathValues) {
            hipLaunchKernelGGL((k_vmax_exact<MT, S, KR, 0>), dim3(g1), dim3(kUpdThreads), lds1, s, b);
            DVL_HIP(hipGetLastError());
        }
        if (b.paths & kPathEntries) {
            hipLaunchKernelGGL((k_vmax_exact<MT, S, KR, 1>), dim3(g1), dim3(kUpdThreads), lds1i, s, b);
            DVL_HIP(hipGetLastError());
        }
    }
    if (dvl_status st = mark(1)) return st;
    if (b.paths & kPathValues) {
        const unsigned g = (unsigned)resident_grid<k_tile_sums<MT, S, KR, 0>>(lds1, n_cu, b.k1_units, b.n_jobs);
        hipLaunchKernelGGL((k_tile_sums<MT, S, KR, 0>), dim3(g), dim3(kUpdThreads), lds1, s, b);
        DVL_HIP(hipGetLastError());
    }
    if (b.paths & kPathEntries) {
        const unsigned g = (unsigned)resident_grid<k_tile_sums<MT, S, KR, 1>>(lds1i, n_cu, b.k1_units, b.n_jobs);
        hipLaunchKernelGGL((k_tile_sums<MT, S, KR, 1>), dim3(g), dim3(kUpdThreads), lds1i, s, b);
        DVL_HIP(hipGetLastError());
    }
    if (dvl_status st = mark(2)) return st;
    if (dvl_status st = launch_carry_classify(b, s)) return st;
    if (dvl_status st = mark(3)) return st;
    const size_t lds3 = (size_t)((b.max_req_tf + 3) & ~3) * sizeof(float) + (size_t)b.max_tile_steps * kStageBytesPerStep;
    const unsigned g3 = (unsigned)std::max<int64_t>(1, std::min<int64_t>(b.k3_units, (int64_t)n_cu * 16));
    if (b.paths & kPathValues) {
        hipLaunchKernelGGL((k_bin<MT, S, 0>), dim3(g3), dim3(kBinThreads), lds3, s, b);
        DVL_HIP(hipGetLastError());
    }
    if (b.paths & kPathEntries) {
        hipLaunchKernelGGL((k_bin<MT, S, 1>), dim3(g3), dim3(kBinThreads), lds3, s, b);
        DVL_HIP(hipGetLastError());
    }
    if (b.paths & kPathStoredF) {
        hipLaunchKernelGGL((k_bin<MT, S, 2>), dim3(g3), dim3(kBinThreads), lds3, s, b);
        DVL_HIP(hipGetLastError());
    }
    if (dvl_status st = mark(4)) return st;
    {
        const unsigned g4 = (unsigned)std::max<int64_t>(1, (b.k4_units + 3) / 4);
        hipLaunchKernelGGL((k_bin_stats<MT, S>), dim3(g4), dim3(256), 0, s, b);
        DVL_HIP(hipGetLastError());
    }
    return mark(5);
}

// One storage type and field count (both request-count variants).  Each
// (S, MT) pair is instantiated in a translation unit of its own, generated by
// the build (the fifteen compile in parallel); elsewhere the declarations
// below keep the compiler from instantiating them.
template <typename S, int MT>
dvl_status launch_sm(const BatchDev& b, int max_req, int n_cu, hipStream_t s, uint64_t layout, hipEvent_t* ev) {
    if (layout != kDescriptorLayout) {
        set_error("descriptor layout mismatch between library objects (%llx vs %llx): rebuild the library",
                  (unsigned long long)layout, (unsigned long long)kDescriptorLayout);
        return DVL_E_INVALID;
    }
    if (max_req <= 1) return launch_typed<MT, S, 1>(b, n_cu, s, ev);
    return launch_typed<MT, S, kMaxReqPerJob>(b, n_cu, s, ev);
}

#define DVL_FOR_EACH_LAUNCH(X) \
    X(F32, 1) X(F32, 2) X(F32, 4) X(F32, 8) X(F32, 16) \
    X(F16, 1) X(F16, 2) X(F16, 4) X(F16, 8) X(F16, 16) \
    X(BF16, 1) X(BF16, 2) X(BF16, 4) X(BF16, 8) X(BF16, 16)
#define DVL_EXTERN_LAUNCH(S, MT) \
    extern template dvl_status launch_sm<S, MT>(const BatchDev&, int, int, hipStream_t, uint64_t, hipEvent_t*);
DVL_FOR_EACH_LAUNCH(DVL_EXTERN_LAUNCH)
#undef DVL_EXTERN_LAUNCH

// Field-count variants: batches whose jobs all have 1, 2, 4 or 8 fields run
// the variant with that count fixed at compile time; others (mixed counts,
// 3, 5-7 or more than 8 fields) the general variant, which reads M per job.
template <typename S>
static dvl_status launch_s(const BatchDev& b, int max_m, int max_req, int n_cu, hipStream_t s, uint64_t layout,
                           hipEvent_t* ev) {
    switch (max_m) {
        case 1: return launch_sm<S, 1>(b, max_req, n_cu, s, layout, ev);
        case 2: return launch_sm<S, 2>(b, max_req, n_cu, s, layout, ev);
        case 4: return launch_sm<S, 4>(b, max_req, n_cu, s, layout, ev);
        case 8: return launch_sm<S, 8>(b, max_req, n_cu, s, layout, ev);
        default: return launch_sm<S, 16>(b, max_req, n_cu, s, layout, ev);
    }
}

}  // namespace dvl
