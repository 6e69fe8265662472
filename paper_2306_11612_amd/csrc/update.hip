// Per-update kernels of dynamic volume lines (Eqs. 1-4 and section
// "Projecting Cells to 1D" of Zellmann et al., arXiv 2306.11612), over a
// batch of jobs (a job = one volume and up to 8 TF requests).
//
//   K0 k_vmax_exact   (DVL_VMAX_EXACT requests only) max over cells of V_h
//   K1 k_tile_sums    TF lookup, V_h (Eq. 1) and importance f (Eq. 3) of every
//                     cell for every request of its job (one read of the
//                     cells); fp64 sum of f per tile; each wave owns a run of
//                     consecutive tiles and records their prefix inside it
//   K2 + K3a k_carry_classify (one kernel)
//                     K2, per request: exclusive scan of the run totals (Eq. 4
//                     across runs; fp64 or compensated fp32), made monotone;
//                     K3a, per (request, tile), one lane each, once the
//                     request's carry is published: if the tile's pixel
//                     interval lies inside one bin, the whole tile is that
//                     bin's part; otherwise the tile is queued
//   K3b k_bin         per queued tile: recompute f, monotone in-tile prefix,
//                     pixel interval of every cell; the cell range of every
//                     bin that starts and ends inside the tile, and of the
//                     tile's first and last bin (per-tile records)
//   K4 k_bin_stats    per (request, bin): the bin's cell range (merged from
//                     the records of the tiles it touches), then its mean,
//                     min and max per field from the values of its partial
//                     end steps and the per-step and per-tile statistics of
//                     the steps and tiles it covers whole; the height
//
// The paper's GPU version runs the projection once per field with global
// atomics on the W bins (its Table 1 bottleneck).  Here the projection is
// hierarchical over tiles (the paper's future-work suggestion): only tiles
// that contain a bin edge are read again, to find where bins start and end;
// no atomics on bins, and the statistics of a bin cost work in proportion to
// its two ends, not to its cells.  Results are bitwise deterministic and do
// not depend on what else is in the batch.
//
// K0, K1, K3b and K4 depend on the field storage type and the field count;
// they live in update_kernels.hpp and are instantiated once per (type,
// count) in translation units the build generates.  This file holds K2, K3a,
// the per-tile statistics, the TF entry cache builder and the launcher.
#include "update_kernels.hpp"

namespace dvl {

// ------------------------------------------------------------------ workspace

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t workspace_bytes(int64_t T, int M, int W, int64_t fcells) {
    size_t b = 0;
    b += al256((size_t)T * 8);             // local_prefix
    b += al256((size_t)T * 8);             // run_total
    b += al256((size_t)(T + 1) * 8);       // run_base
    b += 2 * al256((size_t)T * 4);         // head/tail bin
    b += 2 * al256((size_t)2 * T * 4);     // rec first/last
    b += 2 * al256((size_t)W * 4);         // per-bin tile bounds
    b += al256(8 * 8);                     // scalars
    b += al256((size_t)fcells * 4);        // stored importance
    return b;
}

void workspace_carve(void* base, int64_t T, int M, int W, int64_t fcells, UpdWorkspace* w) {
    char* p = (char*)base;
    auto take = [&](size_t bytes) { char* q = p; p += al256(bytes); return (void*)q; };
    w->local_prefix = (double*)take((size_t)T * 8);
    w->run_total = (double*)take((size_t)T * 8);
    w->run_base = (double*)take((size_t)(T + 1) * 8);
    w->head_bin = (int32_t*)take((size_t)T * 4);
    w->tail_bin = (int32_t*)take((size_t)T * 4);
    w->rec_first = (uint32_t*)take((size_t)2 * T * 4);
    w->rec_last = (uint32_t*)take((size_t)2 * T * 4);
    w->bin_t1 = (int32_t*)take((size_t)W * 4);
    w->bin_ta = (int32_t*)take((size_t)W * 4);
    w->scal = (double*)take(8 * 8);
    w->fstore = fcells ? (float*)take((size_t)fcells * 4) : nullptr;
}

// ------------------------------------------------------------------ K2

struct AccF64 {
    double v;
    __device__ static AccF64 zero() { return {0.0}; }
    __device__ void add(double x) { v += x; }
    __device__ static AccF64 combine(const AccF64& a, const AccF64& b) { return {a.v + b.v}; }
    __device__ double value() const { return v; }
    __device__ AccF64 shfl_up(int d) const { return {shfl_up_d(v, d)}; }
};

// compensated fp32: unevaluated sum hi + lo, error-free TwoSum on every add
struct AccKahan32 {
    float hi, lo;
    __device__ static AccKahan32 zero() { return {0.0f, 0.0f}; }
    __device__ static void two_sum(float a, float b, float& s, float& e) {
        s = a + b;
        const float bb = s - a;
        e = (a - (s - bb)) + (b - bb);
    }
    __device__ void add(double xd) {
        const float x = (float)xd;
        float s, e;
        two_sum(hi, x, s, e);
        lo += e;
        two_sum(s, lo, hi, lo);
    }
    __device__ static AccKahan32 combine(const AccKahan32& a, const AccKahan32& b) {
        float s, e;
        two_sum(a.hi, b.hi, s, e);
        AccKahan32 r;
        const float l = e + (a.lo + b.lo);
        two_sum(s, l, r.hi, r.lo);
        return r;
    }
    __device__ double value() const { return (double)hi + (double)lo; }
    __device__ AccKahan32 shfl_up(int d) const { return {shfl_up_f(hi, d), shfl_up_f(lo, d)}; }
};

struct AccF32 {
    float v;
    __device__ static AccF32 zero() { return {0.0f}; }
    __device__ void add(double x) { v += (float)x; }
    __device__ static AccF32 combine(const AccF32& a, const AccF32& b) { return {a.v + b.v}; }
    __device__ double value() const { return (double)v; }
    __device__ AccF32 shfl_up(int d) const { return {shfl_up_f(v, d)}; }
};

constexpr int kCarryThreads = 1024;
constexpr int kCarryItems = 8;                              // run totals per thread and round
constexpr int kCarryRound = kCarryThreads * kCarryItems;
constexpr int kCarryWaves = kCarryThreads / kWave;

// One workgroup per request.  run_base[r] = sum of the run totals before r,
// run_base[R] = F_tot: a sequential prefix over each thread's 8 totals, a
// wave scan of the thread totals made monotone by a running maximum, and
// sequential wave and round bases; every base is clamped to the next thread's
// base, so the bases never decrease.
template <typename Acc>
__device__ void carry_scan(const ReqDev& q, int64_t T, int64_t n_cells) {
    __shared__ double wave_base[kCarryWaves + 1];
    __shared__ Acc wave_acc[kCarryWaves];
    __shared__ Acc round_acc;
    __shared__ double round_end;
    const int tid = thread_x(), lane = lane_id(), w = tid / kWave;
    const double* ts = q.ws.run_total;
    double* base_out = q.ws.run_base;
    if (tid == 0) {
        round_acc = Acc::zero();
        round_end = 0.0;
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < T; r0 += kCarryRound) {
        const int64_t b0 = r0 + (int64_t)tid * kCarryItems;
        double v[kCarryItems];
#pragma unroll
        for (int k = 0; k < kCarryItems; ++k) v[k] = (b0 + k < T) ? gload<double>(ts, b0 + k) : 0.0;
        Acc pre[kCarryItems];
        Acc run = Acc::zero();
#pragma unroll
        for (int k = 0; k < kCarryItems; ++k) {
            pre[k] = run;
            run.add(v[k]);
        }
        Acc inc = run;
        for (int d = 1; d < kWave; d <<= 1) {
            const Acc o = inc.shfl_up(d);
            if (lane >= d) inc = Acc::combine(o, inc);
        }
        if (lane == kWave - 1) wave_acc[w] = inc;
        __syncthreads();
        if (tid == 0) {
            Acc base = round_acc;
            double prev = round_end;
            for (int k = 0; k < kCarryWaves; ++k) {
                prev = fmax(prev, base.value());
                wave_base[k] = prev;
                base = Acc::combine(base, wave_acc[k]);
            }
            prev = fmax(prev, base.value());
            wave_base[kCarryWaves] = prev;
            round_end = prev;
            round_acc = base;
        }
        __syncthreads();
        const double wb = wave_base[w], wn = wave_base[w + 1];
        const Acc exc = inc.shfl_up(1);
        double tb = lane == 0 ? wb : fmin(fmax(wb + exc.value(), wb), wn);
        for (int d = 1; d < kWave; d <<= 1) {
            const double o = shfl_up_d(tb, d);
            if (lane >= d) tb = fmax(tb, o);
        }
        const int src = lane + 1 < kWave ? lane + 1 : lane;
        const uint64_t u = __double_as_longlong(tb);
        const int nlo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)u);
        const int nhi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(u >> 32));
        double nb = __longlong_as_double(((uint64_t)(uint32_t)nhi << 32) | (uint32_t)nlo);
        if (lane == kWave - 1) nb = wn;
        double c = tb;
#pragma unroll
        for (int k = 0; k < kCarryItems; ++k) {
            c = fmax(c, fmin(tb + pre[k].value(), nb));
            if (b0 + k < T) gstore<double>(base_out, b0 + k, c);
        }
        __syncthreads();
    }
    if (tid == 0) {
        gstore<double>(base_out, T, round_end);
        // a zero total means every f was zero: fall back to f = 1 (linear map;
        // the projection then derives the tile offsets from the cell counts)
        const bool degenerate = !(round_end > 0.0);
        gstore<double>(q.ws.scal, 0, degenerate ? (double)n_cells : round_end);
        gstore<double>(q.ws.scal, 1, degenerate ? 1.0 : 0.0);
    }
}

// The carry of request q, in the request's scan arithmetic (the whole
// workgroup; writes run_base and the scalars).
__device__ void scan_request(const BatchDev& b, int q_index) {
    const ReqDev& q = b.reqs[q_index];
    const JobDev& j = b.jobs[q.job];
    if (q.scan_mode == DVL_SCAN_KAHAN_FP32)
        carry_scan<AccKahan32>(q, j.n_runs, j.n);
    else if (q.scan_mode == DVL_SCAN_NAIVE_FP32)
        carry_scan<AccF32>(q, j.n_runs, j.n);
    else
        carry_scan<AccF64>(q, j.n_runs, j.n);
}

// K3a.  A tile whose pixel interval lies inside one bin puts every cell in
// that bin: its head record is the whole tile and no cell is read (the
// projection is hierarchical over tiles).  Other tiles are queued for K3b.
// Every tile also writes, for the bins its interval reaches, where K4 finds
// their tiles: with b0(t) = bin of X0(t) (the bin of the tile's first cell)
// and b1(t) = bin of X1(t) = b0(t + 1), the last tile touching bin b is the
// t with b0(t) <= b < b1(t) (bin_t1, the last tile: b0 <= b), and the first
// is the t with b1(t - 1) < b <= b1(t) (bin_ta, the first tile: b <= b1),
// or the next tile when tile t's last cell ends exactly at bin b's left edge
// (K4 checks it with the tile's tail bin).  These ranges partition the bins.
// Each thread classifies one tile; the workgroup appends its queued tiles
// with one atomic per projection path (a single counter contended by every
// wave was the cost of this pass).
//
// K2 and K3a run as one kernel: workgroup q < n_reqs scans request q's run
// totals and then publishes it (agent-scope release of carry_ready[q]);
// the other workgroups classify 1024 tiles each once the carries of their
// requests are published (agent-scope acquire), which saves a launch and
// its queue drain between the two.  The wait is bounded: a workgroup that
// has not seen the flag after b.carry_wait_polls polls scans the request
// itself (the same code on the same inputs writes the same bits), so the
// kernel finishes whatever the order in which its workgroups run.
constexpr int kClassifyThreads = kCarryThreads;

__device__ __forceinline__ void await_carry(const BatchDev& b, int q) {
    __shared__ int ready;
    if (thread_x() == 0) {
        // polls are relaxed (an acquiring load invalidates the L2 each time,
        // which slowed the scan it waits for); one acquire fence follows
        uint32_t* flag = b.carry_ready + q;
        int spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u && spins < b.carry_wait_polls) {
            __builtin_amdgcn_s_sleep(4);
            ++spins;
        }
        ready = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (!ready) scan_request(b, q);
    __syncthreads();
}

__global__ __launch_bounds__(kClassifyThreads) void k_carry_classify(BatchDev bd) {
    if (block_x() < bd.n_reqs) {
        scan_request(bd, block_x());
        __syncthreads();
        if (thread_x() == 0) {
            __threadfence();
            __hip_atomic_store(bd.carry_ready + block_x(), 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    __shared__ uint32_t wcount[3][kClassifyThreads / kWave];
    __shared__ uint32_t wbase[3];
    const int lane = lane_id(), w = thread_x() / kWave;
    const int64_t u0 = (int64_t)(block_x() - bd.n_reqs) * kClassifyThreads;
    // the requests of this workgroup's tiles: their carries first
    {
        const int qa = find_req_k3(bd, u0);
        const int qb = find_req_k3(bd, min(u0 + kClassifyThreads, bd.k3_units) - 1);
        for (int q = qa; q <= qb; ++q) await_carry(bd, q);
    }
    const int64_t u = u0 + thread_x();
    bool need = false;
    int path = 0;
    if (u < bd.k3_units) {
        const ReqDev& q = bd.reqs[find_req_k3(bd, u)];
        const JobDev& j = bd.jobs[q.job];
        path = q.ws.fstore ? 2 : (j.idx[0] ? 1 : 0);
        const int64_t t = u - q.k3_unit0;
        const TileSpan sp = tile_span(q, j, t);
        const bool last_tile = t == j.n_tiles - 1;
        const int W1 = q.W - 1;
        for (int b = sp.b0, e = last_tile ? W1 : sp.b1 - 1; b <= e; ++b)
            gstore<int32_t>(q.ws.bin_t1, b, (int32_t)t);
        for (int b = t == 0 ? 0 : sp.b0 + 1, e = last_tile ? W1 : sp.b1; b <= e; ++b)
            gstore<int32_t>(q.ws.bin_ta, b, (int32_t)t);
        if (sp.b0 == sp.b1) {
            const int64_t tile_cells = (int64_t)j.tile_steps * kStepCells;
            const int64_t tbase = t * tile_cells;
            gstore<uint32_t>(q.ws.rec_first, t, (uint32_t)tbase);
            gstore<uint32_t>(q.ws.rec_last, t, (uint32_t)(min(tbase + tile_cells, j.n) - 1));
            gstore<int32_t>(q.ws.head_bin, t, sp.b0);
            gstore<int32_t>(q.ws.tail_bin, t, sp.b0);
        } else {
            need = true;
        }
    }
    // per path: the wave's queued tiles, then one atomic for the workgroup
    uint32_t mine_before[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const uint64_t mask = __ballot(need && path == p);
        mine_before[p] = (uint32_t)__popcll(mask & lanemask_lt());
        if (lane == 0) wcount[p][w] = (uint32_t)__popcll(mask);
    }
    __syncthreads();
    if (thread_x() < 3) {
        const int p = thread_x();
        uint32_t tot = 0;
        for (int k = 0; k < kClassifyThreads / kWave; ++k) tot += wcount[p][k];
        wbase[p] = tot ? atomicAdd(bd.rescan_count + p, tot) : 0u;
    }
    __syncthreads();
    if (need) {
        uint32_t base = wbase[path];
        for (int k = 0; k < w; ++k) base += wcount[path][k];
        gstore<uint64_t>(bd.rescan_queue, path * bd.k3_units + base + mine_before[path], (uint64_t)u);
    }
}

// ------------------------------------------------------------------ per-tile statistics

// sum / min / max of one sorted field over every tile and over every 256-cell
// step; one wave per tile (computed once per volume and per data change, not
// per update).  Tile sums: per lane, fp32 sums of 4 values accumulated in fp64
// over the steps, then the wave; step sums: per lane the fp64 sum of its 4
// values, then the wave.
template <typename S>
__global__ __launch_bounds__(kUpdThreads) void k_tile_aggregates(int64_t n, const void* __restrict__ field,
                                                                 int64_t n_tiles, int tile_steps,
                                                                 double* __restrict__ sum,
                                                                 float* __restrict__ mn, float* __restrict__ mx,
                                                                 double* __restrict__ ssum,
                                                                 float* __restrict__ smn, float* __restrict__ smx) {
    const int lane = lane_id();
    const int64_t wave = (int64_t)block_x() * (kUpdThreads / kWave) + thread_x() / kWave;
    const int64_t nwaves = (int64_t)grid_dim_x() * (kUpdThreads / kWave);
    for (int64_t t = wave; t < n_tiles; t += nwaves) {
        const int64_t tbase = t * tile_steps * (int64_t)kStepCells;
        double acc = 0.0;
        float lo = INFINITY, hi = -INFINITY;
        // four steps' loads in flight together (tile_steps is a multiple of 4);
        // the arithmetic runs step after step as in a plain loop
        for (int st0 = 0; st0 < tile_steps; st0 += 4) {
            const int64_t quad0 = ((tbase + (int64_t)st0 * kStepCells) >> 2) + lane;
            Quad<S> qs[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) qs[g].load(field, quad0 + (int64_t)g * kWave);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int st = st0 + g;
                const int64_t quad = quad0 + (int64_t)g * kWave;
                const Quad<S>& q = qs[g];
                float s4 = 0.0f;
                double d4 = 0.0;
                float slo = INFINITY, shi = -INFINITY;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if ((quad << 2) + k < n) {
                        const float v = q.get(k);
                        s4 += v;
                        d4 += (double)v;
                        slo = fminf(slo, v);
                        shi = fmaxf(shi, v);
                    }
                }
                acc += (double)s4;
                lo = fminf(lo, slo);
                hi = fmaxf(hi, shi);
                d4 = wave_sum_d(d4);
                slo = wave_min_f(slo);
                shi = wave_max_f(shi);
                if (lane == 0) {
                    const int64_t gs = t * tile_steps + st;
                    ssum[gs] = d4;
                    smn[gs] = slo;
                    smx[gs] = shi;
                }
            }
        }
        acc = wave_sum_d(acc);
        lo = wave_min_f(lo);
        hi = wave_max_f(hi);
        if (lane == 0) {
            sum[t] = acc;
            mn[t] = lo;
            mx[t] = hi;
        }
    }
}

dvl_status launch_tile_aggregates(int64_t n, int dtype, const void* field, int64_t n_tiles, int tile_steps,
                                  double* sum, float* mn, float* mx, double* ssum, float* smn, float* smx,
                                  int n_cu, hipStream_t s) {
    const int64_t wg_needed = (n_tiles + (kUpdThreads / kWave) - 1) / (kUpdThreads / kWave);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(wg_needed, (int64_t)n_cu * 8));
    if (dtype == DVL_F16)
        hipLaunchKernelGGL(k_tile_aggregates<F16>, dim3(grid), dim3(kUpdThreads), 0, s, n, field, n_tiles,
                           tile_steps, sum, mn, mx, ssum, smn, smx);
    else if (dtype == DVL_BF16)
        hipLaunchKernelGGL(k_tile_aggregates<BF16>, dim3(grid), dim3(kUpdThreads), 0, s, n, field, n_tiles,
                           tile_steps, sum, mn, mx, ssum, smn, smx);
    else
        hipLaunchKernelGGL(k_tile_aggregates<F32>, dim3(grid), dim3(kUpdThreads), 0, s, n, field, n_tiles,
                           tile_steps, sum, mn, mx, ssum, smn, smx);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ level codes

// One 32-bit code per 256-cell step of the sorted levels: byte k describes
// the cells [64 k, 64 k + 64) of the step (the 16 lanes 16 k .. 16 k + 15 of
// a wave reading the step): their common level, or 0xFF when they differ.
// One wave per step.
__global__ __launch_bounds__(256) void k_level_codes(const uint32_t* __restrict__ lev4, int64_t n_steps,
                                                     uint32_t* __restrict__ codes) {
    const int64_t st = ((int64_t)block_x() * block_dim_x() + thread_x()) / kWave;
    if (st >= n_steps) return;   // the whole wave
    const int lane = lane_id();
    const uint32_t w = lev4[st * kWave + lane];
    const uint32_t b0 = w & 0xFFu;
    const uint32_t c = w == b0 * 0x01010101u ? b0 : 0xFFu;
    uint32_t lo = c, hi = c;
    for (int o = 1; o < 16; o <<= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, o));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, o));
    }
    const uint32_t seg = lo == hi ? lo : 0xFFu;
    const uint32_t s0 = (uint32_t)__shfl((int)seg, 0), s1 = (uint32_t)__shfl((int)seg, 16);
    const uint32_t s2 = (uint32_t)__shfl((int)seg, 32), s3 = (uint32_t)__shfl((int)seg, 48);
    if (lane == 0) codes[st] = s0 | (s1 << 8) | (s2 << 16) | (s3 << 24);
}

dvl_status launch_level_codes(const uint8_t* level, int64_t n_steps, uint32_t* codes, hipStream_t s) {
    const int64_t threads = n_steps * kWave;
    const unsigned grid = (unsigned)std::max<int64_t>(1, (threads + 255) / 256);
    hipLaunchKernelGGL(k_level_codes, dim3(grid), dim3(256), 0, s, reinterpret_cast<const uint32_t*>(level),
                       n_steps, codes);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ TF entry cache

// entries of 4 consecutive cells per lane, packed into one 32-bit store
template <typename S>
__global__ __launch_bounds__(256) void k_build_index(int64_t n_quads, const void* __restrict__ field, float s,
                                                     float b, float nmax, uint32_t* __restrict__ out) {
    const int64_t stride = (int64_t)grid_dim_x() * block_dim_x();
    for (int64_t i = (int64_t)block_x() * block_dim_x() + thread_x(); i < n_quads; i += stride) {
        Quad<S> q;
        q.load(field, i);
        uint32_t w = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) w |= (uint32_t)tf_entry(q.get(k), s, b, nmax) << (8 * k);
        out[i] = w;
    }
}

dvl_status launch_build_index(int64_t n_pad, int dtype, const void* field, float s, float b, int n_tf,
                              uint8_t* out, int n_cu, hipStream_t st) {
    const int64_t n_quads = n_pad / 4;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_quads + 255) / 256, (int64_t)n_cu * 16));
    const float nmax = (float)(n_tf - 1);
    if (dtype == DVL_F16)
        hipLaunchKernelGGL(k_build_index<F16>, dim3(grid), dim3(256), 0, st, n_quads, field, s, b, nmax, (uint32_t*)out);
    else if (dtype == DVL_BF16)
        hipLaunchKernelGGL(k_build_index<BF16>, dim3(grid), dim3(256), 0, st, n_quads, field, s, b, nmax, (uint32_t*)out);
    else
        hipLaunchKernelGGL(k_build_index<F32>, dim3(grid), dim3(256), 0, st, n_quads, field, s, b, nmax, (uint32_t*)out);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

// ------------------------------------------------------------------ launchers

dvl_status launch_carry_classify(const BatchDev& b, hipStream_t s) {
    const int64_t blocks = (int64_t)b.n_reqs + (b.k3_units + kClassifyThreads - 1) / kClassifyThreads;
    hipLaunchKernelGGL(k_carry_classify, dim3((unsigned)blocks), dim3(kClassifyThreads), 0, s, b);
    DVL_HIP(hipGetLastError());
    return DVL_OK;
}

dvl_status launch_batch(const BatchDev& b, int dtype, int max_m, int max_req, int n_cu, hipStream_t s,
                        uint64_t layout, hipEvent_t* ev) {
    if (layout != kDescriptorLayout) {
        set_error("descriptor layout mismatch between library objects (%llx vs %llx): rebuild the library",
                  (unsigned long long)layout, (unsigned long long)kDescriptorLayout);
        return DVL_E_INVALID;
    }
    if (dtype == DVL_F16) return launch_s<F16>(b, max_m, max_req, n_cu, s, layout, ev);
    if (dtype == DVL_BF16) return launch_s<BF16>(b, max_m, max_req, n_cu, s, layout, ev);
    return launch_s<F32>(b, max_m, max_req, n_cu, s, layout, ev);
}

}  // namespace dvl
