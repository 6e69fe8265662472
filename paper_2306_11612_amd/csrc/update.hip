// Per-update kernels of dynamic volume lines (Eqs. 1-4 and section
// "Projecting Cells to 1D" of Zellmann et al., arXiv 2306.11612).
//
//   K0 k_vmax_exact   (DVL_VMAX_EXACT only) max over cells of V_h
//   K1 k_tile_sums    TF lookup, V_h (Eq. 1), importance f (Eq. 3) and the
//                     fp64 sum of f over every 4096-cell wave tile
//   K2 k_carry        carry[t] = sum of earlier tile sums (Eq. 4 across
//                     tiles, fp64 or compensated fp32), made monotone
//   K3 k_bin          recompute f; in-tile monotone prefix; pixel interval
//                     of every cell; bins complete inside a tile are reduced
//                     and finalised directly, the tile's first and last bin
//                     go to per-tile partial records
//   K4 k_edges        merge the partial records of bins shared by tiles in
//                     tile order; mean, min, max and height y = alpha(mean)
//
// The paper's GPU version runs the projection once per field with global
// atomics on the W bins (its Table 1 bottleneck).  Here all fields are
// reduced in one pass, atomic-free: a wave owns a contiguous tile, keeps
// per-lane accumulators while a whole 256-cell step falls in one bin, and
// switches to a segmented lane scan only at bin boundaries.  Results are
// bitwise deterministic.
#include "update.hpp"

#include <climits>

namespace dvl {

// ------------------------------------------------------------------ workspace

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t workspace_bytes(int64_t T, int M) {
    size_t b = 0;
    b += al256((size_t)T * 8);             // tile_sum
    b += al256((size_t)(T + 1) * 8);       // carry
    b += 2 * al256((size_t)T * 4);         // head/tail bin
    b += 2 * al256((size_t)2 * T * 4);     // rec first/last
    b += al256((size_t)2 * M * T * 8);     // rec_sum
    b += 2 * al256((size_t)2 * M * T * 4); // rec min/max
    b += al256(8 * 8);                     // scalars
    return b;
}

void workspace_carve(void* base, int64_t T, int M, UpdWorkspace* w) {
    char* p = (char*)base;
    auto take = [&](size_t bytes) { char* q = p; p += al256(bytes); return (void*)q; };
    w->tile_sum = (double*)take((size_t)T * 8);
    w->carry = (double*)take((size_t)(T + 1) * 8);
    w->head_bin = (int32_t*)take((size_t)T * 4);
    w->tail_bin = (int32_t*)take((size_t)T * 4);
    w->rec_first = (uint32_t*)take((size_t)2 * T * 4);
    w->rec_last = (uint32_t*)take((size_t)2 * T * 4);
    w->rec_sum = (double*)take((size_t)2 * M * T * 8);
    w->rec_min = (float*)take((size_t)2 * M * T * 4);
    w->rec_max = (float*)take((size_t)2 * M * T * 4);
    w->scal = (double*)take(8 * 8);
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

__device__ __forceinline__ ImpCtx make_ctx(const UpdArgs& a) {
    ImpCtx c;
    const float vm = *a.vmax_dev;
    c.inv_vmax = vm > 0.0f ? 1.0f / vm : 0.0f;
    c.fmin = a.fmin;
    c.p = a.exponent;
    c.exp_is_one = a.exp_is_one;
    c.clamp_mode = a.clamp_mode;
    c.lshift = a.level_shift;
    return c;
}

// TF entry: clamp(floor(fma(x, s, b)), 0, n_tf - 1)
__device__ __forceinline__ int tf_entry(float x, float s, float b, float nmax) {
    float t = fmaf(x, s, b);
    t = fminf(fmaxf(t, 0.0f), nmax);
    return (int)t;
}

// Eq. 1: V = max_m alpha_m(x_m) - min_m alpha_m(x_m)
template <int MT>
__device__ __forceinline__ float variation(const float (&x)[MT], int M, const float* __restrict__ tf,
                                           const UpdArgs& a, const ImpCtx& c) {
    float amax = -INFINITY, amin = INFINITY;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const int e = tf_entry(x[m], a.s[m], a.b[m], a.nmax[m]);
            const float al = tf[a.tf_off[m] + e];
            amax = fmaxf(amax, al);
            amin = fminf(amin, al);
        }
    }
    return amax - amin;
}

// Eq. 3 with the minimum importance
__device__ __forceinline__ float importance_from_v(float v, uint32_t L, const ImpCtx& c) {
    const float r = v * c.inv_vmax;
    const int e = c.lshift * (int)L;
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

__device__ __forceinline__ void load_tf(float* lds, const float* tf, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) lds[i] = tf[i];
    __syncthreads();
}

template <int MT>
__device__ __forceinline__ int fields_of(const UpdArgs& a) {
    return MT <= 8 ? MT : a.M;
}

// values of the 4 cells of this lane in the given step
template <int MT, typename S>
struct StepData {
    Quad<S> q[MT];
    uint32_t lv;
    __device__ __forceinline__ void load(const UpdArgs& a, int M, int64_t quad) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
            if (m < M) q[m].load(a.fields[m], quad);
        lv = reinterpret_cast<const uint32_t*>(a.level)[quad];
    }
};

// ------------------------------------------------------------------ K0

template <int MT, typename S>
__global__ __launch_bounds__(kUpdThreads) void k_vmax_exact(UpdArgs a) {
    extern __shared__ float tf_lds[];
    load_tf(tf_lds, a.tf, a.tf_total);
    const int M = fields_of<MT>(a);
    const ImpCtx c = make_ctx(a);
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (kUpdThreads / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kUpdThreads / kWave);
    float vmax = 0.0f;
    for (int64_t t = wave; t < a.n_tiles; t += nwaves) {
        for (int s = 0; s < kTileSteps; ++s) {
            const int64_t c0 = t * kTileCells + (int64_t)s * kStepCells;
            if (c0 >= a.n) break;
            const int64_t quad = (c0 >> 2) + lane;
            StepData<MT, S> d;
            d.load(a, M, quad);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float x[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) x[m] = m < M ? d.q[m].get(k) : 0.0f;
                if ((quad << 2) + k < a.n) vmax = fmaxf(vmax, variation<MT>(x, M, tf_lds, a, c));
            }
        }
    }
    vmax = wave_max_f(vmax);
    if (lane == 0 && vmax > 0.0f) atomicMax(reinterpret_cast<unsigned int*>(a.vmax_dev), __float_as_uint(vmax));
}

// ------------------------------------------------------------------ K1

template <int MT, typename S>
__global__ __launch_bounds__(kUpdThreads) void k_tile_sums(UpdArgs a) {
    extern __shared__ float tf_lds[];
    load_tf(tf_lds, a.tf, a.tf_total);
    const int M = fields_of<MT>(a);
    const ImpCtx c = make_ctx(a);
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (kUpdThreads / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kUpdThreads / kWave);
    for (int64_t t = wave; t < a.n_tiles; t += nwaves) {
        double acc = 0.0;
        const int64_t tbase = t * kTileCells;
        const int nsteps = (int)min((int64_t)kTileSteps, (a.n - tbase + kStepCells - 1) / kStepCells);
        StepData<MT, S> cur;
        cur.load(a, M, (tbase >> 2) + lane);
        for (int s = 0; s < nsteps; ++s) {
            const int64_t quad = ((tbase + (int64_t)s * kStepCells) >> 2) + lane;
            StepData<MT, S> nxt;
            if (s + 1 < nsteps) nxt.load(a, M, quad + kWave);
            float f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float x[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) x[m] = m < M ? cur.q[m].get(k) : 0.0f;
                const float v = variation<MT>(x, M, tf_lds, a, c);
                const float fk = importance_from_v(v, (cur.lv >> (8 * k)) & 0xFFu, c);
                f[k] = ((quad << 2) + k < a.n) ? fk : 0.0f;
            }
            acc += (double)((f[0] + f[1]) + (f[2] + f[3]));
            cur = nxt;
        }
        acc = wave_sum_d(acc);
        if (lane == 0) a.ws.tile_sum[t] = acc;
    }
}

// ------------------------------------------------------------------ K2

struct AccF64 {
    double v;
    __device__ static AccF64 zero() { return {0.0}; }
    __device__ void add(double x) { v += x; }
    __device__ static AccF64 combine(const AccF64& a, const AccF64& b) { return {a.v + b.v}; }
    __device__ double value() const { return v; }
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
};

struct AccF32 {
    float v;
    __device__ static AccF32 zero() { return {0.0f}; }
    __device__ void add(double x) { v += (float)x; }
    __device__ static AccF32 combine(const AccF32& a, const AccF32& b) { return {a.v + b.v}; }
    __device__ double value() const { return (double)v; }
};

constexpr int kCarryThreads = 1024;

template <typename Acc>
__global__ __launch_bounds__(kCarryThreads) void k_carry(UpdArgs a) {
    __shared__ Acc sh[kCarryThreads];
    __shared__ double shm[kCarryThreads];
    const int64_t T = a.n_tiles;
    const int tid = threadIdx.x;
    const double* ts = a.ws.tile_sum;
    double* carry = a.ws.carry;

    // 1. every thread sums its contiguous chunk of tile sums
    const int64_t chunk = (T + kCarryThreads - 1) / kCarryThreads;
    const int64_t lo = min(T, (int64_t)tid * chunk), hi = min(T, lo + chunk);
    Acc s = Acc::zero();
    for (int64_t i = lo; i < hi; ++i) s.add(ts[i]);

    // 2. inclusive Hillis-Steele scan of the chunk totals across the block
    sh[tid] = s;
    __syncthreads();
    for (int d = 1; d < kCarryThreads; d <<= 1) {
        Acc v = sh[tid];
        if (tid >= d) v = Acc::combine(sh[tid - d], v);
        __syncthreads();
        sh[tid] = v;
        __syncthreads();
    }
    Acc run = tid == 0 ? Acc::zero() : sh[tid - 1];

    // 3. sequential carries inside the chunk; carry[T] is the total
    for (int64_t i = lo; i < hi; ++i) {
        carry[i] = run.value();
        run.add(ts[i]);
    }
    if (tid == kCarryThreads - 1) carry[T] = sh[kCarryThreads - 1].value();
    __syncthreads();

    // 4. make the carries monotone (rounding of the block scan can step back
    //    by an ulp at chunk boundaries): running maximum over carry[0..T]
    const int64_t n1 = T + 1;
    const int64_t ch1 = (n1 + kCarryThreads - 1) / kCarryThreads;
    const int64_t lo1 = min(n1, (int64_t)tid * ch1), hi1 = min(n1, lo1 + ch1);
    double m = 0.0;
    for (int64_t i = lo1; i < hi1; ++i) m = fmax(m, carry[i]);
    shm[tid] = m;
    __syncthreads();
    for (int d = 1; d < kCarryThreads; d <<= 1) {
        double v = shm[tid];
        if (tid >= d) v = fmax(shm[tid - d], v);
        __syncthreads();
        shm[tid] = v;
        __syncthreads();
    }
    double rm = tid == 0 ? 0.0 : shm[tid - 1];
    for (int64_t i = lo1; i < hi1; ++i) {
        rm = fmax(rm, carry[i]);
        carry[i] = rm;
    }
    __syncthreads();

    // 5. total; a zero total means every f was zero: fall back to f = 1
    const double F = carry[T];
    const bool degenerate = !(F > 0.0);
    if (degenerate) {
        for (int64_t i = tid; i < T; i += kCarryThreads) carry[i] = (double)(i * kTileCells);
        if (tid == 0) carry[T] = (double)a.n;
    }
    if (tid == 0) {
        a.ws.scal[0] = degenerate ? (double)a.n : F;
        a.ws.scal[1] = degenerate ? 1.0 : 0.0;
    }
}

// ------------------------------------------------------------------ K3 helpers

template <int MT>
struct Seg {
    double sum[MT];
    float mn[MT];
    float mx[MT];
    uint32_t first;
    uint32_t last;
};

template <int MT>
__device__ __forceinline__ void seg_clear(Seg<MT>& s) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        s.sum[m] = 0.0;
        s.mn[m] = INFINITY;
        s.mx[m] = -INFINITY;
    }
    s.first = 0xFFFFFFFFu;
    s.last = 0u;
}

template <int MT>
__device__ __forceinline__ void seg_init(Seg<MT>& s, const float (&x)[MT], uint32_t g) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        s.sum[m] = (double)x[m];
        s.mn[m] = x[m];
        s.mx[m] = x[m];
    }
    s.first = g;
    s.last = g;
}

template <int MT>
__device__ __forceinline__ void seg_add(Seg<MT>& s, const float (&x)[MT], uint32_t g) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        s.sum[m] += (double)x[m];
        s.mn[m] = fminf(s.mn[m], x[m]);
        s.mx[m] = fmaxf(s.mx[m], x[m]);
    }
    s.last = g;
}

// a precedes b in cell order
template <int MT>
__device__ __forceinline__ Seg<MT> seg_combine(const Seg<MT>& a, const Seg<MT>& b) {
    Seg<MT> r;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        r.sum[m] = a.sum[m] + b.sum[m];
        r.mn[m] = fminf(a.mn[m], b.mn[m]);
        r.mx[m] = fmaxf(a.mx[m], b.mx[m]);
    }
    r.first = min(a.first, b.first);
    r.last = max(a.last, b.last);
    return r;
}

template <int MT>
__device__ __forceinline__ Seg<MT> seg_shfl_up(const Seg<MT>& s, int d) {
    Seg<MT> r;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        r.sum[m] = shfl_up_d(s.sum[m], d);
        r.mn[m] = shfl_up_f(s.mn[m], d);
        r.mx[m] = shfl_up_f(s.mx[m], d);
    }
    r.first = (uint32_t)shfl_up_i((int)s.first, d);
    r.last = (uint32_t)shfl_up_i((int)s.last, d);
    return r;
}

template <int MT>
__device__ __forceinline__ Seg<MT> seg_readlane(const Seg<MT>& s, int l) {
    Seg<MT> r;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        r.sum[m] = readlane(s.sum[m], l);
        r.mn[m] = readlane(s.mn[m], l);
        r.mx[m] = readlane(s.mx[m], l);
    }
    r.first = readlane(s.first, l);
    r.last = readlane(s.last, l);
    return r;
}

// a bin whose cells all lie in this tile: finalise it
template <int MT>
__device__ void write_final(const UpdArgs& a, int M, int key, const Seg<MT>& s, const float* tf) {
    const uint32_t cnt = s.last - s.first + 1u;
    a.first_cell[key] = s.first;
    a.last_cell[key] = s.last;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const float mean = (float)(s.sum[m] / (double)cnt);
            const int e = tf_entry(mean, a.s[m], a.b[m], a.nmax[m]);
            const int64_t o = (int64_t)m * a.W + key;
            a.mean[o] = mean;
            a.vmin[o] = s.mn[m];
            a.vmax[o] = s.mx[m];
            a.y[o] = tf[a.tf_off[m] + e];
        }
    }
}

// r = 0: head record (the tile's first bin), r = 1: tail record (its last bin)
template <int MT>
__device__ void write_record(const UpdArgs& a, int M, int64_t t, int r, const Seg<MT>& s) {
    const int64_t T = a.n_tiles;
    a.ws.rec_first[r * T + t] = s.first;
    a.ws.rec_last[r * T + t] = s.last;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m < M) {
            const int64_t o = ((int64_t)r * M + m) * T + t;
            a.ws.rec_sum[o] = s.sum[m];
            a.ws.rec_min[o] = s.mn[m];
            a.ws.rec_max[o] = s.mx[m];
        }
    }
}

template <int MT>
__device__ __forceinline__ void emit_bin(const UpdArgs& a, int M, int64_t t, int Bh, int key,
                                         const Seg<MT>& s, const float* tf) {
    if (key == Bh)
        write_record<MT>(a, M, t, 0, s);
    else
        write_final<MT>(a, M, key, s, tf);
}

// ------------------------------------------------------------------ K3

template <int MT, typename S>
__global__ __launch_bounds__(kUpdThreads) void k_bin(UpdArgs a) {
    extern __shared__ float tf_lds[];
    load_tf(tf_lds, a.tf, a.tf_total);
    const int M = fields_of<MT>(a);
    const ImpCtx c = make_ctx(a);
    const bool degenerate = a.ws.scal[1] != 0.0;
    const double Ftot = a.ws.scal[0];
    const double scale_d = (double)a.W / Ftot;
    const float scale_f = (float)scale_d;
    const int W1 = a.W - 1;
    const int lane = lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (kUpdThreads / kWave) + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * (kUpdThreads / kWave);

    for (int64_t t = wave; t < a.n_tiles; t += nwaves) {
        const int64_t tbase = t * kTileCells;
        const float X0 = (float)(a.ws.carry[t] * scale_d);
        const float X1 = (float)(a.ws.carry[t + 1] * scale_d);
        const int64_t tend = min(tbase + (int64_t)kTileCells, a.n);
        const uint32_t last_valid = (uint32_t)(tend - 1);
        const int nsteps = (int)((tend - tbase + kStepCells - 1) / kStepCells);

        float run = 0.0f;
        bool o_valid = false;
        int O = -1, Bh = -1;
        uint32_t O_first = 0, O_last = 0;
        Seg<MT> Ob;
        seg_clear(Ob);
        double asum[MT];
        float amin[MT], amax[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            asum[m] = 0.0;
            amin[m] = INFINITY;
            amax[m] = -INFINITY;
        }

        StepData<MT, S> cur;
        cur.load(a, M, (tbase >> 2) + lane);
        for (int s = 0; s < nsteps; ++s) {
            const int64_t c0 = tbase + (int64_t)s * kStepCells;
            const int64_t quad = (c0 >> 2) + lane;
            StepData<MT, S> nxt;
            if (s + 1 < nsteps) nxt.load(a, M, quad + kWave);

            float x[MT][4];
            float f[4];
            uint32_t g[4];
            bool valid[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float xk[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    xk[m] = m < M ? cur.q[m].get(k) : 0.0f;
                    x[m][k] = xk[m];
                }
                g[k] = (uint32_t)((quad << 2) + k);
                valid[k] = (int64_t)g[k] < a.n;
                float fk = 1.0f;
                if (!degenerate) fk = importance_from_v(variation<MT>(xk, M, tf_lds, a, c),
                                                        (cur.lv >> (8 * k)) & 0xFFu, c);
                f[k] = valid[k] ? fk : 0.0f;
            }

            // monotone in-tile prefix: lane-serial over 4 cells, wave sum scan,
            // running max to undo rounding steps back, min-clamp inside the lane
            const float p1 = f[0], p2 = p1 + f[1], p3 = p2 + f[2], tl = p3 + f[3];
            const float B = wave_incl_max(wave_incl_sum(tl));
            const float Bex = shfl_up1(B, 0.0f);
            const float stot = readlane(B, kWave - 1);
            float xs[5];
            xs[0] = fminf(fmaf(run + fminf(Bex, B), scale_f, X0), X1);
            xs[1] = fminf(fmaf(run + fminf(Bex + p1, B), scale_f, X0), X1);
            xs[2] = fminf(fmaf(run + fminf(Bex + p2, B), scale_f, X0), X1);
            xs[3] = fminf(fmaf(run + fminf(Bex + p3, B), scale_f, X0), X1);
            xs[4] = fminf(fmaf(run + B, scale_f, X0), X1);
            run = run + stot;

            // pixel bins of each cell: [floor(x1), ceil(x2) - 1], clamped
            int blo[4], bhi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float en = (g[k] == last_valid) ? X1 : xs[k + 1];
                blo[k] = max(0, min((int)floorf(xs[k]), W1));
                bhi[k] = max(blo[k], min((int)ceilf(en) - 1, W1));
            }

            const bool full = c0 + kStepCells <= a.n;
            const int key0 = readlane(blo[0], 0);
            if (s == 0) Bh = key0;
            const int key_end = full ? readlane(bhi[3], kWave - 1) : INT_MAX;

            if (full && key0 == key_end && (!o_valid || key0 == O)) {
                // the whole step lies in one bin: per-lane accumulation
                if (!o_valid) {
                    o_valid = true;
                    O = key0;
                    O_first = (uint32_t)c0;
                    seg_clear(Ob);
                }
                O_last = (uint32_t)(c0 + kStepCells - 1);
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    if (m < M) {
                        const float s4 = (x[m][0] + x[m][1]) + (x[m][2] + x[m][3]);
                        asum[m] += (double)s4;
                        amin[m] = fminf(amin[m], fminf(fminf(x[m][0], x[m][1]), fminf(x[m][2], x[m][3])));
                        amax[m] = fmaxf(amax[m], fmaxf(fmaxf(x[m][0], x[m][1]), fmaxf(x[m][2], x[m][3])));
                    }
                }
                cur = nxt;
                continue;
            }

            // ---- bin boundary inside the step: segmented reduction ----
            // (1) the open bin's statistics so far, uniform across the wave
            Seg<MT> Os;
            seg_clear(Os);
            if (o_valid) {
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    Os.sum[m] = Ob.sum[m] + wave_sum_d(asum[m]);
                    Os.mn[m] = fminf(Ob.mn[m], wave_min_f(amin[m]));
                    Os.mx[m] = fmaxf(Ob.mx[m], wave_max_f(amax[m]));
                    asum[m] = 0.0;
                    amin[m] = INFINITY;
                    amax[m] = -INFINITY;
                }
                Os.first = O_first;
                Os.last = O_last;
            }

            // (2) lane-local pass over this lane's elements: every cell
            //     belongs to its first bin; a cell spanning bins is also the
            //     whole content of the bins strictly inside its interval and
            //     the first member of its last bin
            bool any = false, hcl = false;
            int ck = INT_MAX, hk = INT_MAX;
            Seg<MT> cs, hs;
            seg_clear(cs);
            seg_clear(hs);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!valid[k]) continue;
                float xk[MT];
#pragma unroll
                for (int m = 0; m < MT; ++m) xk[m] = x[m][k];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    if (e == 1 && bhi[k] == blo[k]) break;
                    const int key = e == 0 ? blo[k] : bhi[k];
                    if (e == 1) {
                        for (int b = blo[k] + 1; b < bhi[k]; ++b) {
                            Seg<MT> one;
                            seg_init(one, xk, g[k]);
                            write_final<MT>(a, M, b, one, tf_lds);
                        }
                    }
                    if (!any) {
                        any = true;
                        ck = key;
                        seg_init(cs, xk, g[k]);
                    } else if (key == ck) {
                        seg_add(cs, xk, g[k]);
                    } else {
                        if (!hcl) {
                            hcl = true;
                            hk = ck;
                            hs = cs;
                        } else {
                            emit_bin<MT>(a, M, t, Bh, ck, cs, tf_lds);  // complete, inside the lane
                        }
                        ck = key;
                        seg_init(cs, xk, g[k]);
                    }
                }
            }

            // (3) segmented inclusive scan of the lanes' last segments
            const int prev_ck = shfl_up_i(ck, 1);
            const int prev_any = shfl_up_i(any ? 1 : 0, 1);
            bool fl = (lane == 0) || hcl || !any || !prev_any || prev_ck != ck;
            Seg<MT> v = cs;
            for (int d = 1; d < kWave; d <<= 1) {
                const Seg<MT> pv = seg_shfl_up(v, d);
                const bool pf = shfl_up_i(fl ? 1 : 0, d) != 0;
                if (lane >= d && !fl) {
                    v = seg_combine(pv, v);
                    fl = pf;
                }
            }
            const bool o_cont = o_valid && key0 == O;
            const int last_lane = full ? kWave - 1 : (int)((a.n - 1 - c0) >> 2);

            // (4a) first segments that close inside a lane
            const Seg<MT> pvs = seg_shfl_up(v, 1);
            if (hcl) {
                Seg<MT> agg = hs;
                if (lane > 0 && prev_any && prev_ck == hk) agg = seg_combine(pvs, hs);
                if (o_cont && hk == key0) agg = seg_combine(Os, agg);
                emit_bin<MT>(a, M, t, Bh, hk, agg, tf_lds);
            }
            // (4b) last segments that end with this lane (not the last valid lane)
            const int fk = any ? (hcl ? hk : ck) : INT_MAX;
            const int next_fk = __builtin_amdgcn_ds_bpermute(min(lane + 1, kWave - 1) << 2, fk);
            if (any && lane != last_lane && next_fk != ck) {
                Seg<MT> agg = v;
                if (o_cont && ck == key0) agg = seg_combine(Os, agg);
                emit_bin<MT>(a, M, t, Bh, ck, agg, tf_lds);
            }
            // (4c) the open bin ended with the previous step
            if (o_valid && !o_cont && lane == 0) emit_bin<MT>(a, M, t, Bh, O, Os, tf_lds);

            // (5) the last valid lane's segment stays open
            const int newO = readlane(ck, last_lane);
            Seg<MT> nv = seg_readlane(v, last_lane);
            if (o_cont && newO == key0) nv = seg_combine(Os, nv);
            O = newO;
            Ob = nv;
            O_first = nv.first;
            O_last = nv.last;
            o_valid = true;
            cur = nxt;
        }

        // tile end: the open bin is the tile's last bin
        Seg<MT> Os;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            Os.sum[m] = Ob.sum[m] + wave_sum_d(asum[m]);
            Os.mn[m] = fminf(Ob.mn[m], wave_min_f(amin[m]));
            Os.mx[m] = fmaxf(Ob.mx[m], wave_max_f(amax[m]));
        }
        Os.first = O_first;
        Os.last = O_last;
        if (lane == 0 && O >= 0) {
            write_record<MT>(a, M, t, O == Bh ? 0 : 1, Os);
            a.ws.head_bin[t] = Bh;
            a.ws.tail_bin[t] = O;
        }
    }
}

// ------------------------------------------------------------------ K4

template <int MT>
__global__ __launch_bounds__(256) void k_edges(UpdArgs a) {
    const int M = fields_of<MT>(a);
    const int lane = lane_id();
    const int b = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.f_total = a.ws.scal[0];
        *a.vmax_used = *a.vmax_dev;
    }
    if (b >= a.W) return;
    const int64_t T = a.n_tiles;
    const int32_t* hb = a.ws.head_bin;
    const int32_t* tb = a.ws.tail_bin;
    // tiles touching bin b: t0 = first with tail >= b, t1 = last with head <= b
    int64_t lo = 0, hi = T;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (tb[mid] < b) lo = mid + 1; else hi = mid;
    }
    const int64_t t0 = lo;
    lo = 0;
    hi = T;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (hb[mid] <= b) lo = mid + 1; else hi = mid;
    }
    const int64_t t1 = lo - 1;
    if (t0 <= t1 && t0 == t1 && hb[t0] < b && b < tb[t0]) return;  // finalised by K3

    Seg<MT> acc;
    seg_clear(acc);
    for (int64_t t = t0 + lane; t <= t1; t += kWave) {
        const int r = hb[t] == b ? 0 : (tb[t] == b ? 1 : -1);
        if (r < 0) continue;
        Seg<MT> s;
        s.first = a.ws.rec_first[r * T + t];
        s.last = a.ws.rec_last[r * T + t];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (m < M) {
                const int64_t o = ((int64_t)r * M + m) * T + t;
                s.sum[m] = a.ws.rec_sum[o];
                s.mn[m] = a.ws.rec_min[o];
                s.mx[m] = a.ws.rec_max[o];
            } else {
                s.sum[m] = 0.0;
                s.mn[m] = INFINITY;
                s.mx[m] = -INFINITY;
            }
        }
        acc = seg_combine(acc, s);
    }
    // deterministic butterfly merge
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        acc.sum[m] = wave_sum_d(acc.sum[m]);
        acc.mn[m] = wave_min_f(acc.mn[m]);
        acc.mx[m] = wave_max_f(acc.mx[m]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        acc.first = min(acc.first, (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ o) << 2, (int)acc.first));
        acc.last = max(acc.last, (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ o) << 2, (int)acc.last));
    }
    if (lane != 0) return;
    if (acc.first == 0xFFFFFFFFu) {  // no cell (cannot happen with a positive total width)
        a.first_cell[b] = 0xFFFFFFFFu;
        a.last_cell[b] = 0xFFFFFFFEu;
        for (int m = 0; m < M; ++m) {
            const int64_t o = (int64_t)m * a.W + b;
            a.mean[o] = 0.0f;
            a.vmin[o] = INFINITY;
            a.vmax[o] = -INFINITY;
            a.y[o] = 0.0f;
        }
        return;
    }
    const uint32_t cnt = acc.last - acc.first + 1u;
    a.first_cell[b] = acc.first;
    a.last_cell[b] = acc.last;
    for (int m = 0; m < M; ++m) {
        const float mean = (float)(acc.sum[m] / (double)cnt);
        const int e = tf_entry(mean, a.s[m], a.b[m], a.nmax[m]);
        const int64_t o = (int64_t)m * a.W + b;
        a.mean[o] = mean;
        a.vmin[o] = acc.mn[m];
        a.vmax[o] = acc.mx[m];
        a.y[o] = a.tf[a.tf_off[m] + e];
    }
}

// ------------------------------------------------------------------ launcher

template <int MT, typename S>
static dvl_status launch_typed(const UpdArgs& a, int n_cu, hipStream_t s, hipEvent_t* ev) {
    const size_t lds = (size_t)a.tf_total * sizeof(float);
    const int64_t wg_needed = (a.n_tiles + (kUpdThreads / kWave) - 1) / (kUpdThreads / kWave);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(wg_needed, (int64_t)n_cu * 8));
    auto mark = [&](int i) -> dvl_status {
        if (ev) DVL_HIP(hipEventRecord(ev[i], s));
        return DVL_OK;
    };
    if (dvl_status st = mark(0)) return st;
    if (a.vmax_exact) {
        hipLaunchKernelGGL((k_vmax_exact<MT, S>), dim3(grid), dim3(kUpdThreads), lds, s, a);
        DVL_HIP(hipGetLastError());
    }
    if (dvl_status st = mark(1)) return st;
    hipLaunchKernelGGL((k_tile_sums<MT, S>), dim3(grid), dim3(kUpdThreads), lds, s, a);
    DVL_HIP(hipGetLastError());
    if (dvl_status st = mark(2)) return st;
    if (a.scan_mode == DVL_SCAN_KAHAN_FP32)
        hipLaunchKernelGGL(k_carry<AccKahan32>, dim3(1), dim3(kCarryThreads), 0, s, a);
    else if (a.scan_mode == DVL_SCAN_NAIVE_FP32)
        hipLaunchKernelGGL(k_carry<AccF32>, dim3(1), dim3(kCarryThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_carry<AccF64>, dim3(1), dim3(kCarryThreads), 0, s, a);
    DVL_HIP(hipGetLastError());
    if (dvl_status st = mark(3)) return st;
    hipLaunchKernelGGL((k_bin<MT, S>), dim3(grid), dim3(kUpdThreads), lds, s, a);
    DVL_HIP(hipGetLastError());
    if (dvl_status st = mark(4)) return st;
    const unsigned g4 = (unsigned)((a.W + 3) / 4);
    hipLaunchKernelGGL((k_edges<MT>), dim3(g4), dim3(256), 0, s, a);
    DVL_HIP(hipGetLastError());
    return mark(5);
}

template <typename S>
static dvl_status launch_m(const UpdArgs& a, int n_cu, hipStream_t s, hipEvent_t* ev) {
    switch (a.M) {
        case 1: return launch_typed<1, S>(a, n_cu, s, ev);
        case 2: return launch_typed<2, S>(a, n_cu, s, ev);
        case 3: return launch_typed<3, S>(a, n_cu, s, ev);
        case 4: return launch_typed<4, S>(a, n_cu, s, ev);
        case 5: return launch_typed<5, S>(a, n_cu, s, ev);
        case 6: return launch_typed<6, S>(a, n_cu, s, ev);
        case 7: return launch_typed<7, S>(a, n_cu, s, ev);
        case 8: return launch_typed<8, S>(a, n_cu, s, ev);
        default: return launch_typed<16, S>(a, n_cu, s, ev);
    }
}

dvl_status launch_update(const UpdArgs& a, int n_cu, hipStream_t s, hipEvent_t* ev) {
    if (a.dtype == DVL_F16) return launch_m<F16>(a, n_cu, s, ev);
    if (a.dtype == DVL_BF16) return launch_m<BF16>(a, n_cu, s, ev);
    return launch_m<F32>(a, n_cu, s, ev);
}

}  // namespace dvl
