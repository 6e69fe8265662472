// C ABI of the DVL library: validation, buffer ownership, host-side TF
// preparation (Eqs. 5-6 run on the host, as in the paper's GPU section),
// batch planning and kernel launches.  Declarations and contracts:
// include/dvl.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "order.hpp"
#include "update.hpp"
#include "views.hpp"

namespace dvl {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

dvl_status hip_fail(hipError_t e, const char* what) {
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return DVL_E_HIP;
}

static dvl_status fail(dvl_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static int elem_bytes_of(int dtype) { return dtype == DVL_F32 ? 4 : 2; }

// Device memory of the library: through the caller's dvl_allocator when one
// was given, else hipMalloc / hipFree.  Every buffer is released through the
// allocator that made it.
struct Alloc {
    dvl_allocator a{};
    bool custom = false;
    void* get(size_t bytes, hipStream_t s) const {
        if (bytes == 0) bytes = 1;
        if (custom) return a.alloc(a.ctx, bytes, (void*)s);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p, hipStream_t s) const {
        if (!p) return;
        if (custom)
            a.release(a.ctx, p, (void*)s);
        else
            (void)hipFree(p);
    }
};

static dvl_status make_alloc(const dvl_allocator* a, Alloc& out) {
    out = Alloc();
    if (!a) return DVL_OK;
    if (!a->alloc || !a->release) return fail(DVL_E_INVALID, "allocator needs both alloc and release");
    out.a = *a;
    out.custom = true;
    return DVL_OK;
}

// device buffer owned by RAII until released
struct DevBuf {
    const Alloc* A;
    void* p = nullptr;
    explicit DevBuf(const Alloc& a) : A(&a) {}
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    // a buffer still owned here is a temporary or the leftover of a failing
    // call: kernels enqueued on it may still run, so wait before handing it back
    ~DevBuf() {
        if (p) {
            (void)hipDeviceSynchronize();
            A->put(p, nullptr);
        }
    }
    dvl_status alloc(size_t bytes, const char* what) {
        p = A->get(bytes, nullptr);
        if (!p) return fail(DVL_E_NOMEM, "device allocation of %zu bytes for %s failed", bytes, what);
        return DVL_OK;
    }
    void* release() { void* q = p; p = nullptr; return q; }
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// order-preserving uint key (as produced by the range kernel) back to float
static float unkey(unsigned int u) {
    const unsigned int b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    float f;
    memcpy(&f, &b, 4);
    return f;
}

constexpr int kRing = 4;                 // descriptor uploads that may be in flight
constexpr int kJobTfFloats = 32768;      // LDS budget of one job's tables (128 KB)

// The quantisers of every field: the TF entry of a cell depends on its value
// and on these only, not on the alpha tables.
struct CacheKey {
    int M = 0;
    int n_tf[kMaxFields] = {};
    float s[kMaxFields] = {}, b[kMaxFields] = {};
    float lo[kMaxFields] = {}, hi[kMaxFields] = {};   // the windows (informational, not compared)
    bool operator==(const CacheKey& o) const {
        return M == o.M && memcmp(n_tf, o.n_tf, sizeof n_tf) == 0 && memcmp(s, o.s, sizeof s) == 0 &&
               memcmp(b, o.b, sizeof b) == 0;
    }
};

// Uploads through kernel arguments (the allocation-free entry point): k_poke
// writes up to kPokeWords words carried in its arguments, in the stream's own
// queue (no memcpy or memset node).
constexpr int kPokeWords = 768;
struct PokeArgs {
    uint32_t* dst;
    uint32_t n;
    uint32_t w[kPokeWords];
};

__global__ __launch_bounds__(256) void k_poke(PokeArgs a) {
    for (uint32_t i = threadIdx.x; i < a.n; i += blockDim.x) a.dst[i] = a.w[i];
}

static dvl_status poke(char* dst, const char* src, size_t bytes, hipStream_t s) {
    const size_t nw = bytes / 4;
    PokeArgs a;
    for (size_t i = 0; i < nw; i += kPokeWords) {
        a.dst = reinterpret_cast<uint32_t*>(dst) + i;
        a.n = (uint32_t)std::min<size_t>(kPokeWords, nw - i);
        memcpy(a.w, src + 4 * i, (size_t)a.n * 4);
        hipLaunchKernelGGL(k_poke, dim3(1), dim3(256), 0, s, a);
        DVL_HIP(hipGetLastError());
    }
    return DVL_OK;
}

struct Executor;

}  // namespace dvl

using namespace dvl;

struct dvl_volume {
    int64_t n = 0;
    int64_t n_pad = 0;       // cells rounded up to whole tiles
    int64_t n_tiles = 0;
    int32_t tile_steps = kDefaultTileSteps;
    int64_t tiles_per_run = 1;
    int64_t n_runs = 1;
    int32_t M = 0;
    int32_t dtype = DVL_F32;
    int32_t bits = 0;
    int32_t max_level = 0;
    int device = 0;
    int n_cu = 256;
    uint8_t* level_s = nullptr;
    uint32_t* lcode_s = nullptr;      // per-step level codes [n_pad / 256]
    void* fields_s[kMaxFields] = {};
    uint64_t* keys_s = nullptr;
    uint32_t* perm = nullptr;
    float dmin[kMaxFields] = {};
    float dmax[kMaxFields] = {};
    // per-tile statistics of the sorted fields: sum [M][T], min [M][T], max [M][T],
    // and per 256-cell step: [M][S], S = T * tile_steps
    double* agg_sum = nullptr;
    float* agg_min = nullptr;
    float* agg_max = nullptr;
    double* step_sum = nullptr;
    float* step_min = nullptr;
    float* step_max = nullptr;
    // TF entry cache: one byte per sorted cell and field for one CacheKey
    // (policy DVL_ENTRY_CACHE_*); `cand` is the key of the last update that
    // could have used a cache, so a key seen twice in a row gets one
    uint8_t* idx_s[kMaxFields] = {};
    int32_t idx_policy = DVL_ENTRY_CACHE_AUTO;
    bool idx_valid = false;
    CacheKey idx_key;
    bool cand_set = false;
    CacheKey cand_key;
    // Ordering of cache rebuilds against the launches that read the cache,
    // by events instead of device synchronisation: a rebuild on stream s
    // first waits for the last reading launch on every stream; a launch that
    // reads the cache first waits for the rebuild (`cache_ready`).
    hipEvent_t cache_ready = nullptr;
    bool cache_ready_recorded = false;
    hipStream_t cache_ready_stream = nullptr;   // where the last rebuild ran
    std::vector<hipStream_t> cache_readers;     // streams whose launches read the cache
    // the volume's own transfer functions (used by dvl_update)
    bool tf_set[kMaxFields] = {};
    std::vector<float> alpha[kMaxFields];
    float lo[kMaxFields] = {}, hi[kMaxFields] = {};
    Executor* ex = nullptr;  // private executor of dvl_update
    dvl::Alloc alloc;        // every device buffer of the volume comes from here
    unsigned int* scratch_range = nullptr;   // 4 words for dvl_set_field's range check
    dvl_status sticky = DVL_OK;
    size_t bytes = 0;
};

namespace dvl {

// ================================================================== host TF prep

// FP32 quantiser of the window [lo, hi] for n_tf entries
static void quantiser(int n_tf, float lo, float hi, float* s, float* b) {
    const float sf = (float)((double)n_tf / ((double)hi - (double)lo));
    *s = sf;
    *b = (float)(-(double)lo * (double)sf);
}

static int host_entry(float x, float s, float b, int n_tf) {
    float t = fmaf(x, s, b);
    if (!(t >= 0.0f)) return 0;
    if (t > (float)(n_tf - 1)) return n_tf - 1;
    return (int)t;
}

// One update request as the host sees it: tables, windows, parameters, outputs.
struct ReqHost {
    dvl_volume* v = nullptr;
    int n_tf[kMaxFields] = {};       // entries of field m's table
    int off[kMaxFields] = {};        // start of field m's table in `alpha`
    int total = 0;                   // floats in `alpha`
    std::vector<float> alpha;        // tables, field after field
    float lo[kMaxFields] = {}, hi[kMaxFields] = {};
    float qs[kMaxFields] = {}, qb[kMaxFields] = {};
    dvl_params p{};
    dvl_bins out{};
    int job = 0;
    size_t tf_pos = 0;               // floats from the start of the batch's tables
};

// Eqs. 5-6 and the bound variant (section "Computing the Maximum Local
// Ensemble Variation"): max(V_h) from the TFs and the fields' data ranges
static float host_vmax(const ReqHost& r) {
    const dvl_volume* v = r.v;
    const int M = v->M;
    auto A = [&](int m, int a) { return r.alpha[(size_t)r.off[m] + std::min(a, r.n_tf[m] - 1)]; };
    int im[kMaxFields], jm[kMaxFields];
    for (int m = 0; m < M; ++m) {
        im[m] = host_entry(v->dmin[m], r.qs[m], r.qb[m], r.n_tf[m]);
        jm[m] = host_entry(v->dmax[m], r.qs[m], r.qb[m], r.n_tf[m]);
    }
    auto bound = [&]() {
        float hi = -INFINITY, lo = INFINITY;
        for (int m = 0; m < M; ++m)
            for (int a = im[m]; a <= jm[m]; ++a) {
                hi = std::max(hi, A(m, a));
                lo = std::min(lo, A(m, a));
            }
        return hi - lo;
    };
    if (r.p.vmax_mode == DVL_VMAX_TF_BOUND) return bound();
    int i = im[0], j = jm[0];
    for (int m = 1; m < M; ++m) { i = std::min(i, im[m]); j = std::max(j, jm[m]); }
    float best = 0.0f;
    for (int a = i; a <= j; ++a) {
        float hi = -INFINITY, lo = INFINITY;
        for (int m = 0; m < M; ++m) {
            hi = std::max(hi, A(m, a));
            lo = std::min(lo, A(m, a));
        }
        best = std::max(best, hi - lo);
    }
    if (best <= 0.0f) best = bound();   // the literal approximation can vanish (e.g. equal TFs)
    return best;
}

static dvl_status check_params(const dvl_params* p) {
    if (!p) return fail(DVL_E_INVALID, "params is NULL");
    if (p->n_bins < 1 || p->n_bins > (1 << 20)) return fail(DVL_E_INVALID, "n_bins=%d outside [1, 2^20]", p->n_bins);
    if (!(p->exponent >= 0.0f && p->exponent <= 16.0f)) return fail(DVL_E_INVALID, "exponent %g outside [0, 16]", p->exponent);
    if (!(p->min_importance >= 0.0f) || !isfinite(p->min_importance))
        return fail(DVL_E_INVALID, "min_importance %g must be finite and >= 0", p->min_importance);
    if (p->vmax_mode < 0 || p->vmax_mode > 2) return fail(DVL_E_INVALID, "vmax_mode %d", p->vmax_mode);
    if (p->clamp_mode < 0 || p->clamp_mode > 1) return fail(DVL_E_INVALID, "clamp_mode %d", p->clamp_mode);
    if (p->level_scale != 1 && p->level_scale != 3) return fail(DVL_E_INVALID, "level_scale %d (1 or 3)", p->level_scale);
    if (p->scan_mode < 0 || p->scan_mode > 2) return fail(DVL_E_INVALID, "scan_mode %d", p->scan_mode);
    return DVL_OK;
}

static dvl_status check_bins(const dvl_bins* b) {
    if (!b) return fail(DVL_E_INVALID, "bins is NULL");
    if (!b->first_cell || !b->last_cell || !b->mean || !b->vmin || !b->vmax || !b->y || !b->f_total ||
        !b->vmax_used)
        return fail(DVL_E_INVALID, "a bins pointer is NULL");
    return DVL_OK;
}

static dvl_status check_volume(const dvl_volume* v) {
    if (!v) return fail(DVL_E_INVALID, "volume is NULL");
    if (v->sticky != DVL_OK) return fail(v->sticky, "volume is in a failed state after an earlier device error");
    return DVL_OK;
}

// Resolve field m's window (NULL bounds: the data range), its quantiser, and
// check both are usable in fp32.
static dvl_status set_window(ReqHost& r, int m, const float* lo, const float* hi) {
    const dvl_volume* v = r.v;
    float l = lo ? lo[m] : v->dmin[m], h = hi ? hi[m] : v->dmax[m];
    if (!lo && !hi && !(h > l)) h = nextafterf(l, INFINITY);   // constant field
    if (!isfinite(l) || !isfinite(h) || !(l < h))
        return fail(DVL_E_INVALID, "window [%g, %g] of field %d is not finite with lo < hi", l, h, m);
    r.lo[m] = l;
    r.hi[m] = h;
    quantiser(r.n_tf[m], l, h, &r.qs[m], &r.qb[m]);
    if (!isfinite(r.qs[m]) || !isfinite(r.qb[m]))
        return fail(DVL_E_INVALID, "window [%g, %g] of field %d is too narrow for fp32", l, h, m);
    return DVL_OK;
}

static dvl_status check_tables(const ReqHost& r) {
    if (r.total > kMaxTfTotal) return fail(DVL_E_INVALID, "sum of TF sizes %d exceeds %d", r.total, kMaxTfTotal);
    for (float a : r.alpha)
        if (!isfinite(a)) return fail(DVL_E_INVALID, "an alpha entry is not finite");
    return DVL_OK;
}

// A request from caller inputs: alpha [M][n_tf], windows lo/hi [M] or NULL.
static dvl_status make_request(dvl_volume* v, const float* alpha, int n_tf, const float* lo, const float* hi,
                               const dvl_params* p, const dvl_bins* out, ReqHost& r) {
    if (dvl_status st = check_volume(v)) return st;
    if (dvl_status st = check_params(p)) return st;
    if (dvl_status st = check_bins(out)) return st;
    if (!alpha) return fail(DVL_E_INVALID, "alpha is NULL");
    if (n_tf < 2 || n_tf > kMaxTfEntries) return fail(DVL_E_INVALID, "n_tf=%d outside [2, %d]", n_tf, kMaxTfEntries);
    r = ReqHost();
    r.v = v;
    for (int m = 0; m < v->M; ++m) {
        r.n_tf[m] = n_tf;
        r.off[m] = m * n_tf;
    }
    r.total = v->M * n_tf;
    if (r.total > kMaxTfTotal) return fail(DVL_E_INVALID, "n_fields * n_tf = %d exceeds %d", r.total, kMaxTfTotal);
    r.alpha.assign(alpha, alpha + r.total);
    if (dvl_status st = check_tables(r)) return st;
    for (int m = 0; m < v->M; ++m)
        if (dvl_status st = set_window(r, m, lo, hi)) return st;
    r.p = *p;
    r.out = *out;
    return DVL_OK;
}

// A request from the volume's own TF state (dvl_set_tf).
static dvl_status volume_request(dvl_volume* v, const dvl_params* p, const dvl_bins* out, ReqHost& r) {
    if (dvl_status st = check_volume(v)) return st;
    for (int m = 0; m < v->M; ++m)
        if (!v->tf_set[m]) return fail(DVL_E_STATE, "field %d has no transfer function", m);
    if (dvl_status st = check_params(p)) return st;
    if (dvl_status st = check_bins(out)) return st;
    r = ReqHost();
    r.v = v;
    for (int m = 0; m < v->M; ++m) {
        r.n_tf[m] = (int)v->alpha[m].size();
        r.off[m] = r.total;
        r.total += r.n_tf[m];
        r.alpha.insert(r.alpha.end(), v->alpha[m].begin(), v->alpha[m].end());
        r.lo[m] = v->lo[m];
        r.hi[m] = v->hi[m];
        quantiser(r.n_tf[m], r.lo[m], r.hi[m], &r.qs[m], &r.qb[m]);
    }
    r.p = *p;
    r.out = *out;
    return DVL_OK;
}

// the largest importance a cell can reach, times a tile, must stay finite in fp32
static dvl_status check_range(const ReqHost& r, float vmax) {
    float amax = -INFINITY, amin = INFINITY;
    for (float a : r.alpha) { amax = std::max(amax, a); amin = std::min(amin, a); }
    const double vr = (double)amax - (double)amin;
    const bool exact = r.p.vmax_mode == DVL_VMAX_EXACT;
    const double rmax = exact ? 1.0 : (vmax > 0.0f ? vr / (double)vmax : 0.0);
    const double g = std::max((double)r.p.min_importance, rmax) * ldexp(1.0, r.p.level_scale * r.v->max_level);
    const double fmax_cell = std::max((double)r.p.min_importance, pow(g, (double)r.p.exponent));
    if (!(fmax_cell * (double)r.v->tile_steps * kStepCells < 1e37))
        return fail(DVL_E_RANGE, "importance can reach %g: exponent and levels overflow fp32", fmax_cell);
    return DVL_OK;
}

// ================================================================== batch plans

struct Plan {
    std::vector<ReqHost> reqs;       // grouped by volume
    std::vector<int> where;          // caller's request index -> index in `reqs`
    std::vector<JobDev> jobs;
    std::vector<ReqDev> rdev;
    int dtype = DVL_F32;
    int max_m = 1;
    int max_req = 1;
    int max_req_tf = 0;
    int max_job_tf = 0;
    int any_exact = 0;
    int64_t k1_units = 0, k3_units = 0, k4_units = 0;
    size_t tf_floats = 0;
    // descriptor block, uploaded before every launch:
    //   [header: 3 rescan counters][JobDev x jobs][ReqDev x reqs][max V x reqs][tables]
    // followed on the device (not uploaded) by the rescan queues [3][k3_units]
    size_t off_jobs = 0, off_reqs = 0, off_vmax = 0, off_tf = 0, block_bytes = 0;
    size_t off_queue = 0, device_bytes = 0;
};

// Group the requests into jobs (one volume; at most kMaxReqPerJob requests
// whose tables fit the importance pass's LDS) and lay out the work units of
// every phase and the descriptor block.
static dvl_status plan_batch(std::vector<ReqHost>&& reqs, Plan& P) {
    P = Plan();
    if (reqs.empty()) return fail(DVL_E_INVALID, "empty batch");
    P.dtype = reqs[0].v->dtype;
    for (auto& r : reqs)
        if (r.v->dtype != P.dtype) return fail(DVL_E_INVALID, "a batch mixes field storage types");
    std::vector<bool> taken(reqs.size(), false);
    P.where.assign(reqs.size(), 0);
    for (size_t i = 0; i < reqs.size(); ++i) {
        if (taken[i]) continue;
        for (size_t k = i; k < reqs.size(); ++k)
            if (!taken[k] && reqs[k].v == reqs[i].v) {
                P.where[k] = (int)P.reqs.size();
                P.reqs.push_back(std::move(reqs[k]));
                taken[k] = true;
            }
    }
    size_t tf_pos = 0;
    for (size_t i = 0; i < P.reqs.size();) {
        dvl_volume* v = P.reqs[i].v;
        JobDev j{};
        j.n = v->n;
        j.n_tiles = v->n_tiles;
        j.tiles_per_run = v->tiles_per_run;
        j.n_runs = v->n_runs;
        j.k1_unit0 = P.k1_units;
        j.M = v->M;
        j.req0 = (int)i;
        j.tile_steps = v->tile_steps;
        j.level = v->level_s;
        j.lcode = v->lcode_s;
        for (int m = 0; m < v->M; ++m) j.fields[m] = v->fields_s[m];
        j.agg_sum = v->agg_sum;
        j.agg_min = v->agg_min;
        j.agg_max = v->agg_max;
        j.step_sum = v->step_sum;
        j.step_min = v->step_min;
        j.step_max = v->step_max;
        int tf_job = 0;
        size_t k = i;
        while (k < P.reqs.size() && P.reqs[k].v == v && (int)(k - i) < kMaxReqPerJob &&
               (k == i || tf_job + P.reqs[k].total <= kJobTfFloats)) {
            ReqHost& r = P.reqs[k];
            r.job = (int)P.jobs.size();
            r.tf_pos = tf_pos;
            tf_pos += r.total;
            tf_job += r.total;
            P.max_req_tf = std::max(P.max_req_tf, r.total);
            if (r.p.vmax_mode == DVL_VMAX_EXACT) P.any_exact = 1;
            ++k;
        }
        j.n_req = (int)(k - i);
        j.tf_total_all = tf_job;
        P.max_job_tf = std::max(P.max_job_tf, tf_job);
        P.max_m = std::max(P.max_m, v->M);
        P.max_req = std::max(P.max_req, j.n_req);
        // one importance-pass unit is one workgroup: a run per wave
        P.k1_units += (j.n_runs + (kUpdThreads / kWave) - 1) / (kUpdThreads / kWave);
        P.jobs.push_back(j);
        i = k;
    }
    // The kernels are specialised on the field count: batches whose volumes
    // all have M <= 8 fields run the M-field variant; batches that mix field
    // counts (or have more than 8) run the general one, which reads M per job.
    for (const JobDev& j : P.jobs)
        if (j.M != P.jobs[0].M) P.max_m = kMaxFields;
    if (P.max_m > 8) P.max_m = kMaxFields;
    P.tf_floats = tf_pos;
    P.rdev.resize(P.reqs.size());
    for (size_t q = 0; q < P.reqs.size(); ++q) {
        const ReqHost& r = P.reqs[q];
        const JobDev& j = P.jobs[r.job];
        ReqDev& d = P.rdev[q];
        d = ReqDev{};
        for (int m = 0; m < r.v->M; ++m) {
            d.nmax[m] = (float)(r.n_tf[m] - 1);
            d.tf_off[m] = r.off[m];
        }
        d.tf_job_off = (int)(r.tf_pos - P.reqs[j.req0].tf_pos);
        d.tf_total = r.total;
        d.W = r.p.n_bins;
        d.exponent = r.p.exponent;
        d.fmin = r.p.min_importance;
        d.exp_is_one = r.p.exponent == 1.0f;
        d.clamp_mode = r.p.clamp_mode;
        d.level_shift = r.p.level_scale;
        d.scan_mode = r.p.scan_mode;
        d.vmax_exact = r.p.vmax_mode == DVL_VMAX_EXACT;
        d.job = r.job;
        d.k3_unit0 = P.k3_units;
        d.k4_unit0 = P.k4_units;
        P.k3_units += j.n_tiles;
        P.k4_units += r.p.n_bins;
        d.first_cell = r.out.first_cell;
        d.last_cell = r.out.last_cell;
        d.mean = r.out.mean;
        d.vmin = r.out.vmin;
        d.vmax = r.out.vmax;
        d.y = r.out.y;
        d.f_total = r.out.f_total;
        d.vmax_used = r.out.vmax_used;
    }
    P.off_jobs = 256 + al256(P.rdev.size() * sizeof(uint32_t));   // counters, then carry flags
    P.off_reqs = P.off_jobs + al256(P.jobs.size() * sizeof(JobDev));
    P.off_vmax = P.off_reqs + al256(P.rdev.size() * sizeof(ReqDev));
    P.off_tf = P.off_vmax + al256(P.rdev.size() * sizeof(float));
    P.block_bytes = P.off_tf + al256(P.tf_floats * sizeof(float));
    P.off_queue = P.block_bytes;
    P.device_bytes = P.off_queue + al256((size_t)3 * P.k3_units * sizeof(uint64_t));
    return DVL_OK;
}

// Write the descriptor block into host image `h` for device address `d`:
// current tables and quantisers, max(V) of the TF modes (0 for the exact
// mode, which the first kernel raises with atomics), pointers into the block.
static dvl_status fill_block(Plan& P, char* h, char* d) {
    float* vmax_h = (float*)(h + P.off_vmax);
    float* tf_h = (float*)(h + P.off_tf);
    for (size_t q = 0; q < P.reqs.size(); ++q) {
        ReqHost& r = P.reqs[q];
        const float vm = r.p.vmax_mode == DVL_VMAX_EXACT ? 0.0f : host_vmax(r);
        if (dvl_status st = check_range(r, vm)) return st;
        vmax_h[q] = vm;
        memcpy(tf_h + r.tf_pos, r.alpha.data(), r.alpha.size() * sizeof(float));
        for (int m = 0; m < r.v->M; ++m) {
            P.rdev[q].s[m] = r.qs[m];
            P.rdev[q].b[m] = r.qb[m];
        }
        P.rdev[q].tf = (const float*)(d + P.off_tf) + r.tf_pos;
        P.rdev[q].vmax_dev = (float*)(d + P.off_vmax) + q;
    }
    for (auto& j : P.jobs) j.tf_all = (const float*)(d + P.off_tf) + P.reqs[j.req0].tf_pos;
    memset(h, 0, P.off_jobs);   // rescan counters and carry flags start at 0
    memcpy(h + P.off_jobs, P.jobs.data(), P.jobs.size() * sizeof(JobDev));
    memcpy(h + P.off_reqs, P.rdev.data(), P.rdev.size() * sizeof(ReqDev));
    return DVL_OK;
}

// The entry-cache key of a request, if its tables fit in a byte index.
static bool key_of(const ReqHost& r, CacheKey& k) {
    k = CacheKey();
    k.M = r.v->M;
    for (int m = 0; m < r.v->M; ++m) {
        if (r.n_tf[m] > 256) return false;
        k.n_tf[m] = r.n_tf[m];
        k.s[m] = r.qs[m];
        k.b[m] = r.qb[m];
        k.lo[m] = r.lo[m];
        k.hi[m] = r.hi[m];
    }
    return true;
}

struct CacheBuild {
    dvl_volume* v;
    CacheKey key;
};

// Choose, per job, between reading the field values and reading the
// volume's TF entry cache; schedule the cache (re)builds this launch needs.
// A job reads the cache if all its requests share one key and the cache holds
// it (or is built for it now).  One volume's cache serves one key per launch.
static dvl_status decide_cache(Plan& P, std::vector<CacheBuild>& builds) {
    builds.clear();
    std::vector<std::pair<dvl_volume*, CacheKey>> serving;   // cache contents per volume in this launch
    for (JobDev& j : P.jobs) {
        for (int m = 0; m < kMaxFields; ++m) j.idx[m] = nullptr;
        dvl_volume* v = P.reqs[j.req0].v;
        if (v->idx_policy == DVL_ENTRY_CACHE_NEVER) continue;
        CacheKey key;
        bool agree = key_of(P.reqs[j.req0], key);
        for (int k = 1; agree && k < j.n_req; ++k) {
            CacheKey k2;
            agree = key_of(P.reqs[j.req0 + k], k2) && k2 == key;
        }
        if (!agree) continue;
        auto it = std::find_if(serving.begin(), serving.end(), [&](const auto& e) { return e.first == v; });
        bool use = false;
        if (it != serving.end()) {
            use = it->second == key;            // another key already serves this launch: values
        } else if (v->idx_valid && v->idx_key == key) {
            use = true;
        } else if (v->idx_policy == DVL_ENTRY_CACHE_ALWAYS || (v->cand_set && v->cand_key == key)) {
            for (int m = 0; m < v->M; ++m) {
                if (v->idx_s[m]) continue;
                DevBuf b(v->alloc);
                if (dvl_status st = b.alloc((size_t)v->n_pad, "TF entry cache")) return st;
                v->idx_s[m] = (uint8_t*)b.release();
                v->bytes += (size_t)v->n_pad;
            }
            builds.push_back({v, key});
            use = true;
        } else {
            v->cand_key = key;
            v->cand_set = true;
        }
        if (use) {
            if (it == serving.end()) serving.push_back({v, key});
            for (int m = 0; m < v->M; ++m) j.idx[m] = v->idx_s[m];
        }
    }
    return DVL_OK;
}

// Rebuild the scheduled caches on stream s.  Launches on other streams may
// still read a cache and later launches on any stream must see the new one;
// both are ordered by events (see dvl_volume::cache_readers), so the host
// never waits here.
// One reader event per (device, stream), shared by every volume: re-recorded
// after each launch on that stream that reads an entry cache.  A rebuild
// waits for the latest record on each other reader stream, which follows
// every earlier launch there (stream order): one record per launch instead
// of one per volume, each of which is a queue packet.  The events live until
// the process ends.
struct ReaderEvent {
    int dev;
    hipStream_t s;
    hipEvent_t ev;
};
static std::mutex g_reader_mu;
static std::vector<ReaderEvent> g_readers;

static dvl_status reader_event(hipStream_t s, bool create, hipEvent_t* out) {
    *out = nullptr;
    int dev = -1;
    DVL_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_reader_mu);
    for (const ReaderEvent& r : g_readers)
        if (r.dev == dev && r.s == s) {
            *out = r.ev;
            return DVL_OK;
        }
    if (!create) return DVL_OK;
    hipEvent_t ev = nullptr;
    DVL_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    g_readers.push_back({dev, s, ev});
    *out = ev;
    return DVL_OK;
}

static dvl_status run_cache_builds(const std::vector<CacheBuild>& builds, hipStream_t s) {
    for (const CacheBuild& cb : builds) {
        dvl_volume* v = cb.v;
        for (hipStream_t r : v->cache_readers) {
            if (r == s) continue;
            hipEvent_t ev = nullptr;
            if (dvl_status st = reader_event(r, false, &ev)) return st;
            if (ev) DVL_HIP(hipStreamWaitEvent(s, ev, 0));
        }
        v->idx_valid = false;
        for (int m = 0; m < v->M; ++m)
            if (dvl_status st = launch_build_index(v->n_pad, v->dtype, v->fields_s[m], cb.key.s[m], cb.key.b[m],
                                                   cb.key.n_tf[m], v->idx_s[m], v->n_cu, s))
                return st;
        DVL_HIP(hipEventRecord(v->cache_ready, s));
        v->cache_ready_recorded = true;
        v->cache_ready_stream = s;
        v->idx_key = cb.key;
        v->idx_valid = true;
        v->cand_set = false;
    }
    return DVL_OK;
}

// Before a launch on stream s that reads the caches of the jobs in `P`: wait
// for their latest rebuild when it ran on another stream (on s itself the
// stream order already follows it).
static dvl_status cache_wait(const Plan& P, hipStream_t s) {
    for (const JobDev& j : P.jobs) {
        if (!j.idx[0]) continue;
        dvl_volume* v = P.reqs[j.req0].v;
        if (v->cache_ready_recorded && v->cache_ready_stream != s)
            DVL_HIP(hipStreamWaitEvent(s, v->cache_ready, 0));
    }
    return DVL_OK;
}

// After such a launch: s is a reader stream of those volumes (returns
// whether any job read a cache).  The caller records s's reader event.
static bool cache_add_readers(const Plan& P, hipStream_t s) {
    bool any = false;
    for (const JobDev& j : P.jobs) {
        if (!j.idx[0]) continue;
        dvl_volume* v = P.reqs[j.req0].v;
        if (std::find(v->cache_readers.begin(), v->cache_readers.end(), s) == v->cache_readers.end())
            v->cache_readers.push_back(s);
        any = true;
    }
    return any;
}

// ... and records its reader event once when one did
static dvl_status cache_mark_readers(const Plan& P, hipStream_t s) {
    if (!cache_add_readers(P, s)) return DVL_OK;
    hipEvent_t ev = nullptr;
    if (dvl_status st = reader_event(s, true, &ev)) return st;
    DVL_HIP(hipEventRecord(ev, s));
    return DVL_OK;
}

// polls of a request's carry flag before a classifying workgroup computes the
// carry itself (dvl_set_carry_wait)
static std::atomic<int> g_carry_wait_polls{kCarryWaitPolls};

// `paths`: importance-pass variants to launch (a captured graph takes both,
// since its jobs choose at every launch)
static BatchDev batch_dev(const Plan& P, char* d, int paths) {
    BatchDev b{};
    b.paths = paths;
    b.jobs = (const JobDev*)(d + P.off_jobs);
    b.reqs = (const ReqDev*)(d + P.off_reqs);
    b.rescan_count = (uint32_t*)d;
    b.carry_ready = (uint32_t*)(d + 256);
    b.rescan_queue = (uint64_t*)(d + P.off_queue);
    b.n_jobs = (int)P.jobs.size();
    b.n_reqs = (int)P.rdev.size();
    b.k1_units = P.k1_units;
    b.k3_units = P.k3_units;
    b.k4_units = P.k4_units;
    b.any_exact = P.any_exact;
    b.max_req_tf = P.max_req_tf;
    b.max_job_tf = P.max_job_tf;
    b.max_req_job = P.max_req;
    b.max_tile_steps = 8;
    b.carry_wait_polls = g_carry_wait_polls.load(std::memory_order_relaxed);
    for (const JobDev& j : P.jobs) b.max_tile_steps = std::max(b.max_tile_steps, j.tile_steps);
    return b;
}

static int64_t fstore_cells(const dvl_volume* v, int n_bins) {
    return wants_fstore(v->n_tiles, n_bins) ? v->n_pad : 0;
}
static size_t request_ws_bytes(const dvl_volume* v, int n_bins) {
    return workspace_bytes(v->n_tiles, v->M, n_bins, fstore_cells(v, n_bins));
}

// ================================================================== executor

struct Executor {
    int n_cu = 256;
    Alloc alloc;                    // workspaces and descriptor blocks
    // The descriptor block: one device buffer, rewritten before each launch.
    // Launches on one stream run in order, so a launch rewrites the block
    // only after the previous launch's kernels have read it.  Blocks of up
    // to kPokeMaxBytes (a few requests) are written by k_poke from a host
    // image carried in kernel arguments: no staging buffer whose reuse the
    // host would have to wait for, and no event.  Larger ones (a batch of
    // many requests: tens of KB of tables) are copied from a ring of pinned
    // staging buffers, each released by an event after its copy.
    static constexpr size_t kPokeMaxBytes = (size_t)4 * kPokeWords * 4;
    char* blk = nullptr;
    size_t blk_cap = 0;
    std::vector<char> img;
    struct Staging {
        char* host = nullptr;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool used = false;
    };
    Staging ring[kRing];
    int next = 0;
    std::vector<std::pair<void*, size_t>> ws;   // workspace pool: one per request position
    // The end of the latest launch is marked by the reader event of its
    // stream (reader_event), recorded after every launch: it serves the
    // entry-cache ordering and this executor alike, one queue packet.
    hipStream_t last_stream = nullptr;
    bool launched = false;
    int timing = 0;                 // 0 off, 1 every phase, 2 the importance pass only
    std::vector<std::vector<hipEvent_t>> ev_pool, ev_pending;
    std::vector<int> ev_mode;       // the timing mode of each pending event set
    std::vector<hipEvent_t> ev_sel; // the events handed to the launcher (unused phases NULL)
    double phase_ms[kPhases] = {};
    int32_t timed = 0;
    size_t bytes = 0;

    ~Executor() {
        (void)hipDeviceSynchronize();
        alloc.put(blk, nullptr);
        for (auto& r : ring) {
            if (r.host) (void)hipHostFree(r.host);
            if (r.ev) (void)hipEventDestroy(r.ev);
        }
        for (auto& w : ws) alloc.put(w.first, nullptr);
        for (auto* pool : {&ev_pool, &ev_pending})
            for (auto& set : *pool)
                for (auto e : set) (void)hipEventDestroy(e);
    }

    dvl_status init() {
        int dev = 0;
        DVL_HIP(hipGetDevice(&dev));
        DVL_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        return DVL_OK;
    }

    // the end of the latest launch (the reader event of its stream, recorded
    // after it or after later work on that stream)
    dvl_status last_event(hipEvent_t* ev) {
        *ev = nullptr;
        if (!launched) return DVL_OK;
        return reader_event(last_stream, false, ev);
    }

    // the executor's earlier launches are the only users of its buffers:
    // waiting for the latest one frees them for reuse
    dvl_status wait_idle() {
        hipEvent_t ev = nullptr;
        if (dvl_status st = last_event(&ev)) return st;
        if (ev) DVL_HIP(hipEventSynchronize(ev));
        return DVL_OK;
    }

    // grow workspace i to `need` bytes; if the allocation fails the old
    // workspace stays, so smaller requests keep working
    dvl_status ensure_ws(size_t i, size_t need) {
        if (ws.size() <= i) ws.resize(i + 1, {nullptr, 0});
        if (ws[i].second >= need) return DVL_OK;
        DevBuf b(alloc);
        if (dvl_status st = b.alloc(need, "request workspace")) return st;
        if (ws[i].first) {
            if (dvl_status st = wait_idle()) return st;
            alloc.put(ws[i].first, nullptr);
            bytes -= ws[i].second;
        }
        ws[i] = {b.release(), need};
        bytes += need;
        return DVL_OK;
    }

    // a descriptor block of at least `need` device bytes (the uploaded image
    // is a prefix of them); the old block is released once the launches that
    // read it are done
    dvl_status ensure_block(size_t need) {
        if (blk_cap >= need) return DVL_OK;
        const size_t cap = std::max(need * 2, (size_t)65536);
        DevBuf d(alloc);
        if (dvl_status st = d.alloc(cap, "batch descriptors")) return st;
        if (blk) {
            if (dvl_status st = wait_idle()) return st;
            alloc.put(blk, nullptr);
            bytes -= blk_cap;
        }
        blk = (char*)d.release();
        blk_cap = cap;
        bytes += cap;
        return DVL_OK;
    }

    // the next pinned staging buffer, its previous copy complete, of at
    // least `need` bytes
    dvl_status take_staging(size_t need, Staging** out) {
        Staging& r = ring[next];
        next = (next + 1) % kRing;
        if (!r.ev) DVL_HIP(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
        if (r.used) DVL_HIP(hipEventSynchronize(r.ev));
        if (r.cap < need) {
            const size_t cap = std::max(need * 2, (size_t)65536);
            char* host = nullptr;
            if (hipHostMalloc((void**)&host, cap, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(DVL_E_NOMEM, "pinned host allocation of %zu bytes failed", cap);
            }
            if (r.host) (void)hipHostFree(r.host);
            r.host = host;
            r.cap = cap;
        }
        *out = &r;
        return DVL_OK;
    }

    // write the plan's descriptor block into blk on stream s
    dvl_status upload(Plan& P, hipStream_t s) {
        if (P.block_bytes <= kPokeMaxBytes) {
            img.resize(P.block_bytes);
            if (dvl_status st = fill_block(P, img.data(), blk)) return st;
            return poke(blk, img.data(), P.block_bytes, s);
        }
        Staging* r = nullptr;
        if (dvl_status st = take_staging(P.block_bytes, &r)) return st;
        if (dvl_status st = fill_block(P, r->host, blk)) return st;
        DVL_HIP(hipMemcpyAsync(blk, r->host, P.block_bytes, hipMemcpyHostToDevice, s));
        DVL_HIP(hipEventRecord(r->ev, s));
        r->used = true;
        return DVL_OK;
    }

    dvl_status timing_events(hipEvent_t** out) {
        *out = nullptr;
        if (!timing) return DVL_OK;
        if (ev_pool.empty()) {
            std::vector<hipEvent_t> set(kPhases + 1, nullptr);
            for (auto& e : set)
                if (hipError_t err = hipEventCreate(&e)) {
                    for (auto x : set)
                        if (x) (void)hipEventDestroy(x);
                    return hip_fail(err, "hipEventCreate");
                }
            ev_pool.push_back(set);
        }
        ev_pending.push_back(ev_pool.back());
        ev_pool.pop_back();
        ev_mode.push_back(timing);
        ev_sel.assign(kPhases + 1, nullptr);
        for (int p = 0; p <= kPhases; ++p)
            if (timing == 1 || p == 1 || p == 2) ev_sel[p] = ev_pending.back()[p];
        *out = ev_sel.data();
        return DVL_OK;
    }

    dvl_status run(Plan& P, hipStream_t s) {
        for (size_t q = 0; q < P.reqs.size(); ++q) {
            const ReqHost& r = P.reqs[q];
            if (dvl_status st = ensure_ws(q, request_ws_bytes(r.v, r.p.n_bins))) return st;
            workspace_carve(ws[q].first, r.v->n_tiles, r.v->M, r.p.n_bins, fstore_cells(r.v, r.p.n_bins), &P.rdev[q].ws);
        }
        std::vector<CacheBuild> builds;
        if (dvl_status st = decide_cache(P, builds)) return st;
        if (dvl_status st = run_cache_builds(builds, s)) return st;
        if (dvl_status st = cache_wait(P, s)) return st;
        if (dvl_status st = ensure_block(P.device_bytes)) return st;
        // a launch on another stream than the previous one first waits for it
        // (it may still read the block and the workspaces)
        if (launched && s != last_stream) {
            hipEvent_t prev = nullptr;
            if (dvl_status st = last_event(&prev)) return st;
            if (prev) DVL_HIP(hipStreamWaitEvent(s, prev, 0));
        }
        if (dvl_status st = upload(P, s)) return st;
        hipEvent_t* ev = nullptr;
        if (dvl_status st = timing_events(&ev)) return st;
        int paths = 0;
        for (const JobDev& j : P.jobs) paths |= j.idx[0] ? kPathEntries : kPathValues;
        for (const ReqDev& d : P.rdev)
            if (d.ws.fstore) paths |= kPathStoredF;
        if (dvl_status st = launch_batch(batch_dev(P, blk, paths), P.dtype, P.max_m, P.max_req, n_cu, s, kDescriptorLayout, ev))
            return st;
        cache_add_readers(P, s);
        hipEvent_t done = nullptr;
        if (dvl_status st = reader_event(s, true, &done)) return st;
        DVL_HIP(hipEventRecord(done, s));
        last_stream = s;
        launched = true;
        return DVL_OK;
    }

    dvl_status kernel_times(double* ms, int32_t* n) {
        for (size_t i = 0; i < ev_pending.size(); ++i) {
            auto& set = ev_pending[i];
            const bool all = ev_mode[i] == 1;
            DVL_HIP(hipEventSynchronize(set[all ? kPhases : 2]));
            for (int p = all ? 0 : 1; p < (all ? kPhases : 2); ++p) {
                float t = 0.0f;
                DVL_HIP(hipEventElapsedTime(&t, set[p], set[p + 1]));
                phase_ms[p] += t;
            }
            timed += 1;
            ev_pool.push_back(set);
        }
        ev_pending.clear();
        ev_mode.clear();
        if (ms)
            for (int p = 0; p < kPhases; ++p) ms[p] = phase_ms[p];
        if (n) *n = timed;
        for (int p = 0; p < kPhases; ++p) phase_ms[p] = 0.0;
        timed = 0;
        return DVL_OK;
    }
};

static dvl_status new_executor(const Alloc& a, Executor** out) {
    Executor* ex = new (std::nothrow) Executor();
    if (!ex) return fail(DVL_E_NOMEM, "host allocation failed");
    ex->alloc = a;
    if (dvl_status st = ex->init()) {
        delete ex;
        return st;
    }
    *out = ex;
    return DVL_OK;
}

static dvl_status requests_from(const dvl_request* reqs, int32_t n, std::vector<ReqHost>& out) {
    if (!reqs || n < 1) return fail(DVL_E_INVALID, "no requests");
    out.resize(n);
    for (int i = 0; i < n; ++i) {
        const dvl_request& r = reqs[i];
        if (dvl_status st = make_request(r.volume, r.alpha, r.n_tf, r.lo, r.hi, &r.params, &r.out, out[i])) {
            const std::string msg = g_err;
            return fail(st, "request %d: %s", i, msg.c_str());
        }
    }
    return DVL_OK;
}

}  // namespace dvl

// ================================================================== graphs

struct dvl_graph {
    Plan plan;
    Alloc alloc;                         // the first request's volume's allocator
    int n_cu = 256;
    // two descriptor blocks, each read by its own captured graphs; launches
    // alternate between them, so consecutive replays are different
    // executable graphs (one executable graph is not replayed while its
    // previous launch may still run)
    static constexpr int kSlots = 2;
    char* dev[kSlots] = {};
    int launches = 0;
    std::vector<void*> ws;               // one workspace per request
    char* host[kRing] = {};              // pinned staging of the descriptor block
    hipEvent_t ev[kRing] = {};
    bool used[kRing] = {};
    int next = 0;
    // one captured graph per set of projection paths (values, cached
    // entries, stored f): a replay launches only the kernel variants its jobs
    // use, and the set can change between launches as entry caches appear
    struct Captured {
        int paths;
        int slot;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Captured> captured;
    ~dvl_graph() {
        (void)hipDeviceSynchronize();
        for (auto& c : captured) {
            if (c.exec) (void)hipGraphExecDestroy(c.exec);
            if (c.graph) (void)hipGraphDestroy(c.graph);
        }
        for (char* d : dev) alloc.put(d, nullptr);
        for (void* w : ws) alloc.put(w, nullptr);
        for (int r = 0; r < kRing; ++r) {
            if (host[r]) (void)hipHostFree(host[r]);
            if (ev[r]) (void)hipEventDestroy(ev[r]);
        }
    }
};

// per-tile and per-step statistics of sorted field m
static dvl_status tile_aggregates(dvl_volume* v, int m, hipStream_t s) {
    const size_t ot = (size_t)m * v->n_tiles, os = ot * v->tile_steps;
    return launch_tile_aggregates(v->n, v->dtype, v->fields_s[m], v->n_tiles, v->tile_steps, v->agg_sum + ot,
                                  v->agg_min + ot, v->agg_max + ot, v->step_sum + os, v->step_min + os,
                                  v->step_max + os, v->n_cu, s);
}

extern "C" {

const char* dvl_last_error(void) { return g_err.c_str(); }

size_t dvl_update_workspace_bytes(int64_t n_cells, int32_t n_fields, int32_t n_bins) {
    if (n_cells < 1 || n_fields < 1 || n_bins < 1) return 0;
    const int64_t cells = (int64_t)kDefaultTileSteps * kStepCells;
    const int64_t T = (n_cells + cells - 1) / cells;
    return workspace_bytes(T, n_fields, n_bins, wants_fstore(T, n_bins) ? T * cells : 0);
}

size_t dvl_request_bytes(const dvl_volume* v, int32_t n_bins) {
    if (!v || n_bins < 1) return 0;
    // workspace + outputs (first/last, mean/min/max/y per field, two scalars)
    return request_ws_bytes(v, n_bins) + (size_t)n_bins * (8 + 16 * (size_t)v->M) + 16;
}

dvl_status dvl_build_order_ex(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                              const uint8_t* level, int32_t M, int32_t dtype, const void* const* fields,
                              const dvl_build_options* opt, void* stream, dvl_volume** out) {
    g_err.clear();
    if (!out) return fail(DVL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(DVL_E_INVALID, "n_cells=%lld outside [1, 2^32)", (long long)n);
    if (M < 1 || M > kMaxFields) return fail(DVL_E_INVALID, "n_fields=%d outside [1, %d]", M, kMaxFields);
    if (dtype != DVL_F32 && dtype != DVL_F16 && dtype != DVL_BF16) return fail(DVL_E_INVALID, "unknown dtype %d", dtype);
    if (!x || !y || !z || !level || !fields) return fail(DVL_E_INVALID, "NULL input pointer");
    for (int m = 0; m < M; ++m)
        if (!fields[m]) return fail(DVL_E_INVALID, "field %d pointer is NULL", m);
    int tile_steps = kDefaultTileSteps, run_waves = 0, entry_cache = DVL_ENTRY_CACHE_AUTO;
    Alloc alloc;
    if (opt) {
        if (dvl_status st = make_alloc(opt->allocator, alloc)) return st;
        if (opt->entry_cache < DVL_ENTRY_CACHE_AUTO || opt->entry_cache > DVL_ENTRY_CACHE_NEVER)
            return fail(DVL_E_INVALID, "entry_cache %d", opt->entry_cache);
        entry_cache = opt->entry_cache;
        if (opt->tile_steps != 0 && opt->tile_steps != 8 && opt->tile_steps != 16 && opt->tile_steps != 32)
            return fail(DVL_E_INVALID, "tile_steps %d (0, 8, 16 or 32)", opt->tile_steps);
        if (opt->run_waves != 0 && (opt->run_waves < 64 || opt->run_waves > 65536))
            return fail(DVL_E_INVALID, "run_waves %d outside [64, 65536]", opt->run_waves);
        if (opt->tile_steps) tile_steps = opt->tile_steps;
        run_waves = opt->run_waves;
    }
    hipStream_t s = (hipStream_t)stream;
    const int eb = elem_bytes_of(dtype);

    dvl_volume* v = new (std::nothrow) dvl_volume();
    if (!v) return fail(DVL_E_NOMEM, "host allocation failed");
    struct Guard { dvl_volume* v; ~Guard() { if (v) dvl_destroy(v); } } guard{v};
    v->alloc = alloc;
    const Alloc& A = v->alloc;
    v->n = n;
    v->M = M;
    v->dtype = dtype;
    v->tile_steps = tile_steps;
    v->idx_policy = entry_cache;
    const int64_t tile_cells = (int64_t)tile_steps * kStepCells;
    v->n_tiles = (n + tile_cells - 1) / tile_cells;
    v->n_pad = v->n_tiles * tile_cells;
    DVL_HIP(hipGetDevice(&v->device));
    DVL_HIP(hipDeviceGetAttribute(&v->n_cu, hipDeviceAttributeMultiprocessorCount, v->device));
    {
        // runs of consecutive tiles, one per wave of the importance pass; the
        // default (32 per compute unit) is two rounds of resident waves: a
        // wave that finishes early takes another run, which evens out the
        // finishing times of the compute units
        const int64_t waves = run_waves ? run_waves : (int64_t)v->n_cu * 32;
        v->tiles_per_run = std::max<int64_t>(1, (v->n_tiles + waves - 1) / waves);
        v->n_runs = (v->n_tiles + v->tiles_per_run - 1) / v->tiles_per_run;
    }

    // extent, validity, grid bits
    DevBuf ext(A);
    if (dvl_status st = ext.alloc(4 * sizeof(unsigned long long), "extent")) return st;
    DVL_HIP(hipMemsetAsync(ext.p, 0, 4 * sizeof(unsigned long long), s));
    if (dvl_status st = launch_extent(n, x, y, z, level, (unsigned long long*)ext.p, s)) return st;
    unsigned long long eh[4] = {};
    DVL_HIP(hipMemcpyAsync(eh, ext.p, sizeof eh, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (eh[1]) return fail(DVL_E_RANGE, "a cell has a negative corner or a level above 20");
    int bits = 1;
    while (((unsigned long long)1 << bits) < eh[0]) ++bits;
    if (bits > 21) return fail(DVL_E_RANGE, "logical grid extent %llu exceeds 2^21 per axis", eh[0]);
    v->bits = bits;
    v->max_level = (int)eh[2];

    // keys + sort
    DevBuf ka(A), kb(A), va(A), vb(A), counts(A), partial(A);
    if (dvl_status st = ka.alloc((size_t)n * 8, "keys")) return st;
    if (dvl_status st = kb.alloc((size_t)n * 8, "keys (sort buffer)")) return st;
    if (dvl_status st = va.alloc((size_t)n * 4, "permutation")) return st;
    if (dvl_status st = vb.alloc((size_t)n * 4, "permutation (sort buffer)")) return st;
    const int64_t n_counts = 256 * sort_tile_count(n);
    if (dvl_status st = counts.alloc((size_t)n_counts * 4, "sort counts")) return st;
    if (dvl_status st = partial.alloc((size_t)scan_partial_count(n_counts) * 4 + 16, "scan partials")) return st;
    if (dvl_status st = launch_keys(n, x, y, z, level, bits, (uint64_t*)ka.p, (uint32_t*)va.p, s)) return st;
    uint64_t* ksorted = nullptr;
    uint32_t* vsorted = nullptr;
    if (dvl_status st = radix_sort(n, 3 * bits, (uint64_t*)ka.p, (uint32_t*)va.p, (uint64_t*)kb.p,
                                   (uint32_t*)vb.p, (uint32_t*)counts.p, (uint32_t*)partial.p, s,
                                   &ksorted, &vsorted))
        return st;
    DVL_HIP(hipMemsetAsync(ext.p, 0, 4 * sizeof(unsigned long long), s));
    if (dvl_status st = launch_dup(n, ksorted, (unsigned long long*)ext.p, s)) return st;
    DVL_HIP(hipMemcpyAsync(eh, ext.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (eh[0]) return fail(DVL_E_OVERLAP, "two cells share a Hilbert key (overlapping AMR cells)");
    // keep the sorted pair, free the other
    if (ksorted == ka.p) { v->keys_s = (uint64_t*)ka.release(); } else { v->keys_s = (uint64_t*)kb.release(); }
    if (vsorted == va.p) { v->perm = (uint32_t*)va.release(); } else { v->perm = (uint32_t*)vb.release(); }
    v->bytes += (size_t)n * 12;

    // gather into sorted order (padded to whole tiles, padding zeroed)
    DevBuf lv(A);
    if (dvl_status st = lv.alloc((size_t)v->n_pad, "sorted levels")) return st;
    DVL_HIP(hipMemsetAsync((char*)lv.p + n, 0, (size_t)(v->n_pad - n), s));
    if (dvl_status st = launch_gather(n, v->perm, level, lv.p, 1, s)) return st;
    v->level_s = (uint8_t*)lv.release();
    v->bytes += (size_t)v->n_pad;
    {
        DevBuf lc(A);
        const int64_t n_steps = v->n_pad / kStepCells;
        if (dvl_status st = lc.alloc((size_t)n_steps * 4, "level codes")) return st;
        if (dvl_status st = launch_level_codes(v->level_s, n_steps, (uint32_t*)lc.p, s)) return st;
        v->lcode_s = (uint32_t*)lc.release();
        v->bytes += (size_t)n_steps * 4;
    }
    DevBuf rng(A);
    if (dvl_status st = rng.alloc((size_t)kMaxFields * 4 * sizeof(unsigned int), "ranges")) return st;
    std::vector<unsigned int> rinit(kMaxFields * 4, 0u);
    for (int m = 0; m < kMaxFields; ++m) rinit[m * 4] = 0xFFFFFFFFu;
    DVL_HIP(hipMemcpyAsync(rng.p, rinit.data(), rinit.size() * 4, hipMemcpyHostToDevice, s));
    for (int m = 0; m < M; ++m) {
        DevBuf fb(A);
        if (dvl_status st = fb.alloc((size_t)v->n_pad * eb, "sorted field")) return st;
        DVL_HIP(hipMemsetAsync((char*)fb.p + (size_t)n * eb, 0, (size_t)(v->n_pad - n) * eb, s));
        if (dvl_status st = launch_gather_range(n, v->perm, dtype, fields[m], fb.p, (unsigned int*)rng.p + 4 * m, s))
            return st;
        v->fields_s[m] = fb.release();
        v->bytes += (size_t)v->n_pad * eb;
    }
    {
        DevBuf as(A), an(A), ax(A), ss(A), sn(A), sx(A);
        const size_t mt = (size_t)M * v->n_tiles;
        const size_t ms = mt * v->tile_steps;
        if (dvl_status st = as.alloc(mt * 8, "tile sums")) return st;
        if (dvl_status st = an.alloc(mt * 4, "tile minima")) return st;
        if (dvl_status st = ax.alloc(mt * 4, "tile maxima")) return st;
        if (dvl_status st = ss.alloc(ms * 8, "step sums")) return st;
        if (dvl_status st = sn.alloc(ms * 4, "step minima")) return st;
        if (dvl_status st = sx.alloc(ms * 4, "step maxima")) return st;
        v->agg_sum = (double*)as.release();
        v->agg_min = (float*)an.release();
        v->agg_max = (float*)ax.release();
        v->step_sum = (double*)ss.release();
        v->step_min = (float*)sn.release();
        v->step_max = (float*)sx.release();
        v->bytes += (mt + ms) * 16;
        for (int m = 0; m < M; ++m)
            if (dvl_status st = tile_aggregates(v, m, s)) return st;
    }
    DVL_HIP(hipMemcpyAsync(rinit.data(), rng.p, rinit.size() * 4, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < M; ++m) {
        if (rinit[m * 4 + 2]) return fail(DVL_E_RANGE, "field %d holds a NaN", m);
        v->dmin[m] = unkey(rinit[m * 4]);
        v->dmax[m] = unkey(rinit[m * 4 + 1]);
    }

    {
        DevBuf sr(A);
        if (dvl_status st = sr.alloc(4 * sizeof(unsigned int), "range scratch")) return st;
        v->scratch_range = (unsigned int*)sr.release();
        v->bytes += 4 * sizeof(unsigned int);
    }
    DVL_HIP(hipEventCreateWithFlags(&v->cache_ready, hipEventDisableTiming));

    // private executor of dvl_update, with the workspace of one request ready
    if (dvl_status st = new_executor(A, &v->ex)) return st;
    if (dvl_status st = v->ex->ensure_ws(0, request_ws_bytes(v, 1))) return st;
    guard.v = nullptr;
    *out = v;
    return DVL_OK;
}

dvl_status dvl_build_order(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                           const uint8_t* level, int32_t M, int32_t dtype, const void* const* fields,
                           void* stream, dvl_volume** out) {
    return dvl_build_order_ex(n, x, y, z, level, M, dtype, fields, nullptr, stream, out);
}

dvl_status dvl_set_field(dvl_volume* v, int32_t m, const void* values, void* stream) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (m < 0 || m >= v->M) return fail(DVL_E_INVALID, "field index %d outside [0, %d)", m, v->M);
    if (!values) return fail(DVL_E_INVALID, "values is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int eb = elem_bytes_of(v->dtype);
    // The data range (and the NaN check) does not depend on the order, so it
    // is taken from the new values as given, before anything of the volume
    // changes: a rejected field leaves the volume as it was.
    unsigned int r[4] = {0xFFFFFFFFu, 0u, 0u, 0u};
    DVL_HIP(hipMemcpyAsync(v->scratch_range, r, sizeof r, hipMemcpyHostToDevice, s));
    if (dvl_status st = launch_range(v->n, v->dtype, values, v->scratch_range, s)) return st;
    DVL_HIP(hipMemcpyAsync(r, v->scratch_range, sizeof r, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (r[2]) return fail(DVL_E_RANGE, "field %d holds a NaN; the volume is unchanged", m);
    v->idx_valid = false;      // the cached entries describe the old values
    v->cand_set = false;
    if (dvl_status st = launch_gather(v->n, v->perm, values, v->fields_s[m], eb, s)) {
        v->sticky = st;
        return st;
    }
    if (dvl_status st = tile_aggregates(v, m, s)) {
        v->sticky = st;
        return st;
    }
    v->dmin[m] = unkey(r[0]);
    v->dmax[m] = unkey(r[1]);
    return DVL_OK;
}

dvl_status dvl_field_range(const dvl_volume* v, int32_t m, float* vmin, float* vmax) {
    g_err.clear();
    if (!v) return fail(DVL_E_INVALID, "volume is NULL");
    if (m < 0 || m >= v->M) return fail(DVL_E_INVALID, "field index %d outside [0, %d)", m, v->M);
    if (vmin) *vmin = v->dmin[m];
    if (vmax) *vmax = v->dmax[m];
    return DVL_OK;
}

dvl_status dvl_set_tf(dvl_volume* v, int32_t m, const float* alpha, int32_t n_tf, float lo, float hi) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (m < 0 || m >= v->M) return fail(DVL_E_INVALID, "field index %d outside [0, %d)", m, v->M);
    if (!alpha) return fail(DVL_E_INVALID, "alpha is NULL");
    if (n_tf < 2 || n_tf > kMaxTfEntries) return fail(DVL_E_INVALID, "n_tf=%d outside [2, %d]", n_tf, kMaxTfEntries);
    if (!isfinite(lo) || !isfinite(hi) || !(lo < hi)) return fail(DVL_E_INVALID, "window [%g, %g] is not finite with lo < hi", lo, hi);
    size_t total = n_tf;
    for (int q = 0; q < v->M; ++q)
        if (q != m && v->tf_set[q]) total += v->alpha[q].size();
    if (total > (size_t)kMaxTfTotal) return fail(DVL_E_INVALID, "sum of TF sizes %zu exceeds %d", total, kMaxTfTotal);
    for (int i = 0; i < n_tf; ++i)
        if (!isfinite(alpha[i])) return fail(DVL_E_INVALID, "alpha[%d] is not finite", i);
    float s, b;
    quantiser(n_tf, lo, hi, &s, &b);
    if (!isfinite(s) || !isfinite(b)) return fail(DVL_E_INVALID, "window [%g, %g] is too narrow for fp32", lo, hi);
    v->alpha[m].assign(alpha, alpha + n_tf);
    v->lo[m] = lo;
    v->hi[m] = hi;
    v->tf_set[m] = true;
    return DVL_OK;
}

dvl_status dvl_update(dvl_volume* v, const dvl_params* p, const dvl_bins* out, void* stream) {
    g_err.clear();
    std::vector<ReqHost> reqs(1);
    if (dvl_status st = volume_request(v, p, out, reqs[0])) return st;
    Plan P;
    if (dvl_status st = plan_batch(std::move(reqs), P)) return st;
    const dvl_status st = v->ex->run(P, (hipStream_t)stream);
    if (st == DVL_E_HIP) v->sticky = st;
    return st;
}

// ------------------------------------------------------------------ allocation-free update

}  // extern "C"

namespace dvl {

// The fixed device scratch of dvl_update_noalloc: the descriptor block
// (descriptors, tables, rescan queues) followed by the request workspace.
// Every call on a device shares its copy.  In host code `scratch` names a
// host-side stand-in, never the device memory: its device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_dev[kMaxDevices] = {};

// device address of this device's scratch (the device must be current)
static dvl_status scratch_address(int dev, char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return fail(DVL_E_INVALID, "device %d outside [0, %d)", dev, kMaxDevices);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = (char*)p;
    }
    *out = g_scratch_dev[dev];
    return DVL_OK;
}

// Upload of a host image into device memory through kernel arguments (the
// runtime copies them at launch): no staging buffer, no memcpy node.

// A job reads the volume's entry cache here only when the cache already holds
// its key (it is never built here) and this stream is already one of the
// volume's reader streams (its reader event exists and is re-recorded below,
// creating nothing), so a later rebuild elsewhere still waits for this launch.
static void use_existing_cache(Plan& P, hipStream_t s) {
    for (JobDev& j : P.jobs) {
        for (int m = 0; m < kMaxFields; ++m) j.idx[m] = nullptr;
        dvl_volume* v = P.reqs[j.req0].v;
        if (v->idx_policy == DVL_ENTRY_CACHE_NEVER || !v->idx_valid) continue;
        CacheKey key;
        if (!key_of(P.reqs[j.req0], key) || !(key == v->idx_key)) continue;
        if (std::find(v->cache_readers.begin(), v->cache_readers.end(), s) == v->cache_readers.end()) continue;
        for (int m = 0; m < v->M; ++m) j.idx[m] = v->idx_s[m];
    }
}

}  // namespace dvl

extern "C" {

dvl_status dvl_update_noalloc(dvl_volume* v, const dvl_params* p, const dvl_bins* out, void* stream) {
    g_err.clear();
    std::vector<ReqHost> reqs(1);
    if (dvl_status st = volume_request(v, p, out, reqs[0])) return st;
    int dev = -1;
    DVL_HIP(hipGetDevice(&dev));
    if (dev != v->device) return fail(DVL_E_INVALID, "volume lives on device %d, device %d is current", v->device, dev);
    hipStream_t s = (hipStream_t)stream;
    Plan P;
    if (dvl_status st = plan_batch(std::move(reqs), P)) return st;
    const size_t block = al256(P.device_bytes);
    const size_t need = block + workspace_bytes(v->n_tiles, v->M, p->n_bins, 0);
    if (need > kScratchBytes)
        return fail(DVL_E_NOMEM, "this update needs %zu bytes of scratch; dvl_update_noalloc has %zu "
                    "(use dvl_update)", need, kScratchBytes);
    char* base = nullptr;
    if (dvl_status st = scratch_address(dev, &base)) return st;
    workspace_carve(base + block, v->n_tiles, v->M, p->n_bins, 0, &P.rdev[0].ws);
    use_existing_cache(P, s);
    if (dvl_status st = cache_wait(P, s)) return st;
    std::vector<char> img(P.block_bytes);
    if (dvl_status st = fill_block(P, img.data(), base)) return st;
    if (dvl_status st = poke(base, img.data(), P.block_bytes, s)) {
        v->sticky = st;
        return st;
    }
    int paths = 0;
    for (const JobDev& j : P.jobs) paths |= j.idx[0] ? kPathEntries : kPathValues;
    if (dvl_status st = launch_batch(batch_dev(P, base, paths), P.dtype, P.max_m, P.max_req, v->n_cu, s, kDescriptorLayout, nullptr)) {
        if (st == DVL_E_HIP) v->sticky = st;
        return st;
    }
    for (const JobDev& j : P.jobs)
        if (j.idx[0]) {
            hipEvent_t ev = nullptr;   // exists: s is a reader stream of the volume
            if (dvl_status st = reader_event(s, false, &ev)) return st;
            if (ev) DVL_HIP(hipEventRecord(ev, s));
            break;
        }
    return DVL_OK;
}

size_t dvl_update_noalloc_max_bytes(void) { return kScratchBytes; }

dvl_status dvl_set_carry_wait(int32_t polls) {
    g_err.clear();
    if (polls < 0) return fail(DVL_E_INVALID, "polls %d < 0", (int)polls);
    g_carry_wait_polls.store(polls, std::memory_order_relaxed);
    return DVL_OK;
}

dvl_status dvl_read_bins(const dvl_volume* v, const dvl_bins* b, int32_t W, void* stream, uint32_t* count,
                         uint32_t* first, uint32_t* last, float* mean, float* vmin, float* vmax, float* y,
                         double* f_total, float* vmax_used) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (!b) return fail(DVL_E_INVALID, "bins is NULL");
    if (W < 1 || W > (1 << 20)) return fail(DVL_E_INVALID, "n_bins=%d outside [1, 2^20]", W);
    hipStream_t s = (hipStream_t)stream;
    DVL_HIP(hipStreamSynchronize(s));
    const size_t mw = (size_t)v->M * W;
    std::vector<uint32_t> f_tmp, l_tmp;
    uint32_t* fh = first;
    uint32_t* lh = last;
    if (count && !fh) { f_tmp.resize(W); fh = f_tmp.data(); }
    if (count && !lh) { l_tmp.resize(W); lh = l_tmp.data(); }
    if (fh) DVL_HIP(hipMemcpy(fh, b->first_cell, (size_t)W * 4, hipMemcpyDeviceToHost));
    if (lh) DVL_HIP(hipMemcpy(lh, b->last_cell, (size_t)W * 4, hipMemcpyDeviceToHost));
    if (count)
        for (int i = 0; i < W; ++i) count[i] = (fh[i] == 0xFFFFFFFFu) ? 0u : lh[i] - fh[i] + 1u;
    if (mean) DVL_HIP(hipMemcpy(mean, b->mean, mw * 4, hipMemcpyDeviceToHost));
    if (vmin) DVL_HIP(hipMemcpy(vmin, b->vmin, mw * 4, hipMemcpyDeviceToHost));
    if (vmax) DVL_HIP(hipMemcpy(vmax, b->vmax, mw * 4, hipMemcpyDeviceToHost));
    if (y) DVL_HIP(hipMemcpy(y, b->y, mw * 4, hipMemcpyDeviceToHost));
    if (f_total) DVL_HIP(hipMemcpy(f_total, b->f_total, 8, hipMemcpyDeviceToHost));
    if (vmax_used) DVL_HIP(hipMemcpy(vmax_used, b->vmax_used, 4, hipMemcpyDeviceToHost));
    return DVL_OK;
}

dvl_status dvl_export_order(const dvl_volume* v, uint64_t* keys, uint32_t* perm, void* stream) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (keys) {
        if (dvl_status st = launch_scatter_back(v->n, v->perm, v->keys_s, keys, 8, s)) return st;
    }
    if (perm) DVL_HIP(hipMemcpyAsync(perm, v->perm, (size_t)v->n * 4, hipMemcpyDeviceToDevice, s));
    return DVL_OK;
}

dvl_status dvl_export_sorted(const dvl_volume* v, uint8_t* level, void* const* fields, void* stream) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (level) DVL_HIP(hipMemcpyAsync(level, v->level_s, (size_t)v->n, hipMemcpyDeviceToDevice, s));
    if (fields) {
        const size_t eb = elem_bytes_of(v->dtype);
        for (int m = 0; m < v->M; ++m)
            if (fields[m]) DVL_HIP(hipMemcpyAsync(fields[m], v->fields_s[m], (size_t)v->n * eb, hipMemcpyDeviceToDevice, s));
    }
    return DVL_OK;
}

// ------------------------------------------------------------------ bin views, brushing, zoom

static dvl_status check_bins_of(const dvl_volume* v, const dvl_bins* b, int32_t W) {
    if (dvl_status st = check_volume(v)) return st;
    if (!b || !b->first_cell || !b->last_cell) return fail(DVL_E_INVALID, "bins is NULL or lacks first/last");
    if (W < 1 || W > (1 << 20)) return fail(DVL_E_INVALID, "n_bins=%d outside [1, 2^20]", W);
    return DVL_OK;
}

dvl_status dvl_select_bins(const dvl_volume* v, const dvl_bins* bins, int32_t W, int32_t b0, int32_t b1,
                           void* stream, uint32_t* first, uint32_t* last, uint64_t* key_lo, uint64_t* key_hi) {
    g_err.clear();
    if (dvl_status st = check_bins_of(v, bins, W)) return st;
    if (b0 < 0 || b1 < b0 || b1 >= W) return fail(DVL_E_INVALID, "bin range [%d, %d] outside [0, %d)", b0, b1, W);
    hipStream_t s = (hipStream_t)stream;
    uint32_t f = 0, l = 0;
    DVL_HIP(hipMemcpyAsync(&f, bins->first_cell + b0, 4, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipMemcpyAsync(&l, bins->last_cell + b1, 4, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (f > l || (int64_t)l >= v->n) return fail(DVL_E_STATE, "the bins do not hold a cell range of this volume");
    uint64_t klo = 0, khi = 0;
    DVL_HIP(hipMemcpyAsync(&klo, v->keys_s + f, 8, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipMemcpyAsync(&khi, v->keys_s + l, 8, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (first) *first = f;
    if (last) *last = l;
    if (key_lo) *key_lo = klo;
    if (key_hi) *key_hi = khi;
    return DVL_OK;
}

dvl_status dvl_select_mask(const dvl_volume* v, const uint64_t* ranges, int32_t n_ranges, uint8_t* mask,
                           void* stream) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (n_ranges < 1 || n_ranges > kMaxSelectRanges)
        return fail(DVL_E_INVALID, "n_ranges=%d outside [1, %d]", n_ranges, kMaxSelectRanges);
    if (!ranges || !mask) return fail(DVL_E_INVALID, "ranges or mask is NULL");
    for (int i = 0; i < n_ranges; ++i)
        if (ranges[2 * i] > ranges[2 * i + 1]) return fail(DVL_E_INVALID, "range %d has lo > hi", i);
    return launch_select_mask(v->n, v->keys_s, v->perm, n_ranges, ranges, mask, (hipStream_t)stream);
}

dvl_status dvl_bin_histograms(const dvl_volume* v, const dvl_bins* bins, int32_t W, int32_t m, int32_t n_buckets,
                              float lo, float hi, uint32_t* counts, void* stream) {
    g_err.clear();
    if (dvl_status st = check_bins_of(v, bins, W)) return st;
    if (m < 0 || m >= v->M) return fail(DVL_E_INVALID, "field index %d outside [0, %d)", m, v->M);
    if (n_buckets < 1 || n_buckets > kMaxTfEntries)
        return fail(DVL_E_INVALID, "n_buckets=%d outside [1, %d]", n_buckets, kMaxTfEntries);
    if (!counts) return fail(DVL_E_INVALID, "counts is NULL");
    if (!isfinite(lo) || !isfinite(hi) || !(lo < hi)) return fail(DVL_E_INVALID, "window [%g, %g] is not finite with lo < hi", lo, hi);
    float qs, qb;
    quantiser(n_buckets, lo, hi, &qs, &qb);
    if (!isfinite(qs) || !isfinite(qb)) return fail(DVL_E_INVALID, "window [%g, %g] is too narrow for fp32", lo, hi);
    return launch_bin_histograms(v->dtype, v->fields_s[m], W, bins->first_cell, bins->last_cell, n_buckets, qs, qb,
                                 counts, v->n_cu, (hipStream_t)stream);
}

dvl_status dvl_rasterize(const float* y, int32_t n_lines, int32_t W, int32_t n_rows, int32_t mode, uint8_t* image,
                         void* stream) {
    g_err.clear();
    if (!y || !image) return fail(DVL_E_INVALID, "y or image is NULL");
    if (n_lines < 1 || n_lines > kMaxFields) return fail(DVL_E_INVALID, "n_lines=%d outside [1, %d]", n_lines, kMaxFields);
    if (W < 1 || W > (1 << 20)) return fail(DVL_E_INVALID, "n_bins=%d outside [1, 2^20]", W);
    if (n_rows < 1 || n_rows > 16384) return fail(DVL_E_INVALID, "n_rows=%d outside [1, 16384]", n_rows);
    if (mode != DVL_RASTER_POLYLINE && mode != DVL_RASTER_BARS) return fail(DVL_E_INVALID, "raster mode %d", mode);
    return launch_rasterize(y, W, n_rows, n_lines, mode, image, (hipStream_t)stream);
}

dvl_status dvl_zoom(const dvl_volume* v, uint32_t first, uint32_t last, const dvl_build_options* opt, void* stream,
                    dvl_volume** out) {
    g_err.clear();
    if (!out) return fail(DVL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (dvl_status st = check_volume(v)) return st;
    if (first > last || (int64_t)last >= v->n)
        return fail(DVL_E_INVALID, "cell range [%u, %u] outside [0, %lld)", first, last, (long long)v->n);
    int tile_steps = kDefaultTileSteps, run_waves = 0, entry_cache = DVL_ENTRY_CACHE_AUTO;
    Alloc alloc = v->alloc;
    if (opt) {
        if (opt->allocator)
            if (dvl_status st = make_alloc(opt->allocator, alloc)) return st;
        if (opt->entry_cache < DVL_ENTRY_CACHE_AUTO || opt->entry_cache > DVL_ENTRY_CACHE_NEVER)
            return fail(DVL_E_INVALID, "entry_cache %d", opt->entry_cache);
        if (opt->tile_steps != 0 && opt->tile_steps != 8 && opt->tile_steps != 16 && opt->tile_steps != 32)
            return fail(DVL_E_INVALID, "tile_steps %d (0, 8, 16 or 32)", opt->tile_steps);
        if (opt->run_waves != 0 && (opt->run_waves < 64 || opt->run_waves > 65536))
            return fail(DVL_E_INVALID, "run_waves %d outside [64, 65536]", opt->run_waves);
        entry_cache = opt->entry_cache;
        if (opt->tile_steps) tile_steps = opt->tile_steps;
        run_waves = opt->run_waves;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)last - first + 1;
    const int eb = elem_bytes_of(v->dtype);
    dvl_volume* z = new (std::nothrow) dvl_volume();
    if (!z) return fail(DVL_E_NOMEM, "host allocation failed");
    struct Guard { dvl_volume* v; ~Guard() { if (v) dvl_destroy(v); } } guard{z};
    z->alloc = alloc;
    const Alloc& A = z->alloc;
    z->n = n;
    z->M = v->M;
    z->dtype = v->dtype;
    z->bits = v->bits;
    z->max_level = v->max_level;
    z->device = v->device;
    z->n_cu = v->n_cu;
    z->tile_steps = tile_steps;
    z->idx_policy = entry_cache;
    const int64_t tile_cells = (int64_t)tile_steps * kStepCells;
    z->n_tiles = (n + tile_cells - 1) / tile_cells;
    z->n_pad = z->n_tiles * tile_cells;
    {
        const int64_t waves = run_waves ? run_waves : (int64_t)z->n_cu * 32;
        z->tiles_per_run = std::max<int64_t>(1, (z->n_tiles + waves - 1) / waves);
        z->n_runs = (z->n_tiles + z->tiles_per_run - 1) / z->tiles_per_run;
    }
    // the range's keys, an identity permutation (its original order is the range)
    {
        DevBuf kb(A), pb(A);
        if (dvl_status st = kb.alloc((size_t)n * 8, "keys")) return st;
        if (dvl_status st = pb.alloc((size_t)n * 4, "permutation")) return st;
        DVL_HIP(hipMemcpyAsync(kb.p, v->keys_s + first, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
        if (dvl_status st = launch_iota(n, (uint32_t*)pb.p, s)) return st;
        z->keys_s = (uint64_t*)kb.release();
        z->perm = (uint32_t*)pb.release();
        z->bytes += (size_t)n * 12;
    }
    {
        DevBuf lv(A);
        if (dvl_status st = lv.alloc((size_t)z->n_pad, "sorted levels")) return st;
        DVL_HIP(hipMemsetAsync((char*)lv.p + n, 0, (size_t)(z->n_pad - n), s));
        DVL_HIP(hipMemcpyAsync(lv.p, v->level_s + first, (size_t)n, hipMemcpyDeviceToDevice, s));
        z->level_s = (uint8_t*)lv.release();
        z->bytes += (size_t)z->n_pad;
        DevBuf lc(A);
        const int64_t n_steps = z->n_pad / kStepCells;
        if (dvl_status st = lc.alloc((size_t)n_steps * 4, "level codes")) return st;
        if (dvl_status st = launch_level_codes(z->level_s, n_steps, (uint32_t*)lc.p, s)) return st;
        z->lcode_s = (uint32_t*)lc.release();
        z->bytes += (size_t)n_steps * 4;
    }
    DevBuf rng(A);
    if (dvl_status st = rng.alloc((size_t)kMaxFields * 4 * sizeof(unsigned int), "ranges")) return st;
    std::vector<unsigned int> rinit(kMaxFields * 4, 0u);
    for (int m = 0; m < kMaxFields; ++m) rinit[m * 4] = 0xFFFFFFFFu;
    DVL_HIP(hipMemcpyAsync(rng.p, rinit.data(), rinit.size() * 4, hipMemcpyHostToDevice, s));
    for (int m = 0; m < z->M; ++m) {
        DevBuf fb(A);
        if (dvl_status st = fb.alloc((size_t)z->n_pad * eb, "sorted field")) return st;
        DVL_HIP(hipMemsetAsync((char*)fb.p + (size_t)n * eb, 0, (size_t)(z->n_pad - n) * eb, s));
        DVL_HIP(hipMemcpyAsync(fb.p, (const char*)v->fields_s[m] + (size_t)first * eb, (size_t)n * eb,
                               hipMemcpyDeviceToDevice, s));
        if (dvl_status st = launch_range(n, z->dtype, fb.p, (unsigned int*)rng.p + 4 * m, s)) return st;
        z->fields_s[m] = fb.release();
        z->bytes += (size_t)z->n_pad * eb;
    }
    {
        DevBuf as(A), an(A), ax(A), ss(A), sn(A), sx(A);
        const size_t mt = (size_t)z->M * z->n_tiles;
        const size_t ms = mt * z->tile_steps;
        if (dvl_status st = as.alloc(mt * 8, "tile sums")) return st;
        if (dvl_status st = an.alloc(mt * 4, "tile minima")) return st;
        if (dvl_status st = ax.alloc(mt * 4, "tile maxima")) return st;
        if (dvl_status st = ss.alloc(ms * 8, "step sums")) return st;
        if (dvl_status st = sn.alloc(ms * 4, "step minima")) return st;
        if (dvl_status st = sx.alloc(ms * 4, "step maxima")) return st;
        z->agg_sum = (double*)as.release();
        z->agg_min = (float*)an.release();
        z->agg_max = (float*)ax.release();
        z->step_sum = (double*)ss.release();
        z->step_min = (float*)sn.release();
        z->step_max = (float*)sx.release();
        z->bytes += (mt + ms) * 16;
        for (int m = 0; m < z->M; ++m)
            if (dvl_status st = tile_aggregates(z, m, s)) return st;
    }
    DVL_HIP(hipMemcpyAsync(rinit.data(), rng.p, rinit.size() * 4, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < z->M; ++m) {
        z->dmin[m] = unkey(rinit[m * 4]);
        z->dmax[m] = unkey(rinit[m * 4 + 1]);
    }
    {
        DevBuf sr(A);
        if (dvl_status st = sr.alloc(4 * sizeof(unsigned int), "range scratch")) return st;
        z->scratch_range = (unsigned int*)sr.release();
        z->bytes += 4 * sizeof(unsigned int);
    }
    DVL_HIP(hipEventCreateWithFlags(&z->cache_ready, hipEventDisableTiming));
    if (dvl_status st = new_executor(A, &z->ex)) return st;
    if (dvl_status st = z->ex->ensure_ws(0, request_ws_bytes(z, 1))) return st;
    guard.v = nullptr;
    *out = z;
    return DVL_OK;
}

dvl_status dvl_set_timing(dvl_volume* v, int32_t enable) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (enable < 0 || enable > 2) return fail(DVL_E_INVALID, "timing mode %d (0, 1 or 2)", (int)enable);
    v->ex->timing = enable;
    return DVL_OK;
}

dvl_status dvl_kernel_times(dvl_volume* v, double* ms, int32_t* n_updates) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    return v->ex->kernel_times(ms, n_updates);
}

dvl_status dvl_set_entry_cache(dvl_volume* v, int32_t policy) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    if (policy < DVL_ENTRY_CACHE_AUTO || policy > DVL_ENTRY_CACHE_NEVER)
        return fail(DVL_E_INVALID, "entry_cache %d", policy);
    v->idx_policy = policy;
    if (policy == DVL_ENTRY_CACHE_NEVER) {
        DVL_HIP(hipDeviceSynchronize());   // queued updates may still read it
        for (int m = 0; m < kMaxFields; ++m) {
            if (!v->idx_s[m]) continue;
            v->alloc.put(v->idx_s[m], nullptr);
            v->idx_s[m] = nullptr;
            v->bytes -= (size_t)v->n_pad;
        }
        v->idx_valid = false;
        v->cand_set = false;
    }
    return DVL_OK;
}

int32_t dvl_entry_cache_info(const dvl_volume* v, float* lo, float* hi, int32_t* n_tf) {
    if (!v || !v->idx_valid) return 0;
    for (int m = 0; m < v->M; ++m) {
        if (lo) lo[m] = v->idx_key.lo[m];
        if (hi) hi[m] = v->idx_key.hi[m];
        if (n_tf) n_tf[m] = v->idx_key.n_tf[m];
    }
    return 1;
}

int64_t dvl_num_cells(const dvl_volume* v) { return v ? v->n : 0; }
int32_t dvl_num_fields(const dvl_volume* v) { return v ? v->M : 0; }
int32_t dvl_grid_bits(const dvl_volume* v) { return v ? v->bits : 0; }
int32_t dvl_dtype(const dvl_volume* v) { return v ? v->dtype : -1; }
size_t dvl_volume_bytes(const dvl_volume* v) { return v ? v->bytes + (v->ex ? v->ex->bytes : 0) : 0; }

dvl_status dvl_level_segments(const dvl_volume* v, int64_t* n_segments, int64_t* n_mixed) {
    g_err.clear();
    if (dvl_status st = check_volume(v)) return st;
    const int64_t n_steps = v->n_pad / kStepCells;
    std::vector<uint32_t> codes((size_t)n_steps);
    DVL_HIP(hipDeviceSynchronize());
    DVL_HIP(hipMemcpy(codes.data(), v->lcode_s, (size_t)n_steps * 4, hipMemcpyDeviceToHost));
    int64_t mixed = 0;
    for (uint32_t c : codes)
        for (int k = 0; k < 4; ++k) mixed += ((c >> (8 * k)) & 0xFFu) == 0xFFu;
    if (n_segments) *n_segments = n_steps * 4;
    if (n_mixed) *n_mixed = mixed;
    return DVL_OK;
}

void dvl_destroy(dvl_volume* v) {
    if (!v) return;
    (void)hipDeviceSynchronize();
    delete v->ex;
    const Alloc& A = v->alloc;
    A.put(v->level_s, nullptr);
    A.put(v->lcode_s, nullptr);
    for (int m = 0; m < kMaxFields; ++m) A.put(v->fields_s[m], nullptr);
    A.put(v->keys_s, nullptr);
    A.put(v->perm, nullptr);
    A.put(v->agg_sum, nullptr);
    A.put(v->agg_min, nullptr);
    A.put(v->agg_max, nullptr);
    A.put(v->step_sum, nullptr);
    A.put(v->step_min, nullptr);
    A.put(v->step_max, nullptr);
    A.put(v->scratch_range, nullptr);
    for (int m = 0; m < kMaxFields; ++m) A.put(v->idx_s[m], nullptr);
    if (v->cache_ready) (void)hipEventDestroy(v->cache_ready);
    delete v;
}


// ------------------------------------------------------------------ executors and batches

dvl_status dvl_executor_create_ex(const dvl_allocator* allocator, dvl_executor** out) {
    g_err.clear();
    if (!out) return fail(DVL_E_INVALID, "out is NULL");
    *out = nullptr;
    Alloc a;
    if (dvl_status st = make_alloc(allocator, a)) return st;
    Executor* ex = nullptr;
    if (dvl_status st = new_executor(a, &ex)) return st;
    *out = reinterpret_cast<dvl_executor*>(ex);
    return DVL_OK;
}

dvl_status dvl_executor_create(dvl_executor** out) { return dvl_executor_create_ex(nullptr, out); }

void dvl_executor_destroy(dvl_executor* ex) { delete reinterpret_cast<Executor*>(ex); }

size_t dvl_executor_bytes(const dvl_executor* ex) {
    return ex ? reinterpret_cast<const Executor*>(ex)->bytes : 0;
}

dvl_status dvl_executor_set_timing(dvl_executor* ex, int32_t enable) {
    g_err.clear();
    if (!ex) return fail(DVL_E_INVALID, "executor is NULL");
    if (enable < 0 || enable > 2) return fail(DVL_E_INVALID, "timing mode %d (0, 1 or 2)", (int)enable);
    reinterpret_cast<Executor*>(ex)->timing = enable;
    return DVL_OK;
}

dvl_status dvl_executor_kernel_times(dvl_executor* ex, double* ms, int32_t* n) {
    g_err.clear();
    if (!ex) return fail(DVL_E_INVALID, "executor is NULL");
    return reinterpret_cast<Executor*>(ex)->kernel_times(ms, n);
}

dvl_status dvl_update_batch(dvl_executor* exh, const dvl_request* reqs, int32_t n_reqs, void* stream) {
    g_err.clear();
    if (!exh) return fail(DVL_E_INVALID, "executor is NULL");
    std::vector<ReqHost> rh;
    if (dvl_status st = requests_from(reqs, n_reqs, rh)) return st;
    Plan P;
    if (dvl_status st = plan_batch(std::move(rh), P)) return st;
    return reinterpret_cast<Executor*>(exh)->run(P, (hipStream_t)stream);
}

dvl_status dvl_graph_create(const dvl_request* reqs, int32_t n_reqs, dvl_graph** out) {
    g_err.clear();
    if (!out) return fail(DVL_E_INVALID, "out is NULL");
    *out = nullptr;
    std::vector<ReqHost> rh;
    if (dvl_status st = requests_from(reqs, n_reqs, rh)) return st;
    dvl_graph* g = new (std::nothrow) dvl_graph();
    if (!g) return fail(DVL_E_NOMEM, "host allocation failed");
    struct Guard { dvl_graph* g; ~Guard() { delete g; } } guard{g};
    if (dvl_status st = plan_batch(std::move(rh), g->plan)) return st;
    Plan& P = g->plan;
    g->alloc = P.reqs[0].v->alloc;
    int dev = 0;
    DVL_HIP(hipGetDevice(&dev));
    DVL_HIP(hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    for (size_t q = 0; q < P.reqs.size(); ++q) {
        DevBuf w(g->alloc);
        const ReqHost& r = P.reqs[q];
        if (dvl_status st = w.alloc(request_ws_bytes(r.v, r.p.n_bins), "request workspace")) return st;
        g->ws.push_back(w.release());
        workspace_carve(g->ws.back(), r.v->n_tiles, r.v->M, r.p.n_bins, fstore_cells(r.v, r.p.n_bins), &P.rdev[q].ws);
    }
    for (int k = 0; k < dvl_graph::kSlots; ++k) {
        DevBuf d(g->alloc);
        if (dvl_status st = d.alloc(P.device_bytes, "graph descriptors")) return st;
        g->dev[k] = (char*)d.release();
    }
    {
        // a first descriptor image validates the tables (range checks) before anything is captured
        std::vector<char> probe(P.block_bytes);
        if (dvl_status st = fill_block(P, probe.data(), g->dev[0])) return st;
    }
    for (int r = 0; r < kRing; ++r) {
        if (hipHostMalloc((void**)&g->host[r], P.block_bytes, hipHostMallocDefault) != hipSuccess) {
            g->host[r] = nullptr;
            (void)hipGetLastError();
            return fail(DVL_E_NOMEM, "pinned host allocation failed");
        }
        DVL_HIP(hipEventCreateWithFlags(&g->ev[r], hipEventDisableTiming));
    }
    // the kernels are captured at the first launch with each set of paths;
    // the descriptors they read are refreshed before every replay
    guard.g = nullptr;
    *out = g;
    return DVL_OK;
}

// The executable graph of this path set, captured on first use.
static dvl_status graph_exec_for(dvl_graph* g, int paths, int slot, hipGraphExec_t* out) {
    for (auto& c : g->captured)
        if (c.paths == paths && c.slot == slot) {
            *out = c.exec;
            return DVL_OK;
        }
    Plan& P = g->plan;
    hipStream_t cs;
    DVL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    if (hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    const dvl_status cst =
        launch_batch(batch_dev(P, g->dev[slot], paths), P.dtype, P.max_m, P.max_req, g->n_cu, cs, kDescriptorLayout, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (cst != DVL_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return cst;
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    if (hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    g->captured.push_back({paths, slot, graph, exec});
    *out = exec;
    return DVL_OK;
}

dvl_status dvl_graph_set_tf(dvl_graph* g, int32_t req, const float* alpha, const float* lo, const float* hi) {
    g_err.clear();
    if (!g) return fail(DVL_E_INVALID, "graph is NULL");
    Plan& P = g->plan;
    if (req < 0 || req >= (int)P.where.size())
        return fail(DVL_E_INVALID, "request %d outside [0, %zu)", req, P.where.size());
    ReqHost& r = P.reqs[P.where[req]];
    ReqHost tmp;
    if (dvl_status st = make_request(r.v, alpha, r.n_tf[0], lo, hi, &r.p, &r.out, tmp)) return st;
    r.alpha = std::move(tmp.alpha);
    for (int m = 0; m < r.v->M; ++m) {
        r.lo[m] = tmp.lo[m];
        r.hi[m] = tmp.hi[m];
        r.qs[m] = tmp.qs[m];
        r.qb[m] = tmp.qb[m];
    }
    return DVL_OK;
}

dvl_status dvl_graph_set_tf_all(dvl_graph* g, const float* const* alpha, const float* const* lo,
                                const float* const* hi) {
    g_err.clear();
    if (!g) return fail(DVL_E_INVALID, "graph is NULL");
    if (!alpha) return fail(DVL_E_INVALID, "alpha is NULL");
    const int n = (int)g->plan.where.size();
    for (int i = 0; i < n; ++i)
        if (dvl_status st = dvl_graph_set_tf(g, i, alpha[i], lo ? lo[i] : nullptr, hi ? hi[i] : nullptr)) {
            const std::string msg = g_err;
            return fail(st, "request %d: %s", i, msg.c_str());
        }
    return DVL_OK;
}

dvl_status dvl_graph_launch(dvl_graph* g, void* stream) {
    g_err.clear();
    if (!g) return fail(DVL_E_INVALID, "graph is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int r = g->next;
    if (g->used[r]) DVL_HIP(hipEventSynchronize(g->ev[r]));
    std::vector<CacheBuild> builds;
    if (dvl_status st = decide_cache(g->plan, builds)) return st;
    if (dvl_status st = run_cache_builds(builds, s)) return st;
    if (dvl_status st = cache_wait(g->plan, s)) return st;
    int paths = 0;
    for (const JobDev& j : g->plan.jobs) paths |= j.idx[0] ? kPathEntries : kPathValues;
    for (const ReqDev& d : g->plan.rdev)
        if (d.ws.fstore) paths |= kPathStoredF;
    const int slot = g->launches % dvl_graph::kSlots;
    hipGraphExec_t exec = nullptr;
    if (dvl_status st = graph_exec_for(g, paths, slot, &exec)) return st;
    if (dvl_status st = fill_block(g->plan, g->host[r], g->dev[slot])) return st;
    g->next = (r + 1) % kRing;
    DVL_HIP(hipMemcpyAsync(g->dev[slot], g->host[r], g->plan.block_bytes, hipMemcpyHostToDevice, s));
    DVL_HIP(hipEventRecord(g->ev[r], s));
    g->used[r] = true;
    DVL_HIP(hipGraphLaunch(exec, s));
    ++g->launches;
    return cache_mark_readers(g->plan, s);
}

void dvl_graph_destroy(dvl_graph* g) { delete g; }

}  // extern "C"
