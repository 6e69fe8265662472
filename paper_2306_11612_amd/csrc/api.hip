// C ABI of the DVL library: validation, buffer ownership, host-side TF
// preparation (Eqs. 5-6 run on the host, as in the paper's GPU section) and
// kernel launches.  Declarations and contracts: include/dvl.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "order.hpp"
#include "update.hpp"

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

// device buffer owned by RAII until released into the volume
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    dvl_status alloc(size_t bytes, const char* what) {
        hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(DVL_E_NOMEM, "hipMalloc of %zu bytes for %s failed", bytes, what);
        }
        return DVL_OK;
    }
    void* release() { void* q = p; p = nullptr; return q; }
};

constexpr int kRing = 4;   // parameter uploads that may be in flight per volume

}  // namespace dvl

using namespace dvl;

struct dvl_volume {
    int64_t n = 0;
    int64_t n_pad = 0;       // cells rounded up to whole update tiles
    int64_t n_tiles = 0;
    int32_t M = 0;
    int32_t dtype = DVL_F32;
    int32_t bits = 0;
    int32_t max_level = 0;
    int device = 0;
    int n_cu = 256;
    uint8_t* level_s = nullptr;
    void* fields_s[kMaxFields] = {};
    uint64_t* keys_s = nullptr;
    uint32_t* perm = nullptr;
    float dmin[kMaxFields] = {};
    float dmax[kMaxFields] = {};
    // transfer functions (host copies)
    bool tf_set[kMaxFields] = {};
    std::vector<float> alpha[kMaxFields];
    float lo[kMaxFields] = {}, hi[kMaxFields] = {};
    float qs[kMaxFields] = {}, qb[kMaxFields] = {};
    // parameter block ring (pinned host staging -> device)
    size_t param_bytes = 0;
    void* param_dev[kRing] = {};
    void* param_host[kRing] = {};
    hipEvent_t param_ev[kRing] = {};
    bool param_used[kRing] = {};
    int param_next = 0;
    // per-tile statistics of the sorted fields: sum [M][T], min [M][T], max [M][T]
    double* agg_sum = nullptr;
    float* agg_min = nullptr;
    float* agg_max = nullptr;
    // update workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    UpdWorkspace wsv{};
    dvl_status sticky = DVL_OK;
    size_t bytes = 0;
    // optional per-kernel timing
    bool timing = false;
    std::vector<std::vector<hipEvent_t>> ev_pool, ev_pending;
    double phase_ms[kPhases] = {};
    int32_t timed_updates = 0;
};

namespace {

dvl_status check_sticky(const dvl_volume* v) {
    if (!v) return fail(DVL_E_INVALID, "volume is NULL");
    if (v->sticky != DVL_OK) return fail(v->sticky, "volume is in a failed state after an earlier device error");
    return DVL_OK;
}

// FP32 quantiser of the window [lo, hi] for n_tf entries
void quantiser(int n_tf, float lo, float hi, float* s, float* b) {
    const float sf = (float)((double)n_tf / ((double)hi - (double)lo));
    *s = sf;
    *b = (float)(-(double)lo * (double)sf);
}

int host_entry(float x, float s, float b, int n_tf) {
    float t = fmaf(x, s, b);
    if (!(t >= 0.0f)) return 0;
    if (t > (float)(n_tf - 1)) return n_tf - 1;
    return (int)t;
}

// Eqs. 5-6 and the bound variant (section "Computing the Maximum Local
// Ensemble Variation"): max(V_h) from the TFs and the fields' data ranges
float host_vmax(const dvl_volume* v, int mode) {
    const int M = v->M;
    int im[kMaxFields], jm[kMaxFields];
    for (int m = 0; m < M; ++m) {
        const int n_tf = (int)v->alpha[m].size();
        im[m] = host_entry(v->dmin[m], v->qs[m], v->qb[m], n_tf);
        jm[m] = host_entry(v->dmax[m], v->qs[m], v->qb[m], n_tf);
    }
    auto bound = [&]() {
        float hi = -INFINITY, lo = INFINITY;
        for (int m = 0; m < M; ++m)
            for (int a = im[m]; a <= jm[m]; ++a) {
                hi = std::max(hi, v->alpha[m][a]);
                lo = std::min(lo, v->alpha[m][a]);
            }
        return hi - lo;
    };
    if (mode == DVL_VMAX_TF_BOUND) return bound();
    int i = im[0], j = jm[0];
    for (int m = 1; m < M; ++m) { i = std::min(i, im[m]); j = std::max(j, jm[m]); }
    float best = 0.0f;
    for (int a = i; a <= j; ++a) {
        float hi = -INFINITY, lo = INFINITY;
        for (int m = 0; m < M; ++m) {
            const std::vector<float>& t = v->alpha[m];
            const float al = t[std::min<int>(a, (int)t.size() - 1)];
            hi = std::max(hi, al);
            lo = std::min(lo, al);
        }
        best = std::max(best, hi - lo);
    }
    if (best <= 0.0f) best = bound();   // the literal approximation can vanish (e.g. equal TFs)
    return best;
}

unsigned grid_small(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

extern "C" {

const char* dvl_last_error(void) { return g_err.c_str(); }

size_t dvl_update_workspace_bytes(int64_t n_cells, int32_t n_fields, int32_t n_bins) {
    (void)n_bins;
    if (n_cells < 1 || n_fields < 1) return 0;
    const int64_t T = (n_cells + kTileCells - 1) / kTileCells;
    return workspace_bytes(T, n_fields);
}

dvl_status dvl_build_order(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                           const uint8_t* level, int32_t M, int32_t dtype, const void* const* fields,
                           void* stream, dvl_volume** out) {
    g_err.clear();
    if (!out) return fail(DVL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 32)) return fail(DVL_E_INVALID, "n_cells=%lld outside [1, 2^32)", (long long)n);
    if (M < 1 || M > kMaxFields) return fail(DVL_E_INVALID, "n_fields=%d outside [1, %d]", M, kMaxFields);
    if (dtype != DVL_F32 && dtype != DVL_F16 && dtype != DVL_BF16) return fail(DVL_E_INVALID, "unknown dtype %d", dtype);
    if (!x || !y || !z || !level || !fields) return fail(DVL_E_INVALID, "NULL input pointer");
    for (int m = 0; m < M; ++m)
        if (!fields[m]) return fail(DVL_E_INVALID, "field %d pointer is NULL", m);
    hipStream_t s = (hipStream_t)stream;
    const int eb = elem_bytes_of(dtype);

    dvl_volume* v = new (std::nothrow) dvl_volume();
    if (!v) return fail(DVL_E_NOMEM, "host allocation failed");
    struct Guard { dvl_volume* v; ~Guard() { if (v) dvl_destroy(v); } } guard{v};
    v->n = n;
    v->M = M;
    v->dtype = dtype;
    v->n_tiles = (n + kTileCells - 1) / kTileCells;
    v->n_pad = v->n_tiles * kTileCells;
    DVL_HIP(hipGetDevice(&v->device));
    DVL_HIP(hipDeviceGetAttribute(&v->n_cu, hipDeviceAttributeMultiprocessorCount, v->device));

    // extent, validity, grid bits
    DevBuf ext;
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
    DevBuf ka, kb, va, vb, counts, partial;
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
    DevBuf lv;
    if (dvl_status st = lv.alloc((size_t)v->n_pad, "sorted levels")) return st;
    DVL_HIP(hipMemsetAsync((char*)lv.p + n, 0, (size_t)(v->n_pad - n), s));
    if (dvl_status st = launch_gather(n, v->perm, level, lv.p, 1, s)) return st;
    v->level_s = (uint8_t*)lv.release();
    v->bytes += (size_t)v->n_pad;
    DevBuf rng;
    if (dvl_status st = rng.alloc((size_t)kMaxFields * 4 * sizeof(unsigned int), "ranges")) return st;
    std::vector<unsigned int> rinit(kMaxFields * 4);
    for (int m = 0; m < kMaxFields; ++m) { rinit[m * 4] = 0xFFFFFFFFu; rinit[m * 4 + 1] = 0; rinit[m * 4 + 2] = 0; rinit[m * 4 + 3] = 0; }
    DVL_HIP(hipMemcpyAsync(rng.p, rinit.data(), rinit.size() * 4, hipMemcpyHostToDevice, s));
    for (int m = 0; m < M; ++m) {
        DevBuf fb;
        if (dvl_status st = fb.alloc((size_t)v->n_pad * eb, "sorted field")) return st;
        DVL_HIP(hipMemsetAsync((char*)fb.p + (size_t)n * eb, 0, (size_t)(v->n_pad - n) * eb, s));
        if (dvl_status st = launch_gather(n, v->perm, fields[m], fb.p, eb, s)) return st;
        if (dvl_status st = launch_range(n, dtype, fb.p, (unsigned int*)rng.p + 4 * m, s)) return st;
        v->fields_s[m] = fb.release();
        v->bytes += (size_t)v->n_pad * eb;
    }
    {
        DevBuf as, an, ax;
        const size_t mt = (size_t)M * v->n_tiles;
        if (dvl_status st = as.alloc(mt * 8, "tile sums")) return st;
        if (dvl_status st = an.alloc(mt * 4, "tile minima")) return st;
        if (dvl_status st = ax.alloc(mt * 4, "tile maxima")) return st;
        v->agg_sum = (double*)as.release();
        v->agg_min = (float*)an.release();
        v->agg_max = (float*)ax.release();
        v->bytes += mt * 16;
        for (int m = 0; m < M; ++m)
            if (dvl_status st = launch_tile_aggregates(n, dtype, v->fields_s[m], v->n_tiles,
                                                       v->agg_sum + (size_t)m * v->n_tiles,
                                                       v->agg_min + (size_t)m * v->n_tiles,
                                                       v->agg_max + (size_t)m * v->n_tiles, v->n_cu, s))
                return st;
    }
    DVL_HIP(hipMemcpyAsync(rinit.data(), rng.p, rinit.size() * 4, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < M; ++m) {
        if (rinit[m * 4 + 2]) return fail(DVL_E_RANGE, "field %d holds a NaN", m);
        auto unkey = [](unsigned int u) {
            const unsigned int b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
            float f;
            memcpy(&f, &b, 4);
            return f;
        };
        v->dmin[m] = unkey(rinit[m * 4]);
        v->dmax[m] = unkey(rinit[m * 4 + 1]);
    }

    // update workspace and parameter ring
    v->ws_bytes = workspace_bytes(v->n_tiles, M);
    DevBuf wsb;
    if (dvl_status st = wsb.alloc(v->ws_bytes, "update workspace")) return st;
    v->ws = wsb.release();
    workspace_carve(v->ws, v->n_tiles, M, &v->wsv);
    v->bytes += v->ws_bytes;
    v->param_bytes = sizeof(DevParamsHeader) + (size_t)kMaxTfTotal * sizeof(float);
    for (int r = 0; r < kRing; ++r) {
        DevBuf pd;
        if (dvl_status st = pd.alloc(v->param_bytes, "parameter block")) return st;
        v->param_dev[r] = pd.release();
        v->bytes += v->param_bytes;
        if (hipHostMalloc(&v->param_host[r], v->param_bytes, hipHostMallocDefault) != hipSuccess) {
            v->param_host[r] = nullptr;
            (void)hipGetLastError();
            return fail(DVL_E_NOMEM, "pinned host allocation of the parameter block failed");
        }
        DVL_HIP(hipEventCreateWithFlags(&v->param_ev[r], hipEventDisableTiming));
    }
    guard.v = nullptr;
    *out = v;
    return DVL_OK;
}

dvl_status dvl_set_field(dvl_volume* v, int32_t m, const void* values, void* stream) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
    if (m < 0 || m >= v->M) return fail(DVL_E_INVALID, "field index %d outside [0, %d)", m, v->M);
    if (!values) return fail(DVL_E_INVALID, "values is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int eb = elem_bytes_of(v->dtype);
    DevBuf rng;
    if (dvl_status st = rng.alloc(4 * sizeof(unsigned int), "range")) return st;
    unsigned int r[4] = {0xFFFFFFFFu, 0u, 0u, 0u};
    DVL_HIP(hipMemcpyAsync(rng.p, r, sizeof r, hipMemcpyHostToDevice, s));
    if (dvl_status st = launch_gather(v->n, v->perm, values, v->fields_s[m], eb, s)) { v->sticky = st; return st; }
    if (dvl_status st = launch_range(v->n, v->dtype, v->fields_s[m], (unsigned int*)rng.p, s)) { v->sticky = st; return st; }
    if (dvl_status st = launch_tile_aggregates(v->n, v->dtype, v->fields_s[m], v->n_tiles,
                                               v->agg_sum + (size_t)m * v->n_tiles,
                                               v->agg_min + (size_t)m * v->n_tiles,
                                               v->agg_max + (size_t)m * v->n_tiles, v->n_cu, s)) {
        v->sticky = st;
        return st;
    }
    DVL_HIP(hipMemcpyAsync(r, rng.p, sizeof r, hipMemcpyDeviceToHost, s));
    DVL_HIP(hipStreamSynchronize(s));
    if (r[2]) return fail(DVL_E_RANGE, "field %d holds a NaN", m);
    auto unkey = [](unsigned int u) {
        const unsigned int b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
        float f;
        memcpy(&f, &b, 4);
        return f;
    };
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
    if (dvl_status st = check_sticky(v)) return st;
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
    v->qs[m] = s;
    v->qb[m] = b;
    v->tf_set[m] = true;
    return DVL_OK;
}

dvl_status dvl_update(dvl_volume* v, const dvl_params* p, const dvl_bins* out, void* stream) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
    if (!p || !out) return fail(DVL_E_INVALID, "params or bins is NULL");
    if (p->n_bins < 1 || p->n_bins > (1 << 20)) return fail(DVL_E_INVALID, "n_bins=%d outside [1, 2^20]", p->n_bins);
    if (!(p->exponent >= 0.0f && p->exponent <= 16.0f)) return fail(DVL_E_INVALID, "exponent %g outside [0, 16]", p->exponent);
    if (!(p->min_importance >= 0.0f) || !isfinite(p->min_importance)) return fail(DVL_E_INVALID, "min_importance %g must be finite and >= 0", p->min_importance);
    if (p->vmax_mode < 0 || p->vmax_mode > 2) return fail(DVL_E_INVALID, "vmax_mode %d", p->vmax_mode);
    if (p->clamp_mode < 0 || p->clamp_mode > 1) return fail(DVL_E_INVALID, "clamp_mode %d", p->clamp_mode);
    if (p->level_scale != 1 && p->level_scale != 3) return fail(DVL_E_INVALID, "level_scale %d (1 or 3)", p->level_scale);
    if (p->scan_mode < 0 || p->scan_mode > 2) return fail(DVL_E_INVALID, "scan_mode %d", p->scan_mode);
    if (!out->first_cell || !out->last_cell || !out->mean || !out->vmin || !out->vmax || !out->y ||
        !out->f_total || !out->vmax_used)
        return fail(DVL_E_INVALID, "a bins pointer is NULL");
    for (int m = 0; m < v->M; ++m)
        if (!v->tf_set[m]) return fail(DVL_E_STATE, "field %d has no transfer function", m);
    hipStream_t s = (hipStream_t)stream;

    UpdArgs a{};
    a.n = v->n;
    a.n_tiles = v->n_tiles;
    {
        // runs of consecutive tiles, one per wave of the importance pass
        const int64_t waves = (int64_t)v->n_cu * 8 * (kUpdThreads / kWave);
        a.tiles_per_run = std::max<int64_t>(1, (v->n_tiles + waves - 1) / waves);
        a.n_runs = (v->n_tiles + a.tiles_per_run - 1) / a.tiles_per_run;
    }
    a.M = v->M;
    a.dtype = v->dtype;
    a.W = p->n_bins;
    a.exponent = p->exponent;
    a.fmin = p->min_importance;
    a.exp_is_one = p->exponent == 1.0f;
    a.clamp_mode = p->clamp_mode;
    a.level_shift = p->level_scale;
    a.scan_mode = p->scan_mode;
    a.vmax_exact = p->vmax_mode == DVL_VMAX_EXACT;
    int off = 0;
    float amax = -INFINITY, amin = INFINITY;
    for (int m = 0; m < v->M; ++m) {
        a.s[m] = v->qs[m];
        a.b[m] = v->qb[m];
        a.nmax[m] = (float)(v->alpha[m].size() - 1);
        a.tf_off[m] = off;
        off += (int)v->alpha[m].size();
        for (float al : v->alpha[m]) { amax = std::max(amax, al); amin = std::min(amin, al); }
    }
    a.tf_total = off;
    const float vmax = a.vmax_exact ? 0.0f : host_vmax(v, p->vmax_mode);

    // overflow guard: the largest possible importance times a tile must stay finite in fp32
    {
        const double vr = (double)amax - (double)amin;
        const double rmax = a.vmax_exact ? 1.0 : (vmax > 0.0f ? vr / (double)vmax : 0.0);
        const double g = std::max((double)p->min_importance, rmax) * ldexp(1.0, p->level_scale * v->max_level);
        const double fmax_cell = std::max((double)p->min_importance, pow(g, (double)p->exponent));
        if (!(fmax_cell * kTileCells < 1e37)) return fail(DVL_E_RANGE, "importance can reach %g: exponent and levels overflow fp32", fmax_cell);
    }

    // stage the parameter block: header (max V) + concatenated TF tables
    const int r = v->param_next;
    v->param_next = (r + 1) % kRing;
    if (v->param_used[r]) DVL_HIP(hipEventSynchronize(v->param_ev[r]));
    char* hp = (char*)v->param_host[r];
    DevParamsHeader hdr{};
    hdr.vmax = vmax;
    memcpy(hp, &hdr, sizeof hdr);
    float* tfh = (float*)(hp + sizeof(DevParamsHeader));
    for (int m = 0; m < v->M; ++m) memcpy(tfh + a.tf_off[m], v->alpha[m].data(), v->alpha[m].size() * 4);
    const size_t bytes = sizeof(DevParamsHeader) + (size_t)off * 4;
    DVL_HIP(hipMemcpyAsync(v->param_dev[r], hp, bytes, hipMemcpyHostToDevice, s));
    DVL_HIP(hipEventRecord(v->param_ev[r], s));
    v->param_used[r] = true;

    a.vmax_dev = (float*)v->param_dev[r];
    a.tf = (const float*)((char*)v->param_dev[r] + sizeof(DevParamsHeader));
    a.level = v->level_s;
    for (int m = 0; m < v->M; ++m) a.fields[m] = v->fields_s[m];
    a.ws = v->wsv;
    a.agg_sum = v->agg_sum;
    a.agg_min = v->agg_min;
    a.agg_max = v->agg_max;
    a.first_cell = out->first_cell;
    a.last_cell = out->last_cell;
    a.mean = out->mean;
    a.vmin = out->vmin;
    a.vmax = out->vmax;
    a.y = out->y;
    a.f_total = out->f_total;
    a.vmax_used = out->vmax_used;
    hipEvent_t* ev = nullptr;
    if (v->timing) {
        if (v->ev_pool.empty()) {
            std::vector<hipEvent_t> set(kPhases + 1);
            for (auto& e : set) DVL_HIP(hipEventCreate(&e));
            v->ev_pool.push_back(set);
        }
        v->ev_pending.push_back(v->ev_pool.back());
        v->ev_pool.pop_back();
        ev = v->ev_pending.back().data();
    }
    dvl_status st = launch_update(a, v->n_cu, s, ev);
    if (st != DVL_OK) v->sticky = st;
    return st;
}

dvl_status dvl_read_bins(const dvl_volume* v, const dvl_bins* b, int32_t W, void* stream, uint32_t* count,
                         uint32_t* first, uint32_t* last, float* mean, float* vmin, float* vmax, float* y,
                         double* f_total, float* vmax_used) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
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
    if (dvl_status st = check_sticky(v)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (keys) {
        if (dvl_status st = launch_scatter_back(v->n, v->perm, v->keys_s, keys, 8, s)) return st;
    }
    if (perm) DVL_HIP(hipMemcpyAsync(perm, v->perm, (size_t)v->n * 4, hipMemcpyDeviceToDevice, s));
    return DVL_OK;
}

dvl_status dvl_export_sorted(const dvl_volume* v, uint8_t* level, void* const* fields, void* stream) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
    hipStream_t s = (hipStream_t)stream;
    if (level) DVL_HIP(hipMemcpyAsync(level, v->level_s, (size_t)v->n, hipMemcpyDeviceToDevice, s));
    if (fields) {
        const size_t eb = elem_bytes_of(v->dtype);
        for (int m = 0; m < v->M; ++m)
            if (fields[m]) DVL_HIP(hipMemcpyAsync(fields[m], v->fields_s[m], (size_t)v->n * eb, hipMemcpyDeviceToDevice, s));
    }
    return DVL_OK;
}

dvl_status dvl_set_timing(dvl_volume* v, int32_t enable) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
    v->timing = enable != 0;
    return DVL_OK;
}

dvl_status dvl_kernel_times(dvl_volume* v, double* ms, int32_t* n_updates) {
    g_err.clear();
    if (dvl_status st = check_sticky(v)) return st;
    for (auto& set : v->ev_pending) {
        DVL_HIP(hipEventSynchronize(set[kPhases]));
        for (int p = 0; p < kPhases; ++p) {
            float t = 0.0f;
            DVL_HIP(hipEventElapsedTime(&t, set[p], set[p + 1]));
            v->phase_ms[p] += t;
        }
        v->timed_updates += 1;
        v->ev_pool.push_back(set);
    }
    v->ev_pending.clear();
    if (ms)
        for (int p = 0; p < kPhases; ++p) ms[p] = v->phase_ms[p];
    if (n_updates) *n_updates = v->timed_updates;
    for (int p = 0; p < kPhases; ++p) v->phase_ms[p] = 0.0;
    v->timed_updates = 0;
    return DVL_OK;
}

int64_t dvl_num_cells(const dvl_volume* v) { return v ? v->n : 0; }
int32_t dvl_num_fields(const dvl_volume* v) { return v ? v->M : 0; }
int32_t dvl_grid_bits(const dvl_volume* v) { return v ? v->bits : 0; }
int32_t dvl_dtype(const dvl_volume* v) { return v ? v->dtype : -1; }
size_t dvl_volume_bytes(const dvl_volume* v) { return v ? v->bytes : 0; }

void dvl_destroy(dvl_volume* v) {
    if (!v) return;
    (void)hipDeviceSynchronize();
    if (v->level_s) (void)hipFree(v->level_s);
    for (int m = 0; m < kMaxFields; ++m)
        if (v->fields_s[m]) (void)hipFree(v->fields_s[m]);
    if (v->keys_s) (void)hipFree(v->keys_s);
    if (v->perm) (void)hipFree(v->perm);
    if (v->ws) (void)hipFree(v->ws);
    if (v->agg_sum) (void)hipFree(v->agg_sum);
    if (v->agg_min) (void)hipFree(v->agg_min);
    if (v->agg_max) (void)hipFree(v->agg_max);
    for (auto* pool : {&v->ev_pool, &v->ev_pending})
        for (auto& set : *pool)
            for (auto e : set) (void)hipEventDestroy(e);
    for (int r = 0; r < kRing; ++r) {
        if (v->param_dev[r]) (void)hipFree(v->param_dev[r]);
        if (v->param_host[r]) (void)hipHostFree(v->param_host[r]);
        if (v->param_ev[r]) (void)hipEventDestroy(v->param_ev[r]);
    }
    delete v;
}

}  // extern "C"
