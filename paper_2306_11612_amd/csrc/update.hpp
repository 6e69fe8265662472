// Per-update kernels (update.hip): device descriptors and launchers.
//
// An update batch is a list of jobs; a job is one resident volume and up to
// kMaxReqPerJob requests (TF sets + parameters + outputs) that share one read
// of the volume's cells in the importance pass.  A single dvl_update is a
// batch of one job with one request.
#pragma once

#include "common.hpp"

namespace dvl {

constexpr int kUpdThreads = 256;                 // 4 waves per workgroup
constexpr int kCellsPerLane = 4;                 // one 4-vector per field per step
constexpr int kStepCells = kWave * kCellsPerLane;    // 256 cells per wave step
constexpr int kDefaultTileSteps = 16;            // 4096-cell tiles unless tuned
constexpr int kMaxReqPerJob = 8;
constexpr int kPhases = 5;                       // exact vmax, tile sums, carry + classification, rescan, bin statistics
constexpr int kPathValues = 1;                   // jobs that read the field values
constexpr int kPathEntries = 2;                  // jobs that read cached TF entries
constexpr int kPathStoredF = 4;                  // requests whose projection reads stored f
constexpr int kIdxTable = 256;                   // LDS floats per table on the cached-entry path

// Workspace of one request on a volume of T tiles and M fields.
struct UpdWorkspace {
    double* local_prefix; // [T]  sum of the importance of earlier tiles of the same run
    double* run_total;    // [R]  sum over each run of consecutive tiles
    double* run_base;     // [R + 1]  exclusive prefix of run totals, run_base[R] = F_tot
    int32_t* head_bin;    // [T]  bin of the tile's first cell
    int32_t* tail_bin;    // [T]  bin of the tile's last cell
    uint32_t* rec_first;  // [2][T]  cell range of the tile's head bin, then of its tail bin
    uint32_t* rec_last;   // [2][T]
    int32_t* bin_t1;      // [W]  last tile whose first cell's bin is <= b (the last tile touching bin b)
    int32_t* bin_ta;      // [W]  first tile whose pixel interval ends in bin >= b (bin b's first
                          //      tile, or the one before it when that tile's last cell ends exactly at b)
    double* scal;         // [0] F_tot, [1] degenerate (0/1)
    float* fstore;        // [n_pad] importance of every cell, or NULL (see wants_fstore)
};

// n_bins: the request's W; fcells: cells of the stored importance (0: none)
size_t workspace_bytes(int64_t n_tiles, int M, int n_bins, int64_t fcells = 0);
void workspace_carve(void* base, int64_t n_tiles, int M, int n_bins, int64_t fcells, UpdWorkspace* w);

// Whether a request stores f in the importance pass for the projection to
// reuse: worth its 4 B per cell once about a quarter or more of the tiles
// hold a bin edge (the projection then rescans most of the volume).
inline bool wants_fstore(int64_t n_tiles, int n_bins) { return (int64_t)n_bins * 4 >= n_tiles; }

// One request: TF tables, quantisers, parameters, workspace and outputs.
struct ReqDev {
    float s[kMaxFields];      // quantiser scale per field
    float b[kMaxFields];      // quantiser offset per field
    float nmax[kMaxFields];   // n_tf - 1 per field
    int tf_off[kMaxFields];   // start of field m's table inside this request's block
    const float* tf;          // this request's tables (device)
    float* vmax_dev;          // max(V) used: host value, or computed (exact mode)
    int tf_job_off;           // start of this request's block inside the job's tables
    int tf_total;             // floats in this request's block
    int W;
    float exponent;
    float fmin;
    int exp_is_one;
    int clamp_mode;
    int level_shift;          // 1: 2^L, 3: 8^L
    int scan_mode;
    int vmax_exact;
    int job;
    int pad_;
    int64_t k3_unit0;         // first projection unit (tile) of this request
    int64_t k4_unit0;         // first bin unit of this request
    UpdWorkspace ws;
    uint32_t* first_cell;
    uint32_t* last_cell;
    float* mean;
    float* vmin;
    float* vmax;
    float* y;
    double* f_total;
    float* vmax_used;
};

// One volume and the requests that share its reads.
struct JobDev {
    int64_t n;
    int64_t n_tiles;
    int64_t tiles_per_run;    // importance-pass wave r owns tiles [r k, (r + 1) k)
    int64_t n_runs;
    int64_t k1_unit0;         // first importance-pass unit (4 runs, one workgroup)
    int M;
    int req0;
    int n_req;
    int tf_total_all;         // floats of all requests' tables (LDS of the importance pass)
    int tile_steps;           // 256-cell steps per tile
    int pad_;
    const uint8_t* level;
    const uint32_t* lcode;    // per-step level codes (launch_level_codes)
    const void* fields[kMaxFields];
    const uint8_t* idx[kMaxFields];   // cached TF entries per field, or all NULL: read the values
    const double* agg_sum;    // per-tile field statistics [M][T]
    const float* agg_min;
    const float* agg_max;
    const double* step_sum;   // per-step (256 cells) field statistics [M][T * tile_steps]
    const float* step_min;
    const float* step_max;
    const float* tf_all;      // the requests' tables, request after request
};

struct BatchDev {
    const JobDev* jobs;
    const ReqDev* reqs;
    uint32_t* rescan_count;   // [3] tiles queued for a rescan per projection path (0 when uploaded)
    uint32_t* carry_ready;    // [n_reqs] set once a request's carry is published (0 when uploaded)
    uint64_t* rescan_queue;   // [3][k3_units] projection units of the queued tiles, per path
    int n_jobs;
    int n_reqs;
    int64_t k1_units;
    int64_t k3_units;
    int64_t k4_units;
    int any_exact;
    int paths;                // kPathValues | kPathEntries: which importance-pass variants to launch
    int max_req_tf;           // largest request table block (floats): LDS of the projection
    int max_job_tf;           // largest job table block (floats): LDS of the importance pass
    int max_req_job;          // most requests in one job
    int max_tile_steps;       // largest tile (256-cell steps) of the batch's volumes
    int carry_wait_polls;     // bounded wait of the classification for a published carry
};

// Polls of a request's carry flag before a classifying workgroup computes the
// carry itself (the default; dvl_set_carry_wait changes it for tests).
constexpr int kCarryWaitPolls = 1 << 15;

// The descriptor layout a translation unit was compiled with.  The host
// code that writes the descriptors and every unit whose kernels read them
// must agree; launch_batch refuses a mismatch (objects built from different
// versions of this header) before any kernel runs.
constexpr uint64_t kDescriptorLayout =
    ((uint64_t)sizeof(ReqDev) << 40) | ((uint64_t)sizeof(JobDev) << 20) | (uint64_t)sizeof(BatchDev);

// Launch the five phases for the batch described by `b` (descriptors already
// resident on the device).  `max_m`, `max_req`: largest field count and
// requests per job in the batch.  `layout`: the caller's kDescriptorLayout.
// ev (optional): kPhases + 1 events.
dvl_status launch_batch(const BatchDev& b, int dtype, int max_m, int max_req, int n_cu, hipStream_t s,
                        uint64_t layout, hipEvent_t* ev = nullptr);

// TF entry of every cell of one sorted field under quantiser (s, b) with
// n_tf <= 256 entries, one byte per cell, over all n_pad (padded) cells.
dvl_status launch_build_index(int64_t n_pad, int dtype, const void* field, float s, float b, int n_tf,
                              uint8_t* out, int n_cu, hipStream_t st);

// Level codes of the sorted levels (n_steps * 256 bytes, padded): per
// 256-cell step one 32-bit word whose byte k is the common level of the cells
// [64 k, 64 k + 64) of the step, or 0xFF when they differ.
dvl_status launch_level_codes(const uint8_t* level, int64_t n_steps, uint32_t* codes, hipStream_t s);

// Per-tile and per-step (256 cells) sum / min / max of one sorted field:
// tile arrays [n_tiles], step arrays [n_tiles * tile_steps].
dvl_status launch_tile_aggregates(int64_t n, int dtype, const void* field, int64_t n_tiles, int tile_steps,
                                  double* sum, float* mn, float* mx, double* ssum, float* smn, float* smx,
                                  int n_cu, hipStream_t s);

}  // namespace dvl
