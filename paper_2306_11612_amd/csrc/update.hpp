// Per-update kernels (update.hip): arguments and launcher.
#pragma once

#include "common.hpp"

namespace dvl {

constexpr int kUpdThreads = 256;                 // 4 waves per workgroup
constexpr int kCellsPerLane = 4;                 // one 4-vector per field per step
constexpr int kStepCells = kWave * kCellsPerLane;    // 256 cells per wave step
constexpr int kTileSteps = 16;
constexpr int kTileCells = kStepCells * kTileSteps;  // 4096 cells per wave tile

// Workspace of one update, sized for n_tiles tiles and M fields.
struct UpdWorkspace {
    double* local_prefix; // [T]  sum of the importance of earlier tiles of the same run
    double* run_total;    // [R]  sum over each run of consecutive tiles
    double* run_base;     // [R + 1]  exclusive prefix of run totals, run_base[R] = F_tot
    int32_t* head_bin;    // [T]
    int32_t* tail_bin;    // [T]
    uint32_t* rec_first;  // [2][T]  head records then tail records
    uint32_t* rec_last;   // [2][T]
    double* rec_sum;      // [2][M][T]
    float* rec_min;       // [2][M][T]
    float* rec_max;       // [2][M][T]
    double* scal;         // [0] F_tot, [1] degenerate (as 0/1)
};

size_t workspace_bytes(int64_t n_tiles, int M);
void workspace_carve(void* base, int64_t n_tiles, int M, UpdWorkspace* w);

// Device parameter block uploaded before each update.
struct DevParamsHeader {
    float vmax;           // max(V) used (TF modes: host value; EXACT: device result)
    uint32_t pad[63];     // keep the TF tables 256-byte aligned
};

struct UpdArgs {
    int64_t n;
    int64_t n_tiles;
    int64_t tiles_per_run;    // K1 wave r owns tiles [r * tiles_per_run, (r + 1) * tiles_per_run)
    int64_t n_runs;
    int M;
    int dtype;
    int tf_total;         // sum of the fields' table sizes (LDS floats)
    int W;
    float exponent;
    float fmin;
    int exp_is_one;
    int clamp_mode;
    int level_shift;      // 1: 2^L, 3: 8^L
    int scan_mode;
    int vmax_exact;
    float s[kMaxFields];      // quantiser scale per field
    float b[kMaxFields];      // quantiser offset per field
    float nmax[kMaxFields];   // n_tf - 1 per field
    int tf_off[kMaxFields];   // start of field m's table
    const uint8_t* level;
    const void* fields[kMaxFields];
    const float* tf;      // concatenated tables, field m at tf_off[m]
    float* vmax_dev;      // parameter block header
    UpdWorkspace ws;
    // per-tile field statistics of the sorted volume (independent of the TF):
    // sum [M][T] (fp64), min / max [M][T]
    const double* agg_sum;
    const float* agg_min;
    const float* agg_max;
    // outputs
    uint32_t* first_cell;
    uint32_t* last_cell;
    float* mean;
    float* vmin;
    float* vmax;
    float* y;
    double* f_total;
    float* vmax_used;
};

constexpr int kPhases = 5;   // exact vmax, tile sums, carry, bin, edges

// ev (optional): kPhases + 1 events recorded before the first and after every phase
dvl_status launch_update(const UpdArgs& a, int n_cu, hipStream_t s, hipEvent_t* ev = nullptr);

// Per-tile sum / min / max of one sorted field (the tiles of the update).
dvl_status launch_tile_aggregates(int64_t n, int dtype, const void* field, int64_t n_tiles, double* sum,
                                  float* mn, float* mx, int n_cu, hipStream_t s);

}  // namespace dvl
