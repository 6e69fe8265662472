/* Plain FP64 CPU oracle for dynamic volume lines over AMR cells.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code with the GPU library.
 *
 * Paper: Zellmann, Demirci, Gudukbay, "Visual Analysis of Large Multi-Field
 * AMR Data on GPUs Using Interactive Volume Lines" (arXiv 2306.11612).
 * Each function names the passage it follows.  Arithmetic is FP64 except the
 * transfer-function index quantiser, which is deliberately FP32 (one fmaf)
 * so that an integer decision (the TF entry) is taken in the same precision
 * as in the GPU kernel.
 *
 * Parity pins (what each part is checked against) are listed in the test
 * files; "parity unpinned" items: the specific Hilbert curve variant (the
 * paper names none) and outputs on realistic data beyond the invariants.
 */
#ifndef DVL_ORACLE_H
#define DVL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- ordering (Background: logical grid + Hilbert codes; GPU section:
 *      the order is fixed once) ---- */

/* Bits per dimension of the Hilbert cube: smallest b >= 1 with
 * 2^b >= max over cells and axes of (corner + 2^level).  Returns -1 if a
 * coordinate is negative, a level exceeds 20 or b would exceed 21. */
int32_t ora_grid_bits(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                      const uint8_t* level);

/* Hilbert index (3*bits bits) of the lattice point q on the 2^bits cube:
 * Skilling's transpose method (AIP Conf. Proc. 707, 2004), x being the most
 * significant axis of each 3-bit digit. */
uint64_t ora_hilbert_index(uint32_t qx, uint32_t qy, uint32_t qz, int32_t bits);

/* Key of every cell: Hilbert index of its centroid's finest-level cell
 * q = corner + (2^level >> 1).  keys[n] in original order. */
void ora_cell_keys(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                   const uint8_t* level, int32_t bits, uint64_t* keys);

/* perm[h] = original index of the h-th cell in (key, original index) order.
 * Returns the number of adjacent equal keys (0 when all keys differ). */
int64_t ora_sort_order(int64_t n, const uint64_t* keys, uint32_t* perm);

/* ---- transfer function (Interactive Transfer Function Updates) ---- */

/* FP32 quantiser constants of the normalisation window [lo, hi] for a table
 * of n_tf entries: s = n_tf / (hi - lo), b = -lo * s (each rounded to fp32). */
void ora_quantiser(int32_t n_tf, float lo, float hi, float* s, float* b);

/* TF entry of a value: clamp(floor(fmaf(x, s, b)), 0, n_tf - 1). */
int32_t ora_tf_index(float x, float s, float b, int32_t n_tf);

/* ---- max local variation (section Computing the Maximum Local Ensemble
 *      Variation, Eqs. 5-6) ---- */
enum { ORA_VMAX_TF_RANGE = 0, ORA_VMAX_TF_BOUND = 1, ORA_VMAX_EXACT = 2 };

/* Approximation from TFs and per-field data ranges.  i_m, j_m are the TF
 * entries of each field's data minimum and maximum.  mode TF_RANGE:
 * max over a in [min i_m, max j_m] of (max_m A_m[a] - min_m A_m[a]);
 * mode TF_BOUND: max_m max_{a in [i_m,j_m]} A_m[a] - min_m min_{a in [i_m,j_m]} A_m[a]. */
double ora_vmax_tf(int32_t mode, int32_t n_fields, int32_t n_tf, const float* alpha,
                   const int32_t* i_m, const int32_t* j_m);

/* ---- update (Eqs. 1-4, Projecting Cells to 1D) ---- */
typedef struct {
    int32_t n_bins;          /* W */
    double exponent;         /* P of Eq. 2/3 */
    double min_importance;   /* 0.025 in the paper's evaluation */
    int32_t vmax_mode;       /* ORA_VMAX_* */
    int32_t clamp_mode;      /* 0: f = max(fmin, (r*s)^P); 1: f = (max(fmin, r)*s)^P */
    int32_t level_scale;     /* 1: s = 2^L (Eq. 3); 3: s = 8^L (cell volume) */
} ora_params;

/* Per-bin results.  Arrays are caller-owned: first/last/count [W];
 * sum/mean [M*W] (double); vmin/vmax/y [M*W] (float); index m*W + b. */
typedef struct {
    uint32_t* first;
    uint32_t* last;
    uint32_t* count;
    double* sum;
    double* mean;
    float* vmin;
    float* vmax;
    float* y;
    double f_total;          /* F(max h) of Eq. 4 */
    double vmax_used;        /* max(V_h) (or its approximation) actually used */
    int32_t degenerate;      /* 1 when F_tot was 0 and every f was set to 1 */
} ora_bins;

/* Full per-update computation over cells already in Hilbert order.
 * level[n]; fields[M*n] (float32 storage, field-major); alpha[M*n_tf];
 * lo/hi[M] normalisation windows.  cell_f[n] and cell_e[n+1] (optional,
 * may be NULL) receive f(h) and the exclusive prefix E(h) (E(n) = F_tot).
 * Returns 0, or -1 on invalid arguments. */
int32_t ora_update(int64_t n, int32_t n_fields, const uint8_t* level, const float* fields,
                   int32_t n_tf, const float* alpha, const float* lo, const float* hi,
                   const ora_params* p, ora_bins* out, double* cell_f, double* cell_e);

/* Data range of one field (min and max over all n values). */
void ora_field_range(int64_t n, const float* v, float* vmin, float* vmax);

/* ---- histogram heatmap of a volume line (section Prototypical User
 *      Interface: the histogram heatmap of Weissenboeck et al.'s volume
 *      lines) ---- */
/* For every bin b of an update (sorted cells first[b]..last[b]) the number
 * of its cells whose value falls in bucket k of [lo, hi]: counts[b*H + k],
 * with the bucket of a value chosen as a TF entry is (ora_tf_index with the
 * quantiser of [lo, hi] for H entries; values outside the window go to the
 * end buckets).  values[n] in sorted order.  Returns 0, or -1 on invalid
 * arguments. */
int32_t ora_bin_histograms(int64_t n, const float* values, int32_t n_bins, const uint32_t* first,
                           const uint32_t* last, int32_t n_buckets, float lo, float hi, uint32_t* counts);

/* ---- RasterizeLines (GPU Implementation section: the volume lines drawn as
 *      polylines or as bar charts into the plot) ---- */
enum { ORA_RASTER_POLYLINE = 0, ORA_RASTER_BARS = 1 };
/* Image of one line of W heights y[b] in [0, 1] on H rows (row 0 at the
 * bottom): row(y) = min(H - 1, max(0, floor(y * H))) with y * H in fp32.
 * Polyline: column b holds row(y[b]) and every row between it and
 * row(y[b + 1]).  Bars: column b holds rows 0 .. row(y[b]).  img[r*W + b]
 * is 1 for a drawn pixel, else 0.  Returns 0, or -1 on invalid arguments. */
int32_t ora_rasterize(int32_t n_bins, const float* y, int32_t n_rows, int32_t mode, uint8_t* img);

#ifdef __cplusplus
}
#endif
#endif
