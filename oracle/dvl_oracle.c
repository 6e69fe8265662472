/* Plain FP64 CPU oracle for dynamic volume lines over AMR cells.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the GPU library is checked
 * against.  Single-threaded, unblocked, written in the order the paper
 * describes the method.  It shares no code with the GPU library.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared dvl_oracle.c -lm
 */
#include "dvl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Ordering                                                            */
/* ------------------------------------------------------------------ */

/* Background section, AMR paragraph: a cell is its lower corner on the
 * logical grid plus its level L (0 finest), width 2^L.  The Hilbert cube
 * must contain every cell, so its side 2^b is the smallest power of two
 * not below the largest upper corner. */
int32_t ora_grid_bits(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                      const uint8_t* level)
{
    int64_t extent = 1;
    for (int64_t h = 0; h < n; ++h) {
        if (x[h] < 0 || y[h] < 0 || z[h] < 0 || level[h] > 20) return -1;
        int64_t w = (int64_t)1 << level[h];
        int64_t ux = (int64_t)x[h] + w, uy = (int64_t)y[h] + w, uz = (int64_t)z[h] + w;
        if (ux > extent) extent = ux;
        if (uy > extent) extent = uy;
        if (uz > extent) extent = uz;
    }
    int32_t b = 1;
    while (((int64_t)1 << b) < extent) ++b;
    return b > 21 ? -1 : b;
}

/* Skilling, "Programming the Hilbert curve" (2004): the coordinates are
 * turned in place into the "transposed" Hilbert index by (1) undoing the
 * excess work of the recursive construction from the top bit down (for each
 * bit plane Q and axis i, either invert the low bits of axis 0 or exchange
 * the low bits of axis 0 and axis i) and (2) Gray-encoding across axes.
 * The index is then read bit plane by bit plane from the top, axis 0 first. */
uint64_t ora_hilbert_index(uint32_t qx, uint32_t qy, uint32_t qz, int32_t bits)
{
    uint32_t X[3] = {qx, qy, qz};
    const int n = 3;
    uint32_t top = (uint32_t)1 << (bits - 1);
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < n; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;                        /* invert */
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;   /* exchange */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < n; ++i) X[i] ^= X[i - 1];  /* Gray encode */
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[n - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < n; ++i) X[i] ^= t;

    uint64_t h = 0;
    for (int j = bits - 1; j >= 0; --j)
        for (int i = 0; i < n; ++i)
            h = (h << 1) | ((X[i] >> j) & 1u);
    return h;
}

/* Background section, Dynamic Volume Lines: cells are represented by their
 * centroids, quantised, and the Hilbert code names the quantisation-grid
 * cell the centroid falls in.  Here the quantisation grid is the finest
 * logical grid; the centroid of a cell of width 2^L lies on the corner of
 * its finest sub-cell at offset 2^L / 2 (offset 0 for L = 0). */
void ora_cell_keys(int64_t n, const int32_t* x, const int32_t* y, const int32_t* z,
                   const uint8_t* level, int32_t bits, uint64_t* keys)
{
    for (int64_t h = 0; h < n; ++h) {
        uint32_t half = ((uint32_t)1 << level[h]) >> 1;
        keys[h] = ora_hilbert_index((uint32_t)x[h] + half, (uint32_t)y[h] + half,
                                    (uint32_t)z[h] + half, bits);
    }
}

typedef struct { uint64_t key; uint32_t idx; } ora_pair;

static int ora_pair_cmp(const void* a, const void* b)
{
    const ora_pair* p = (const ora_pair*)a;
    const ora_pair* q = (const ora_pair*)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

/* Abstract / Introduction: the cells are sorted on the space-filling curve;
 * ties (only possible for overlapping cells) are broken by original index
 * and counted. */
int64_t ora_sort_order(int64_t n, const uint64_t* keys, uint32_t* perm)
{
    ora_pair* a = (ora_pair*)malloc((size_t)(n > 0 ? n : 1) * sizeof(ora_pair));
    if (!a) return -1;
    for (int64_t h = 0; h < n; ++h) { a[h].key = keys[h]; a[h].idx = (uint32_t)h; }
    qsort(a, (size_t)n, sizeof(ora_pair), ora_pair_cmp);
    int64_t dup = 0;
    for (int64_t h = 0; h < n; ++h) {
        perm[h] = a[h].idx;
        if (h > 0 && a[h].key == a[h - 1].key) ++dup;
    }
    free(a);
    return dup;
}

/* ------------------------------------------------------------------ */
/* Transfer function                                                   */
/* ------------------------------------------------------------------ */

/* Interactive Transfer Function Updates: the field value is normalised to
 * the window [lo, hi] and mapped to one of the n_tf table entries. */
void ora_quantiser(int32_t n_tf, float lo, float hi, float* s, float* b)
{
    double sd = (double)n_tf / ((double)hi - (double)lo);
    float sf = (float)sd;
    *s = sf;
    *b = (float)(-(double)lo * (double)sf);
}

int32_t ora_tf_index(float x, float s, float b, int32_t n_tf)
{
    float t = fmaf(x, s, b);
    if (!(t >= 0.0f)) return 0;
    double fl = floor((double)t);
    if (fl > (double)(n_tf - 1)) return n_tf - 1;
    return (int32_t)fl;
}

/* ------------------------------------------------------------------ */
/* max(V_h): Eqs. 5-6 (approximation) and the exact maximum            */
/* ------------------------------------------------------------------ */

double ora_vmax_tf(int32_t mode, int32_t n_fields, int32_t n_tf, const float* alpha,
                   const int32_t* i_m, const int32_t* j_m)
{
    if (mode == ORA_VMAX_TF_RANGE) {
        /* Eq. 5: global index range; Eq. 6: V_a at every a of it */
        int32_t i = i_m[0], j = j_m[0];
        for (int32_t m = 1; m < n_fields; ++m) {
            if (i_m[m] < i) i = i_m[m];
            if (j_m[m] > j) j = j_m[m];
        }
        double best = 0.0;
        for (int32_t a = i; a <= j; ++a) {
            double hi = -INFINITY, lo = INFINITY;
            for (int32_t m = 0; m < n_fields; ++m) {
                double v = (double)alpha[(int64_t)m * n_tf + a];
                if (v > hi) hi = v;
                if (v < lo) lo = v;
            }
            if (hi - lo > best) best = hi - lo;
        }
        return best;
    }
    /* TF_BOUND: largest alpha any field can take minus smallest one */
    double hi = -INFINITY, lo = INFINITY;
    for (int32_t m = 0; m < n_fields; ++m)
        for (int32_t a = i_m[m]; a <= j_m[m]; ++a) {
            double v = (double)alpha[(int64_t)m * n_tf + a];
            if (v > hi) hi = v;
            if (v < lo) lo = v;
        }
    return hi - lo;
}

void ora_field_range(int64_t n, const float* v, float* vmin, float* vmax)
{
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t h = 0; h < n; ++h) {
        if (v[h] < lo) lo = v[h];
        if (v[h] > hi) hi = v[h];
    }
    *vmin = lo;
    *vmax = hi;
}

/* ------------------------------------------------------------------ */
/* Update                                                              */
/* ------------------------------------------------------------------ */

/* I(m,h): alpha of field m's TF at the cell's normalised value (Method
 * section: intensities come from the RGBA transfer function). */
static double ora_intensity(const float* fields, int64_t n, int32_t m, int64_t h,
                            const float* alpha, int32_t n_tf, const float* s, const float* b)
{
    float x = fields[(int64_t)m * n + h];
    int32_t a = ora_tf_index(x, s[m], b[m], n_tf);
    return (double)alpha[(int64_t)m * n_tf + a];
}

/* Eq. 1: V_h = max_m I(m,h) - min_m I(m,h). */
static double ora_variation(const float* fields, int64_t n, int32_t n_fields, int64_t h,
                            const float* alpha, int32_t n_tf, const float* s, const float* b)
{
    double hi = -INFINITY, lo = INFINITY;
    for (int32_t m = 0; m < n_fields; ++m) {
        double v = ora_intensity(fields, n, m, h, alpha, n_tf, s, b);
        if (v > hi) hi = v;
        if (v < lo) lo = v;
    }
    return hi - lo;
}

/* Eq. 3 (Eq. 2 when every level is 0): f = (V_h / max V_h * 2^L)^P with the
 * minimum importance enforced. */
static double ora_importance(double v, double vmax, int32_t lev, const ora_params* p)
{
    double r = vmax > 0.0 ? v / vmax : 0.0;
    double scale = ldexp(1.0, (p->level_scale == 3 ? 3 : 1) * lev);
    if (p->clamp_mode == 1) {
        double rc = r > p->min_importance ? r : p->min_importance;
        return pow(rc * scale, p->exponent);
    }
    double f = pow(r * scale, p->exponent);
    return f > p->min_importance ? f : p->min_importance;
}

int32_t ora_update(int64_t n, int32_t n_fields, const uint8_t* level, const float* fields,
                   int32_t n_tf, const float* alpha, const float* lo, const float* hi,
                   const ora_params* p, ora_bins* out, double* cell_f, double* cell_e)
{
    if (n < 1 || n_fields < 1 || n_tf < 2 || p->n_bins < 1) return -1;
    const int32_t M = n_fields, W = p->n_bins;

    float* s = (float*)malloc(sizeof(float) * (size_t)M);
    float* b = (float*)malloc(sizeof(float) * (size_t)M);
    int32_t* im = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    int32_t* jm = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    double* f = cell_f ? cell_f : (double*)malloc(sizeof(double) * (size_t)n);
    double* E = cell_e ? cell_e : (double*)malloc(sizeof(double) * (size_t)(n + 1));
    if (!s || !b || !im || !jm || !f || !E) return -1;

    /* normalisation windows and the TF entries present in the data */
    for (int32_t m = 0; m < M; ++m) {
        ora_quantiser(n_tf, lo[m], hi[m], &s[m], &b[m]);
        float dmin, dmax;
        ora_field_range(n, fields + (int64_t)m * n, &dmin, &dmax);
        im[m] = ora_tf_index(dmin, s[m], b[m], n_tf);
        jm[m] = ora_tf_index(dmax, s[m], b[m], n_tf);
    }

    /* max(V_h) */
    double vmax;
    if (p->vmax_mode == ORA_VMAX_EXACT) {
        vmax = 0.0;
        for (int64_t h = 0; h < n; ++h) {
            double v = ora_variation(fields, n, M, h, alpha, n_tf, s, b);
            if (v > vmax) vmax = v;
        }
    } else {
        vmax = ora_vmax_tf(p->vmax_mode, M, n_tf, alpha, im, jm);
        if (vmax <= 0.0 && p->vmax_mode == ORA_VMAX_TF_RANGE)
            vmax = ora_vmax_tf(ORA_VMAX_TF_BOUND, M, n_tf, alpha, im, jm);
    }
    out->vmax_used = vmax;

    /* importance per cell */
    for (int64_t h = 0; h < n; ++h)
        f[h] = ora_importance(ora_variation(fields, n, M, h, alpha, n_tf, s, b), vmax,
                              level[h], p);

    /* Eq. 4: prefix sum of the importance, Neumaier-compensated.  E(h) is
     * the exclusive prefix F(h-1), E(h+1) the inclusive one F(h). */
    out->degenerate = 0;
    for (int pass = 0; pass < 2; ++pass) {
        double sum = 0.0, comp = 0.0;
        E[0] = 0.0;
        for (int64_t h = 0; h < n; ++h) {
            double t = sum + f[h];
            if (fabs(sum) >= fabs(f[h])) comp += (sum - t) + f[h];
            else comp += (f[h] - t) + sum;
            sum = t;
            E[h + 1] = sum + comp;
        }
        if (E[n] > 0.0 || pass == 1) break;
        /* zero total width: fall back to a linear map */
        for (int64_t h = 0; h < n; ++h) f[h] = 1.0;
        out->degenerate = 1;
    }
    const double F = E[n];
    out->f_total = F;

    /* Projecting Cells to 1D: W zeroed bins; every cell's (xf1, xf2) is
     * projected to the integer bins it overlaps, each of which accumulates
     * the cell's value and increments its counter. */
    for (int32_t k = 0; k < W; ++k) {
        out->first[k] = UINT32_MAX;
        out->last[k] = 0;
        out->count[k] = 0;
        for (int32_t m = 0; m < M; ++m) {
            out->sum[(int64_t)m * W + k] = 0.0;
            out->vmin[(int64_t)m * W + k] = INFINITY;
            out->vmax[(int64_t)m * W + k] = -INFINITY;
        }
    }
    for (int64_t h = 0; h < n; ++h) {
        double xf1 = (E[h] * (double)W) / F;
        double xf2 = (E[h + 1] * (double)W) / F;
        double lo_b = floor(xf1);
        double hi_b = ceil(xf2) - 1.0;
        int32_t blo = lo_b > (double)(W - 1) ? W - 1 : (lo_b < 0.0 ? 0 : (int32_t)lo_b);
        int32_t bhi = hi_b > (double)(W - 1) ? W - 1 : (int32_t)hi_b;
        if (bhi < blo) bhi = blo;
        for (int32_t k = blo; k <= bhi; ++k) {
            if ((uint32_t)h < out->first[k]) out->first[k] = (uint32_t)h;
            if ((uint32_t)h > out->last[k] || out->count[k] == 0) out->last[k] = (uint32_t)h;
            out->count[k] += 1;
            for (int32_t m = 0; m < M; ++m) {
                float x = fields[(int64_t)m * n + h];
                int64_t o = (int64_t)m * W + k;
                out->sum[o] += (double)x;
                if (x < out->vmin[o]) out->vmin[o] = x;
                if (x > out->vmax[o]) out->vmax[o] = x;
            }
        }
    }

    /* Divide by the counter (mean) and apply the TF to get the bin height. */
    for (int32_t k = 0; k < W; ++k)
        for (int32_t m = 0; m < M; ++m) {
            int64_t o = (int64_t)m * W + k;
            if (out->count[k] == 0) {
                out->mean[o] = 0.0;
                out->y[o] = 0.0f;
                continue;
            }
            out->mean[o] = out->sum[o] / (double)out->count[k];
            int32_t a = ora_tf_index((float)out->mean[o], s[m], b[m], n_tf);
            out->y[o] = alpha[(int64_t)m * n_tf + a];
        }

    free(s); free(b); free(im); free(jm);
    if (!cell_f) free(f);
    if (!cell_e) free(E);
    return 0;
}


/* ------------------------------------------------------------------ */
/* Per-bin histograms (histogram heatmap)                              */
/* ------------------------------------------------------------------ */

/* Prototypical User Interface section: besides the lines, volume-line plots
 * can show a histogram heatmap, i.e. per bin the distribution of the values
 * of its cells.  The buckets partition the window [lo, hi] as the entries of
 * a table of H entries do, so a value's bucket is its entry under that
 * quantiser. */
int32_t ora_bin_histograms(int64_t n, const float* values, int32_t n_bins, const uint32_t* first,
                           const uint32_t* last, int32_t n_buckets, float lo, float hi, uint32_t* counts)
{
    if (n < 1 || n_bins < 1 || n_buckets < 1 || !(lo < hi)) return -1;
    float s, b;
    ora_quantiser(n_buckets, lo, hi, &s, &b);
    for (int64_t i = 0; i < (int64_t)n_bins * n_buckets; ++i) counts[i] = 0;
    for (int32_t bin = 0; bin < n_bins; ++bin) {
        if (first[bin] > last[bin] || (int64_t)last[bin] >= n) continue;
        for (int64_t h = first[bin]; h <= (int64_t)last[bin]; ++h) {
            int32_t k = ora_tf_index(values[h], s, b, n_buckets);
            counts[(int64_t)bin * n_buckets + k] += 1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Line rasterisation (RasterizeLines)                                 */
/* ------------------------------------------------------------------ */

static int32_t ora_row(float y, int32_t n_rows)
{
    float t = y * (float)n_rows;
    if (!(t >= 0.0f)) return 0;
    int32_t r = (int32_t)floorf(t);
    return r > n_rows - 1 ? n_rows - 1 : r;
}

/* GPU Implementation section: the volume lines are drawn either as
 * polylines through the bin heights or as bar charts. */
int32_t ora_rasterize(int32_t n_bins, const float* y, int32_t n_rows, int32_t mode, uint8_t* img)
{
    if (n_bins < 1 || n_rows < 1 || (mode != ORA_RASTER_POLYLINE && mode != ORA_RASTER_BARS)) return -1;
    memset(img, 0, (size_t)n_bins * (size_t)n_rows);
    for (int32_t b = 0; b < n_bins; ++b) {
        int32_t r0 = ora_row(y[b], n_rows), lo, hi;
        if (mode == ORA_RASTER_BARS) {
            lo = 0;
            hi = r0;
        } else {
            int32_t r1 = b + 1 < n_bins ? ora_row(y[b + 1], n_rows) : r0;
            lo = r0 < r1 ? r0 : r1;
            hi = r0 < r1 ? r1 : r0;
        }
        for (int32_t r = lo; r <= hi; ++r) img[(int64_t)r * n_bins + b] = 1;
    }
    return 0;
}
