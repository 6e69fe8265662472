/* dvl.h -- C ABI of the MI355X dynamic-volume-line library.
 *
 * Dynamic volume lines (DVLs) over multi-field AMR data, after Zellmann,
 * Demirci and Gudukbay, "Visual Analysis of Large Multi-Field AMR Data on
 * GPUs Using Interactive Volume Lines" (arXiv 2306.11612).
 *
 * Two parts:
 *   ordering (once per volume)   dvl_build_order
 *   update (per TF/data change)  dvl_set_tf, dvl_update, dvl_read_bins
 *
 * Conventions
 *   - Plain C types only.  "device" pointers are HIP device allocations on
 *     the current device; "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it; calls return before it completes
 *     unless stated otherwise.
 *   - Every call returns a dvl_status; on failure dvl_last_error() returns a
 *     message (thread-local, valid until the next call on that thread).
 *     No call ever throws or aborts.
 *   - A volume may be used by one host thread at a time; distinct volumes
 *     are independent.  Updates of one volume must be issued on one stream
 *     (they share the volume's parameter block and workspace).
 *   - The library owns the volume's internal device buffers (sorted fields,
 *     levels, keys, permutation, statistics, entry cache, workspace).  It
 *     allocates them through the caller's dvl_allocator when one is given
 *     (dvl_build_options.allocator, dvl_executor_create_ex), else with
 *     hipMalloc; dvl_destroy gives them back the same way.
 */
#ifndef DVL_H
#define DVL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dvl_status;
#define DVL_OK          0
#define DVL_E_INVALID   1   /* an argument is out of its documented range */
#define DVL_E_NOMEM     2   /* a device or host allocation failed */
#define DVL_E_HIP       3   /* a HIP runtime call or kernel failed (sticky per volume) */
#define DVL_E_STATE     4   /* call not allowed in the volume's state (e.g. a field has no TF) */
#define DVL_E_OVERLAP   5   /* two cells share a Hilbert key: the AMR cells overlap */
#define DVL_E_RANGE     6   /* data out of range: negative corner, level > 20, grid
                               beyond 2^21 per axis, or a NaN field value */

/* storage type of the field values; arithmetic is always fp32 */
#define DVL_F32   0
#define DVL_F16   1
#define DVL_BF16  2

/* how max(V_h) of Eq. 2/3 is obtained (section "Computing the Maximum Local
 * Ensemble Variation") */
#define DVL_VMAX_TF_RANGE 0  /* Eqs. 5-6: max over TF entries a in [min i_m, max j_m]
                                of max_m A_m[a] - min_m A_m[a]; falls back to
                                TF_BOUND when that is 0 (default) */
#define DVL_VMAX_TF_BOUND 1  /* max_m max_{a in [i_m,j_m]} A_m[a] - min_m min A_m[a] */
#define DVL_VMAX_EXACT    2  /* max over all cells of V_h (one extra pass) */

/* arithmetic of the carry propagation of the Eq. 4 prefix sum across tiles */
#define DVL_SCAN_FP64        0  /* default */
#define DVL_SCAN_KAHAN_FP32  1  /* compensated fp32 */
#define DVL_SCAN_NAIVE_FP32  2  /* plain fp32, for error studies only */

typedef struct dvl_volume dvl_volume;

/* Device memory provider.  alloc returns `bytes` of device memory on the
 * current device (NULL when it cannot: the call then fails with DVL_E_NOMEM
 * and gives back everything it had taken); release takes back a pointer that
 * alloc returned.  `stream` is the HIP stream of the call that allocates or
 * releases (NULL when there is none).  The library releases a buffer only
 * after the device has finished every kernel it enqueued on it.  Both
 * functions are called from the thread of the library call, never
 * concurrently for one volume or executor.  The allocator (and `ctx`) must
 * outlive the volume or executor that uses it. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*release)(void* ctx, void* ptr, void* stream);
    void* ctx;
} dvl_allocator;

/* ---------------------------------------------------------------------
 * dvl_build_order -- one-time ordering (Background, AMR paragraph and
 * Dynamic Volume Lines; GPU section: the Hilbert order is computed once and
 * never changes, only the spacing does).
 *
 * Each AMR leaf cell is its lower corner (x, y, z) on the logical grid and
 * its level (0 = finest, width 2^level).  The cell's key is the 3b-bit
 * Hilbert index of its centroid's finest-level cell corner + 2^level / 2 on
 * the 2^b cube, b = smallest b >= 1 with 2^b >= max(corner + 2^level)
 * (b <= 21, so keys fit 63 bits).  Cells are radix-sorted by (key, original
 * index); the level and every field are gathered into that order and each
 * field's data range (min, max) is recorded.
 *
 *   n_cells        1 <= n_cells < 2^32
 *   x, y, z        device int32[n_cells], original cell order, >= 0
 *   level          device uint8[n_cells], <= 20
 *   n_fields       M, 1 <= M <= 16
 *   dtype          DVL_F32 | DVL_F16 | DVL_BF16 (storage of every field)
 *   fields         host array of M device pointers, each [n_cells] values
 *                  of `dtype` in original order
 *   out            receives the new volume (NULL on failure)
 *
 * Inputs are only read, and may be freed once the call returns.  The call
 * synchronises `stream`.  Errors: DVL_E_INVALID (arguments), DVL_E_RANGE
 * (coordinates, levels or NaN values), DVL_E_OVERLAP (duplicate keys),
 * DVL_E_NOMEM, DVL_E_HIP.
 * ------------------------------------------------------------------- */
dvl_status dvl_build_order(int64_t n_cells, const int32_t* x, const int32_t* y,
                           const int32_t* z, const uint8_t* level, int32_t n_fields,
                           int32_t dtype, const void* const* fields, void* stream,
                           dvl_volume** out);

/* Tuning of a volume's update layout, fixed at build time (results of an
 * update depend on it only through the summation order of the fp64 prefix).
 *   tile_steps   cells per tile = 256 * tile_steps; 8, 16 or 32 (0: 16).  The
 *                projection reads again only tiles that contain a bin edge.
 *   run_waves    the importance pass splits the tiles into at most this many
 *                runs of consecutive tiles, one wave each (0: 32 per compute
 *                unit); 64 <= run_waves <= 65536 otherwise.
 *   entry_cache  the TF entry of a cell (Eq. 1's lookup) depends on its value
 *                and the field's window and table size only, not on the
 *                alpha values.  With tables of at most 256 entries the volume
 *                may keep one byte per cell and field holding it, so that the
 *                importance pass reads M + 1 bytes per cell instead of the
 *                values; results are bitwise the same.  The cache is built
 *                for one set of windows and table sizes:
 *                DVL_ENTRY_CACHE_AUTO (0) when two consecutive updates use
 *                the same set, DVL_ENTRY_CACHE_ALWAYS on the first use of a
 *                set, DVL_ENTRY_CACHE_NEVER never.  A (re)build costs one
 *                pass over the fields on the update's stream (ordered by
 *                events against updates in flight on other streams; the host
 *                does not wait) and takes n_cells bytes per field. */
enum { DVL_ENTRY_CACHE_AUTO = 0, DVL_ENTRY_CACHE_ALWAYS = 1, DVL_ENTRY_CACHE_NEVER = 2 };
typedef struct {
    int32_t tile_steps;
    int32_t run_waves;
    int32_t entry_cache;
    const dvl_allocator* allocator;   /* NULL: hipMalloc / hipFree.  Copied;
                                         serves every device buffer of the
                                         volume, its entry cache and the
                                         workspace of its dvl_update calls */
} dvl_build_options;

/* Change the entry-cache policy of a volume (DVL_ENTRY_CACHE_*).  NEVER also
 * frees the cache (after synchronising the device).  Host only.  A cache
 * (re)build is ordered against updates in flight on other streams by events;
 * it never blocks the host. */
dvl_status dvl_set_entry_cache(dvl_volume* v, int32_t policy);
/* 1 if the volume holds a built TF entry cache, with the windows and table
 * sizes it was built for in lo/hi/n_tf (host [n_fields] each, any may be
 * NULL); 0 if not. */
int32_t dvl_entry_cache_info(const dvl_volume* v, float* lo, float* hi, int32_t* n_tf);

/* dvl_build_order with explicit options (NULL: defaults). */
dvl_status dvl_build_order_ex(int64_t n_cells, const int32_t* x, const int32_t* y,
                              const int32_t* z, const uint8_t* level, int32_t n_fields,
                              int32_t dtype, const void* const* fields,
                              const dvl_build_options* options, void* stream, dvl_volume** out);

/* ---------------------------------------------------------------------
 * dvl_set_field -- replace field m's values: the data change of the
 * Introduction (the volume lines are recomputed whenever the data or the
 * alpha TF changes); the Hilbert order of the GPU section stays fixed, only
 * the values move.
 *
 *   m        0 <= m < n_fields
 *   values   device [n_cells] of the volume's dtype, ORIGINAL cell order;
 *            must stay valid until `stream` has reached this call's work
 *
 * First the data range of the new values is taken and checked for NaN
 * (this synchronises `stream` once); a NaN returns DVL_E_RANGE and leaves the
 * volume unchanged.  Then the values are gathered into sorted order and the
 * per-tile / per-step statistics refreshed, asynchronously on `stream`; the
 * TF entry cache is invalidated.  A TF set earlier for m keeps its window.
 * Updates issued later must run on `stream` (or after it).  Errors:
 * DVL_E_INVALID, DVL_E_RANGE, DVL_E_HIP (sticky).
 * ------------------------------------------------------------------- */
dvl_status dvl_set_field(dvl_volume* v, int32_t m, const void* values, void* stream);

/* Data range [min, max] of field m (host outputs). */
dvl_status dvl_field_range(const dvl_volume* v, int32_t m, float* vmin, float* vmax);

/* ---------------------------------------------------------------------
 * dvl_set_tf -- alpha transfer function of field m (section Interactive
 * Transfer Function Updates).  The field value is normalised to the window
 * [lo, hi] and mapped to entry clamp(floor(fmaf(x, s, b)), 0, n_tf - 1),
 * s = (float)(n_tf / (hi - lo)), b = (float)(-lo * s); the entry's alpha is
 * the intensity I(m, h) of Eq. 1 and, applied to a bin's mean, the bin
 * height.
 *
 *   alpha   host float[n_tf], values in [0, 1]; copied, may be freed on return
 *   n_tf    2 <= n_tf <= 4096, and M * n_tf <= 16384 over the volume
 *   lo, hi  finite, lo < hi (use dvl_field_range for the data range)
 *
 * Host only; takes effect at the next dvl_update.  Waits for the previous
 * update's parameter upload if it is still in flight.
 * ------------------------------------------------------------------- */
dvl_status dvl_set_tf(dvl_volume* v, int32_t m, const float* alpha, int32_t n_tf,
                      float lo, float hi);

typedef struct {
    int32_t n_bins;          /* W: plot width in pixels, 1 <= W <= 2^20 */
    float exponent;          /* P of Eqs. 2/3, 0 <= P <= 16 */
    float min_importance;    /* >= 0; 0.025 in the paper's evaluation */
    int32_t vmax_mode;       /* DVL_VMAX_* */
    int32_t clamp_mode;      /* 0: f = max(fmin, (r s_L)^P) (default)
                                1: f = (max(fmin, r) s_L)^P */
    int32_t level_scale;     /* 1: s_L = 2^L (Eq. 3, default); 3: s_L = 8^L (cell volume) */
    int32_t scan_mode;       /* DVL_SCAN_* */
} dvl_params;

/* Per-bin outputs, all device pointers owned by the caller.
 *   first_cell, last_cell  uint32[W]: the bin holds sorted cells
 *                          first..last (count = last - first + 1)
 *   mean, vmin, vmax, y    float[M*W], index m*W + b: mean/min/max of the
 *                          stored field value over the bin's cells and the
 *                          height y = alpha_m[entry(mean)]
 *   f_total                double[1]: F(max h) of Eq. 4
 *   vmax_used              float[1]: the max(V_h) (or approximation) used
 */
typedef struct {
    uint32_t* first_cell;
    uint32_t* last_cell;
    float* mean;
    float* vmin;
    float* vmax;
    float* y;
    double* f_total;
    float* vmax_used;
} dvl_bins;

/* ---------------------------------------------------------------------
 * dvl_update -- one volume-line update (Eqs. 1-4 and section Projecting
 * Cells to 1D): per cell, TF lookup of every field, local variation V (Eq. 1),
 * importance f = (V / max V * 2^L)^P with the minimum importance (Eq. 3),
 * exclusive prefix E of f (Eq. 4), pixel interval [E W / F, (E + f) W / F);
 * every bin b with the interval overlapping [b, b + 1) gets the cell (box
 * basis; zero-width cells go to the bin holding their position); per bin
 * and field the mean, min and max of the stored values and y = alpha(mean).
 *
 * Asynchronous on `stream`; no host synchronisation.  Requires a TF for
 * every field (else DVL_E_STATE).  Outputs are complete when `stream`
 * reaches the end of the enqueued work.  Errors: DVL_E_INVALID,
 * DVL_E_STATE, DVL_E_NOMEM (workspace growth), DVL_E_HIP.
 * ------------------------------------------------------------------- */
dvl_status dvl_update(dvl_volume* v, const dvl_params* p, const dvl_bins* out, void* stream);

/* ---------------------------------------------------------------------
 * dvl_update_noalloc -- dvl_update for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results (bitwise the same as
 * dvl_update) and asynchrony; it calls no allocator and no hipMalloc.
 *
 * Its descriptors and workspace live in one fixed device scratch array of
 * dvl_update_noalloc_max_bytes() bytes (64 MiB) per device, held from the
 * first call on that device until the process ends; the descriptors are
 * written by kernels (no memcpy, no memset).  An update fits when 72 bytes
 * per 4096-cell tile, 8 bytes per bin and about 24 KB stay within it (about
 * 3.8e9 cells at W = 1920, whatever the field count); larger ones get
 * DVL_E_NOMEM with a message and nothing is enqueued.  It never stores f for the projection and never
 * builds the TF entry cache: it reads the cache only when the cache already
 * holds this update's windows and the volume was updated on this stream
 * before.  Every call on a device shares that device's scratch, which keeps
 * the last call's contents: calls that overlap on one device (other streams,
 * other threads) race, so the caller orders them (one stream).  The
 * volume's device must be current.  Errors: as dvl_update, and
 * DVL_E_INVALID when another device is current.
 * ------------------------------------------------------------------- */
dvl_status dvl_update_noalloc(dvl_volume* v, const dvl_params* p, const dvl_bins* out, void* stream);
/* size of the per-device scratch of dvl_update_noalloc */
size_t dvl_update_noalloc_max_bytes(void);

/* ---------------------------------------------------------------------
 * Batched updates (many volumes and TF requests in one launch per phase).
 * Each request is the update of Eqs. 1-4 and section Projecting Cells to 1D
 * (as dvl_update); the paper issued one CUDA stream per field and found no
 * gain (GPU Implementation), so here the batch shares launches instead.
 *
 * A request is one update of one volume with its own TFs, windows,
 * parameters and outputs; it does not touch the volume's own TF state.
 * Requests on the same volume (up to 8 at a time) share one read of its
 * cells in the importance pass.  Every request's results are bitwise equal
 * to those of a dvl_update with the same TFs and parameters, whatever else is
 * in the batch.  All requests of a batch must share the volumes' storage
 * dtype.
 * ------------------------------------------------------------------- */
typedef struct {
    dvl_volume* volume;
    const float* alpha;      /* host [n_fields][n_tf] alpha tables (field-major) */
    int32_t n_tf;            /* entries per table, 2..4096, n_fields * n_tf <= 16384 */
    const float* lo;         /* host [n_fields] windows, or NULL for the data ranges */
    const float* hi;
    dvl_params params;
    dvl_bins out;            /* device outputs, caller-owned, [n_fields][params.n_bins] */
} dvl_request;

/* An executor owns the device descriptors and per-request workspaces of the
 * batches it runs (grown on demand, reused afterwards).  Use one executor
 * from one host thread and one stream at a time; batches on different
 * streams need different executors. */
typedef struct dvl_executor dvl_executor;
dvl_status dvl_executor_create(dvl_executor** out);
/* ... with its workspaces and descriptor blocks from `allocator` (NULL:
 * hipMalloc).  The allocator is copied. */
dvl_status dvl_executor_create_ex(const dvl_allocator* allocator, dvl_executor** out);
void dvl_executor_destroy(dvl_executor* ex);
/* device bytes held (workspaces and descriptor buffers) */
size_t dvl_executor_bytes(const dvl_executor* ex);
/* device workspace a request on this volume with n_bins bins needs */
size_t dvl_request_bytes(const dvl_volume* v, int32_t n_bins);
/* per-kernel timing of this executor's batches (see dvl_set_timing) */
dvl_status dvl_executor_set_timing(dvl_executor* ex, int32_t enable);
dvl_status dvl_executor_kernel_times(dvl_executor* ex, double* ms, int32_t* n_batches);

/* Enqueue all requests on `stream`: one launch per phase for the whole
 * batch.  Asynchronous; errors as dvl_update (DVL_E_INVALID also for mixed
 * dtypes).  Outputs must not overlap between requests. */
dvl_status dvl_update_batch(dvl_executor* ex, const dvl_request* reqs, int32_t n_reqs, void* stream);

/* A captured batch: the requests (volumes, parameters, outputs, table sizes)
 * are fixed at creation and the kernels captured once into a HIP graph;
 * dvl_graph_set_tf changes a request's tables and windows, and
 * dvl_graph_launch uploads the descriptors and replays the graph.  The graph
 * owns its workspaces.  Launches of one graph must use one stream. */
typedef struct dvl_graph dvl_graph;
dvl_status dvl_graph_create(const dvl_request* reqs, int32_t n_reqs, dvl_graph** out);
dvl_status dvl_graph_set_tf(dvl_graph* g, int32_t req, const float* alpha, const float* lo,
                            const float* hi);
/* every request's tables at once: host arrays of n_reqs pointers (lo, hi may
 * be NULL, or hold NULL entries: the data ranges); the first failing request
 * is reported and the later ones are left as they were */
dvl_status dvl_graph_set_tf_all(dvl_graph* g, const float* const* alpha, const float* const* lo,
                                const float* const* hi);
dvl_status dvl_graph_launch(dvl_graph* g, void* stream);
void dvl_graph_destroy(dvl_graph* g);

/* dvl_read_bins -- the per-pixel bins of section Projecting Cells to 1D
 * (a counter and the projected values per bin) and the TF'd heights of
 * section Interactive Transfer Function Updates, copied to the host.
 * Synchronises `stream`, then copies to host arrays (any may be NULL):
 * count/first/last uint32[W], mean/vmin/vmax/y float[M*W], f_total[1],
 * vmax_used[1].  `bins` are an update's device outputs with n_bins = W. */
dvl_status dvl_read_bins(const dvl_volume* v, const dvl_bins* bins, int32_t n_bins,
                         void* stream, uint32_t* count, uint32_t* first, uint32_t* last,
                         float* mean, float* vmin, float* vmax, float* y,
                         double* f_total, float* vmax_used);

/* dvl_export_order -- the ordering of section Dynamic Volume Lines (cells
 * ordered along a Hilbert curve of their quantised centroids; Background,
 * cells on the finest-level logical grid): the Hilbert keys in ORIGINAL cell
 * order and the permutation (perm[h] = original index of the h-th sorted
 * cell), into caller-owned device arrays uint64[n_cells] and uint32[n_cells]
 * (either may be NULL).  Asynchronous. */
dvl_status dvl_export_order(const dvl_volume* v, uint64_t* keys, uint32_t* perm, void* stream);

/* Sorted level and field arrays, into caller-owned device arrays
 * (uint8[n_cells]; fields: host array of M device pointers, each
 * [n_cells] of the volume's dtype; entries may be NULL).  Asynchronous. */
dvl_status dvl_export_sorted(const dvl_volume* v, uint8_t* level, void* const* fields,
                             void* stream);

/* ---------------------------------------------------------------------
 * Brushing and linking (section Brushing and Linking): a region of interest
 * selected in the 1D plot travels to the 3D view as the first and last
 * Hilbert codes of its cells, and a cell sampled in 3D is highlighted when
 * its own Hilbert code lies in such a range.
 *
 * dvl_select_bins: the cells of bins b0..b1 of an update's outputs `bins`
 * (n_bins = W, 0 <= b0 <= b1 < W) are the sorted cells first..last
 * (first = first_cell[b0], last = last_cell[b1]); key_lo/key_hi are their
 * Hilbert keys (keys increase along the sorted order, so every cell of the
 * region has a key in [key_lo, key_hi] and no other cell does).  Host
 * outputs, any may be NULL; synchronises `stream` (after the update on it).
 * Errors: DVL_E_INVALID, DVL_E_STATE (bins not of this volume), DVL_E_HIP.
 *
 * dvl_select_mask: mask[i] = 1 for every cell i (ORIGINAL order) whose key
 * lies in one of the n_ranges closed ranges ranges[2k] .. ranges[2k + 1]
 * (host uint64 pairs, 1 <= n_ranges <= 128, copied), else 0.  mask: device
 * uint8[n_cells], caller-owned.  Asynchronous.
 * ------------------------------------------------------------------- */
dvl_status dvl_select_bins(const dvl_volume* v, const dvl_bins* bins, int32_t n_bins, int32_t b0, int32_t b1,
                           void* stream, uint32_t* first, uint32_t* last, uint64_t* key_lo, uint64_t* key_hi);
dvl_status dvl_select_mask(const dvl_volume* v, const uint64_t* ranges, int32_t n_ranges, uint8_t* mask,
                           void* stream);

/* ---------------------------------------------------------------------
 * dvl_zoom -- the zoom interaction proposed in the Conclusions: a new
 * volume holding the sorted cells first..last of `v` (typically a region
 * from dvl_select_bins), so that its volume line spends the whole plot width
 * on them.  Cell i of the new volume is sorted cell first + i of `v`: that
 * range is its original order (dvl_export_order returns the range's keys
 * and the identity permutation; dvl_set_field takes values in that order).
 * Levels, fields and keys are copied; data ranges and statistics are those
 * of the range; no TF is set.  opt: layout options as for
 * dvl_build_order_ex (NULL: defaults, and `v`'s allocator).  Synchronises
 * `stream`.  Errors: DVL_E_INVALID, DVL_E_NOMEM, DVL_E_HIP.
 * ------------------------------------------------------------------- */
dvl_status dvl_zoom(const dvl_volume* v, uint32_t first, uint32_t last, const dvl_build_options* opt,
                    void* stream, dvl_volume** out);

/* ---------------------------------------------------------------------
 * dvl_bin_histograms -- the histogram heatmap of volume-line plots
 * (section Prototypical User Interface): for every bin b of an update's
 * outputs `bins` (n_bins = W) and field m, counts[b * H + k] = the number of
 * the bin's cells whose value lies in bucket k of the window [lo, hi]
 * (H = n_buckets, 1 <= H <= 4096; the bucket of a value is its entry under
 * the quantiser of [lo, hi] for H entries, as for TF entries; values outside
 * the window count in the end buckets).  A cell shared by two bins counts in
 * both.  counts: device uint32[W * H], caller-owned.  Asynchronous (after
 * the update on `stream`).  Errors: DVL_E_INVALID.
 * ------------------------------------------------------------------- */
dvl_status dvl_bin_histograms(const dvl_volume* v, const dvl_bins* bins, int32_t n_bins, int32_t m,
                              int32_t n_buckets, float lo, float hi, uint32_t* counts, void* stream);

/* ---------------------------------------------------------------------
 * dvl_rasterize -- RasterizeLines (GPU Implementation section): the volume
 * lines drawn as polylines or bar charts.  y: device float[n_lines * W],
 * line l's heights (an update's y output, values in [0, 1]); image: device
 * uint8[n_lines * n_rows * W], image l row r (row 0 at the bottom) column b
 * at (l * n_rows + r) * W + b, 1 for a drawn pixel, else 0.  The row of a
 * height is min(n_rows - 1, floor(y * n_rows)) (fp32).
 * DVL_RASTER_POLYLINE: column b holds the rows from the row of y[b] to the
 * row of y[b + 1] (the last column: its own row); DVL_RASTER_BARS: rows 0 to
 * the row of y[b].  1 <= n_lines <= 16, 1 <= W <= 2^20, 1 <= n_rows <= 16384.
 * Asynchronous.  Errors: DVL_E_INVALID.
 * ------------------------------------------------------------------- */
#define DVL_RASTER_POLYLINE 0
#define DVL_RASTER_BARS     1
dvl_status dvl_rasterize(const float* y, int32_t n_lines, int32_t n_bins, int32_t n_rows, int32_t mode,
                         uint8_t* image, void* stream);

/* ---------------------------------------------------------------------
 * Per-kernel timing of updates (profiling aid).  With enable = 1, every
 * dvl_update records HIP events on its stream around each of its kernels:
 * phase 0 exact max(V) (VMAX_EXACT only), 1 tile sums of the importance,
 * 2 carry scan and tile classification (one kernel), 3 rescan of the tiles
 * holding a bin edge (bin cell ranges), 4 bin statistics (mean, min, max,
 * height per bin).  With
 * enable = 2 only the two events around phase 1 (the importance pass, the
 * dominant kernel) are recorded; the other phases read 0.  0 disables;
 * other values return DVL_E_INVALID.
 * dvl_kernel_times synchronises on the recorded events, returns the summed
 * milliseconds per phase (ms[5]) over the updates since the last call and
 * their number, and resets the sums.  Each recorded event adds a few
 * microseconds to an update.
 * ------------------------------------------------------------------- */
dvl_status dvl_set_timing(dvl_volume* v, int32_t enable);
dvl_status dvl_kernel_times(dvl_volume* v, double* ms, int32_t* n_updates);

/* ---------------------------------------------------------------------
 * Test hook of the carry hand-off (process-wide; read when a launch is
 * enqueued or a batch is captured).  The carry scan of Eq. 4 across runs
 * and the classification of the tiles (section Projecting Cells to 1D) run
 * as one kernel: each classifying workgroup polls a flag the request's scan
 * workgroup sets, and computes the carry itself after `polls` unanswered
 * polls (default 32768), writing the same values.  polls = 0 makes every
 * classifying workgroup take that path, so tests can check that it gives
 * the same bits.  DVL_E_INVALID for polls < 0.
 * ------------------------------------------------------------------- */
dvl_status dvl_set_carry_wait(int32_t polls);

int64_t dvl_num_cells(const dvl_volume* v);
int32_t dvl_num_fields(const dvl_volume* v);
int32_t dvl_grid_bits(const dvl_volume* v);
int32_t dvl_dtype(const dvl_volume* v);
/* device bytes held by the volume (buffers and current workspace) */
size_t dvl_volume_bytes(const dvl_volume* v);
/* Level segments of the sorted order: the padded cells split into segments
 * of 64 (*n_segments of them); a segment whose cells share one level is
 * uniform, the others (*n_mixed) hold mixed levels.  The update passes read
 * the level bytes of mixed segments only (plus one 32-bit code per 256 cells)
 * and take the level of a uniform segment from its code.  Either pointer may
 * be NULL.  Copies the codes to the host (synchronises the device). */
dvl_status dvl_level_segments(const dvl_volume* v, int64_t* n_segments, int64_t* n_mixed);
/* device workspace one update of this shape needs beyond the volume */
size_t dvl_update_workspace_bytes(int64_t n_cells, int32_t n_fields, int32_t n_bins);

/* Free the volume's device buffers (synchronises the device first). NULL ok. */
void dvl_destroy(dvl_volume* v);

/* Message of the calling thread's last failing call ("" if none). */
const char* dvl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DVL_H */
