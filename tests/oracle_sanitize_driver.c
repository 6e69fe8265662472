/* Drives every oracle entry point on small seeded inputs (random AMR-like
 * cells on a 2^5 grid, ragged sizes, W above and below the cell count, all
 * max(V) and clamp modes), for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: any out-of-bounds access, leak or undefined
 * operation aborts the run.  Prints one line per case and "ok" at the end.
 * Test infrastructure only (tests/test_oracle_sanitize.py builds and runs it). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dvl_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void) {   /* SplitMix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static float uniform(void) { return (float)((next_u64() >> 40) * (1.0 / 16777216.0)); }

static int run_case(int64_t n, int32_t M, int32_t W, int32_t vmax_mode, int32_t clamp_mode, double p) {
    /* distinct cells: single-level cells on a 32^3 grid picked without repeats */
    const int side = 32;
    int32_t* x = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* y = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* z = malloc(sizeof(int32_t) * (size_t)n);
    uint8_t* lev = malloc((size_t)n);
    uint8_t* used = calloc((size_t)side * side * side, 1);
    for (int64_t h = 0; h < n; ++h) {
        uint64_t c;
        do c = next_u64() % (uint64_t)(side * side * side); while (used[c]);
        used[c] = 1;
        x[h] = (int32_t)(c % side);
        y[h] = (int32_t)((c / side) % side);
        z[h] = (int32_t)(c / (side * side));
        lev[h] = 0;
    }
    const int32_t bits = ora_grid_bits(n, x, y, z, lev);
    uint64_t* keys = malloc(sizeof(uint64_t) * (size_t)n);
    uint32_t* perm = malloc(sizeof(uint32_t) * (size_t)n);
    ora_cell_keys(n, x, y, z, lev, bits, keys);
    const int64_t dup = ora_sort_order(n, keys, perm);

    const int32_t n_tf = 256;
    float* fields = malloc(sizeof(float) * (size_t)(M * n));
    float* alpha = malloc(sizeof(float) * (size_t)(M * n_tf));
    float* lo = malloc(sizeof(float) * (size_t)M);
    float* hi = malloc(sizeof(float) * (size_t)M);
    for (int32_t m = 0; m < M; ++m) {
        for (int64_t h = 0; h < n; ++h) fields[m * n + h] = uniform() * 10.0f - 3.0f;
        for (int32_t a = 0; a < n_tf; ++a) alpha[m * n_tf + a] = uniform();
        ora_field_range(n, fields + m * n, &lo[m], &hi[m]);
        if (!(hi[m] > lo[m])) hi[m] = lo[m] + 1.0f;
    }
    uint8_t* slev = malloc((size_t)n);
    float* sfields = malloc(sizeof(float) * (size_t)(M * n));
    for (int64_t h = 0; h < n; ++h) {
        slev[h] = lev[perm[h]];
        for (int32_t m = 0; m < M; ++m) sfields[m * n + h] = fields[m * n + perm[h]];
    }
    ora_params prm = {W, p, 0.025, vmax_mode, clamp_mode, 1};
    ora_bins b;
    memset(&b, 0, sizeof b);
    b.first = malloc(sizeof(uint32_t) * (size_t)W);
    b.last = malloc(sizeof(uint32_t) * (size_t)W);
    b.count = malloc(sizeof(uint32_t) * (size_t)W);
    b.sum = malloc(sizeof(double) * (size_t)(M * W));
    b.mean = malloc(sizeof(double) * (size_t)(M * W));
    b.vmin = malloc(sizeof(float) * (size_t)(M * W));
    b.vmax = malloc(sizeof(float) * (size_t)(M * W));
    b.y = malloc(sizeof(float) * (size_t)(M * W));
    double* cf = malloc(sizeof(double) * (size_t)n);
    double* ce = malloc(sizeof(double) * (size_t)(n + 1));
    const int32_t st = ora_update(n, M, slev, sfields, n_tf, alpha, lo, hi, &prm, &b, cf, ce);

    const int32_t H = 37;
    uint32_t* hist = malloc(sizeof(uint32_t) * (size_t)(W * H));
    const int32_t sh = ora_bin_histograms(n, sfields, W, b.first, b.last, H, lo[0], hi[0], hist);
    uint8_t* img = malloc((size_t)(W * 29));
    const int32_t s1 = ora_rasterize(W, b.y, 29, ORA_RASTER_POLYLINE, img);
    const int32_t s2 = ora_rasterize(W, b.y, 29, ORA_RASTER_BARS, img);
    int32_t i_m[16], j_m[16];
    for (int32_t m = 0; m < M; ++m) {
        i_m[m] = ora_tf_index(lo[m], 1.0f, 0.0f, n_tf);
        j_m[m] = n_tf - 1;
    }
    const double vt = ora_vmax_tf(ORA_VMAX_TF_RANGE, M, n_tf, alpha, i_m, j_m);

    printf("n=%lld M=%d W=%d mode=%d clamp=%d p=%g: bits %d dup %lld update %d hist %d raster %d/%d "
           "f_total %.6g vmax %.4g\n", (long long)n, M, W, vmax_mode, clamp_mode, p, bits, (long long)dup, st,
           sh, s1, s2, b.f_total, vt);
    const int bad = st != 0 || sh != 0 || s1 != 0 || s2 != 0 || dup != 0;
    free(x); free(y); free(z); free(lev); free(used); free(keys); free(perm);
    free(fields); free(alpha); free(lo); free(hi); free(slev); free(sfields);
    free(b.first); free(b.last); free(b.count); free(b.sum); free(b.mean); free(b.vmin); free(b.vmax); free(b.y);
    free(cf); free(ce); free(hist); free(img);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run_case(1, 1, 1, ORA_VMAX_TF_RANGE, 0, 1.0);
    bad |= run_case(5, 2, 7, ORA_VMAX_TF_BOUND, 1, 0.0);
    bad |= run_case(257, 4, 64, ORA_VMAX_EXACT, 0, 2.0);
    bad |= run_case(1000, 3, 1500, ORA_VMAX_TF_RANGE, 0, 0.5);
    bad |= run_case(4097, 16, 333, ORA_VMAX_EXACT, 1, 5.0);
    if (bad) {
        printf("FAILED\n");
        return 1;
    }
    printf("ok\n");
    return 0;
}
