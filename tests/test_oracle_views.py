"""Pins of the oracle's per-bin histograms (histogram heatmap) and line
rasterisation (RasterizeLines), CPU only.  Each pin states a fact fixed by
the definition or by an independent computation, not a retyped formula."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


# ---------------------------------------------------------------- histograms

def test_histogram_hand_example(ora):
    # 10 buckets over [0, 1]; bin 0 = cells 0..1, bin 1 = cells 2..3
    v = np.array([0.05, 0.15, 0.15, 0.95], np.float32)
    h = oracle.bin_histograms(v, [0, 2], [1, 3], 10, 0.0, 1.0)
    want = np.zeros((2, 10), np.uint32)
    want[0, 0] = want[0, 1] = want[1, 1] = want[1, 9] = 1
    assert np.array_equal(h, want)


def test_histogram_counts_sum_to_bin_sizes_with_straddles(ora):
    rng = np.random.default_rng(3)
    v = rng.random(1000).astype(np.float32)
    first = np.array([0, 99, 400, 400], np.uint32)     # bins share a straddling cell
    last = np.array([99, 400, 400, 999], np.uint32)
    h = oracle.bin_histograms(v, first, last, 17, 0.0, 1.0)
    assert np.array_equal(h.sum(axis=1), (last - first + 1).astype(np.uint32))


def test_histogram_matches_numpy_away_from_bucket_edges(ora):
    """numpy.histogram with explicit edges lo + k (hi - lo) / H is an
    independent definition; values within 1e-4 of an edge are dropped so
    that fp32 rounding of the quantiser cannot decide a bucket."""
    rng = np.random.default_rng(11)
    lo, hi, H = -3.0, 5.0, 64
    v = (rng.random(20000) * 9.0 - 3.5).astype(np.float32)
    v = np.clip(v, lo, np.nextafter(np.float32(hi), np.float32(-np.inf)))
    t = (v.astype(np.float64) - lo) * H / (hi - lo)
    keep = np.abs(t - np.round(t)) > 1e-4
    v = v[keep]
    n = v.size
    cuts = np.sort(rng.choice(np.arange(1, n), 9, replace=False))
    first = np.concatenate([[0], cuts]).astype(np.uint32)
    last = np.concatenate([cuts - 1, [n - 1]]).astype(np.uint32)
    h = oracle.bin_histograms(v, first, last, H, lo, hi)
    edges = lo + np.arange(H + 1) * (hi - lo) / H
    for b in range(first.size):
        ref, _ = np.histogram(v[first[b]:last[b] + 1].astype(np.float64), bins=edges)
        assert np.array_equal(h[b], ref), b


def test_histogram_values_outside_the_window_go_to_the_end_buckets(ora):
    v = np.array([-10.0, -0.001, 2.0, 1e9, 0.5], np.float32)
    h = oracle.bin_histograms(v, [0], [4], 4, 0.0, 2.0)
    assert h[0].tolist() == [2, 1, 0, 2]


# ---------------------------------------------------------------- raster

def _columns_are_runs(img):
    for b in range(img.shape[1]):
        rows = np.flatnonzero(img[:, b])
        assert rows.size >= 1, f"column {b} is empty"
        assert rows[-1] - rows[0] + 1 == rows.size, f"column {b} is not one run"


def test_raster_constant_line_is_one_row(ora):
    y = np.full(7, 0.5, np.float32)
    img = oracle.rasterize(y, 10, oracle.RASTER_POLYLINE)
    assert img.sum() == 7 and img[5].sum() == 7
    bars = oracle.rasterize(y, 10, oracle.RASTER_BARS)
    assert np.array_equal(bars.sum(axis=0), np.full(7, 6))
    assert bars[:6].all() and not bars[6:].any()


def test_raster_hand_example(ora):
    # H = 4: rows of 0, 1, 0.3 are 0, 3 (clamped from 4), 1
    y = np.array([0.0, 1.0, 0.3], np.float32)
    img = oracle.rasterize(y, 4, oracle.RASTER_POLYLINE)
    want = np.zeros((4, 3), np.uint8)
    want[0:4, 0] = 1          # from row 0 up to row 3
    want[1:4, 1] = 1          # from row 3 down to row 1
    want[1, 2] = 1            # the last column: its own row only
    assert np.array_equal(img, want)
    bars = oracle.rasterize(y, 4, oracle.RASTER_BARS)
    assert bars[:, 0].tolist() == [1, 0, 0, 0] and bars[:, 1].sum() == 4 and bars[:, 2].tolist() == [1, 1, 0, 0]


@pytest.mark.parametrize("seed", range(5))
def test_raster_invariants(ora, seed):
    rng = np.random.default_rng(seed)
    W, H = 257, 61
    y = rng.random(W).astype(np.float32)
    y[::17] = 1.0
    y[::23] = 0.0
    img = oracle.rasterize(y, H, oracle.RASTER_POLYLINE)
    _columns_are_runs(img)
    rows = np.minimum(H - 1, np.floor(y.astype(np.float64) * H)).astype(int)
    for b in range(W):
        col = np.flatnonzero(img[:, b])
        assert col[0] <= rows[b] <= col[-1]
        if b + 1 < W:                      # the segment to the next bin's height
            assert col[0] <= rows[b + 1] <= col[-1]
            assert col.size == abs(rows[b + 1] - rows[b]) + 1
        else:
            assert col.size == 1
    bars = oracle.rasterize(y, H, oracle.RASTER_BARS)
    _columns_are_runs(bars)
    assert np.array_equal(bars.sum(axis=0), rows + 1)
    assert bars[0].all()
