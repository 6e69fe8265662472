"""Pins of the oracle's ordering step (Hilbert keys + sort) against
properties of the Hilbert curve and of sorting, not against itself.

The paper fixes only that cells are ordered along a Hilbert curve of their
quantised centroids (Background, Dynamic Volume Lines; Abstract).  It names
no curve variant or orientation, so the particular variant is parity
unpinned; these tests pin that the oracle's keys ARE a Hilbert order:
bijection, unit steps between consecutive keys, and recursive nesting of
aligned sub-cubes (the property that separates a Hilbert curve from other
continuous curves).
"""
import itertools

import numpy as np
import pytest


def _cube_points(k):
    r = np.arange(1 << k, dtype=np.int64)
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _keys_on_cube(ora, k):
    x, y, z = _cube_points(k)
    lev = np.zeros(x.size, np.uint8)
    return x, y, z, ora.cell_keys(x, y, z, lev, k)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bijection_and_unit_steps(ora, k):
    x, y, z, keys = _keys_on_cube(ora, k)
    n = 1 << (3 * k)
    # bijection onto [0, 8^k)
    assert keys.max() == n - 1
    assert np.array_equal(np.sort(keys), np.arange(n, dtype=np.uint64))
    # walk the curve: consecutive keys are face neighbours (L1 distance 1)
    order = np.argsort(keys)
    p = np.stack([x[order], y[order], z[order]], axis=1)
    step = np.abs(np.diff(p, axis=0)).sum(axis=1)
    assert np.all(step == 1)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_origin_is_first(ora, k):
    assert ora.hilbert_index(0, 0, 0, k) == 0


@pytest.mark.parametrize("k", [4, 5])
def test_aligned_subcubes_are_contiguous(ora, k):
    """Every aligned 2^j sub-cube occupies one contiguous range of 8^j keys,
    aligned to a multiple of 8^j (recursive Hilbert construction)."""
    x, y, z, keys = _keys_on_cube(ora, k)
    for j in range(1, k):
        blk = (x >> j) + ((y >> j) << (k - j)) + ((z >> j) << (2 * (k - j)))
        n_blk = 1 << (3 * (k - j))
        kmin = np.full(n_blk, np.iinfo(np.uint64).max, np.uint64)
        kmax = np.zeros(n_blk, np.uint64)
        np.minimum.at(kmin, blk, keys)
        np.maximum.at(kmax, blk, keys)
        span = 1 << (3 * j)
        assert np.all(kmax - kmin == span - 1)
        assert np.all(kmin % span == 0)


def test_endpoints_are_cube_corners(ora):
    # a Hilbert curve starts and ends at corners of the cube that share an edge
    k = 4
    x, y, z, keys = _keys_on_cube(ora, k)
    n = 1 << k
    last = np.argmax(keys)
    end = (x[last], y[last], z[last])
    assert all(c in (0, n - 1) for c in end)
    assert sum(c != 0 for c in end) == 1


@pytest.mark.parametrize("case,expect", [
    (([0], [0], [0], [0]), 1),
    (([1], [0], [0], [0]), 1),          # upper corner 2 -> 2^1
    (([2], [0], [0], [0]), 2),          # upper corner 3 -> 2^2
    (([0], [0], [0], [3]), 3),          # width 8 -> 2^3
    (([56], [0], [0], [3]), 6),         # 56 + 8 = 64
    (([57], [0], [0], [0]), 6),         # 58 <= 64
    (([64], [0], [0], [0]), 7),         # 65 -> 2^7
    (([-1], [0], [0], [0]), -1),        # negative corner
    (([0], [0], [0], [21]), -1),        # level above 20
    (([(1 << 21) - 1], [0], [0], [0]), 21),
    (([1 << 21], [0], [0], [0]), -1),   # beyond 21 bits
])
def test_grid_bits(ora, case, expect):
    assert ora.grid_bits(*[np.array(c) for c in case]) == expect


def _random_amr(seed, base=4, levels=3, frac=0.4):
    """Tiny aligned AMR: random refinement of a base grid."""
    rng = np.random.default_rng(seed)
    lmax = levels - 1
    r = np.arange(base) << lmax
    cur = np.array(list(itertools.product(r, r, r)), np.int64)
    leaves, lev = [], []
    for L in range(lmax, 0, -1):
        ref = rng.random(cur.shape[0]) < frac
        leaves.append(cur[~ref]); lev.append(np.full((~ref).sum(), L))
        half = 1 << (L - 1)
        off = np.array(list(itertools.product((0, 1), repeat=3)), np.int64) * half
        cur = (cur[ref][:, None, :] + off[None]).reshape(-1, 3)
    leaves.append(cur); lev.append(np.zeros(cur.shape[0], int))
    c = np.concatenate(leaves)
    return c[:, 0].astype(np.int32), c[:, 1].astype(np.int32), c[:, 2].astype(np.int32), \
        np.concatenate(lev).astype(np.uint8)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_representative_point_does_not_change_order(ora, seed):
    """For cells aligned to their own width, the sorted order does not
    depend on which finest sub-cell represents the centroid: every aligned
    block is one contiguous key range, and blocks do not overlap."""
    x, y, z, lev = _random_amr(seed)
    b = ora.grid_bits(x, y, z, lev)
    k_centre = ora.cell_keys(x, y, z, lev, b)
    k_corner = ora.cell_keys(x, y, z, np.zeros_like(lev), b)  # lower corner as representative
    far = ((1 << lev.astype(np.int64)) - 1).astype(np.int32)
    k_far = ora.cell_keys(x + far, y + far, z + far, np.zeros_like(lev), b)
    o1 = np.argsort(k_centre, kind="stable")
    assert np.array_equal(o1, np.argsort(k_corner, kind="stable"))
    assert np.array_equal(o1, np.argsort(k_far, kind="stable"))


@pytest.mark.parametrize("seed", [0, 5])
def test_amr_cells_cover_contiguous_ranges(ora, seed):
    """Expanding each AMR cell into its finest sub-cells gives disjoint key
    ranges of length 8^L that partition the cube's keys covered by cells."""
    x, y, z, lev = _random_amr(seed, base=2, levels=3, frac=0.5)
    b = ora.grid_bits(x, y, z, lev)
    lo, hi = [], []
    for i in range(x.size):
        w = 1 << int(lev[i])
        r = np.arange(w)
        pts = np.array(list(itertools.product(r, r, r)))
        ks = ora.cell_keys(x[i] + pts[:, 0], y[i] + pts[:, 1], z[i] + pts[:, 2],
                           np.zeros(len(pts), np.uint8), b)
        assert ks.max() - ks.min() == w ** 3 - 1
        lo.append(int(ks.min())); hi.append(int(ks.max()))
    o = np.argsort(lo)
    lo, hi = np.array(lo)[o], np.array(hi)[o]
    assert np.all(lo[1:] == hi[:-1] + 1)


def test_sort_matches_stable_library_sort(ora):
    rng = np.random.default_rng(7)
    keys = rng.integers(0, 1 << 40, size=50_000, dtype=np.uint64)
    keys[::97] = keys[5]                      # plant ties
    perm, dup = ora.sort_order(keys)
    assert np.array_equal(perm, np.argsort(keys, kind="stable").astype(np.uint32))
    assert dup == np.sum(np.diff(np.sort(keys)) == 0)


def test_order_independent_of_input_order(ora):
    x, y, z, lev = _random_amr(11, base=4, levels=3)
    o = ora.build_order(x, y, z, lev)
    assert o.duplicates == 0
    rng = np.random.default_rng(3)
    sh = rng.permutation(x.size)
    o2 = ora.build_order(x[sh], y[sh], z[sh], lev[sh])
    a = np.stack([x[o.perm], y[o.perm], z[o.perm], lev[o.perm]])
    b = np.stack([x[sh][o2.perm], y[sh][o2.perm], z[sh][o2.perm], lev[sh][o2.perm]])
    assert np.array_equal(a, b)


def test_overlapping_cells_reported(ora):
    # a coarse cell and one of its own finest sub-cells share a representative
    x = np.array([0, 1], np.int32); y = np.array([0, 1], np.int32); z = np.array([0, 1], np.int32)
    lev = np.array([1, 0], np.uint8)
    assert ora.build_order(x, y, z, lev).duplicates == 1
