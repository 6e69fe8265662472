"""Pins of the oracle's per-update computation (Eqs. 1-6 and the box-basis
projection) against hand-derived examples, closed forms, invariants and an
exact-rational brute force -- never against the oracle itself."""
import json
import math
import os
from fractions import Fraction as Q

import numpy as np
import pytest

from bruteforce import dvl_exact, entry

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


# ---------------------------------------------------------------- golden

def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_examples(ora, ex):
    b = ora.update(np.array(ex["level"], np.uint8), np.array(ex["fields"], np.float32),
                   np.array(ex["alpha"], np.float32), ex["lo"], ex["hi"], ex["n_bins"],
                   ex["exponent"], ex["min_importance"], keep_cells=True)
    e = ex["expect"]
    assert b.vmax_used == e["vmax_used"]
    assert b.f_total == pytest.approx(e["f_total"], rel=1e-15)
    assert np.allclose(b.cell_f, e["cell_f"], rtol=1e-15, atol=0)
    assert b.first.tolist() == e["first"]
    assert b.last.tolist() == e["last"]
    assert b.count.tolist() == e["count"]
    assert np.allclose(b.mean, e["mean"], rtol=1e-15, atol=0)
    assert b.vmin.tolist() == e["vmin"]
    assert b.vmax.tolist() == e["vmax"]
    assert b.y.tolist() == e["y"]


# ---------------------------------------------------------------- closed forms

def _uniform_variation_tfs(n_tf=256):
    """Two TFs, constant 1 and constant 0: every cell has V = 1 = max V."""
    return np.stack([np.ones(n_tf, np.float32), np.zeros(n_tf, np.float32)])


def test_uniform_variation_single_level_is_linear(ora):
    """Uniform variation gives a linear cell-to-pixel map: with N = 2^18
    cells and W = 2^10 bins every operation is exact, so bin b holds
    exactly cells 256 b .. 256 b + 255."""
    n, W = 1 << 18, 1 << 10
    rng = np.random.default_rng(1)
    fields = rng.random((2, n), dtype=np.float32)
    b = ora.update(np.zeros(n, np.uint8), fields, _uniform_variation_tfs(), [0, 0], [1, 1], W,
                   keep_cells=True)
    assert b.vmax_used == 1.0
    assert b.f_total == n
    assert np.array_equal(b.first, np.arange(W, dtype=np.uint32) * 256)
    assert np.array_equal(b.count, np.full(W, 256, np.uint32))
    # bin stats are plain block statistics of the data
    blk = fields.reshape(2, W, 256)
    assert np.array_equal(b.vmin, blk.min(axis=2))
    assert np.array_equal(b.vmax, blk.max(axis=2))
    assert np.allclose(b.mean, blk.astype(np.float64).mean(axis=2), rtol=1e-14)


@pytest.mark.parametrize("p,scale", [(1.0, 2), (2.0, 2), (1.0, 8)])
def test_uniform_variation_amr_widths(ora, p, scale):
    """With V = max V the importance is (2^L)^P (or (8^L)^P): the prefix at
    cell h is sum_{i<h} 2^(P L_i), a dyadic integer, exact in fp64."""
    rng = np.random.default_rng(2)
    n = 4096
    lev = rng.integers(0, 4, n).astype(np.uint8)
    fields = rng.random((2, n), dtype=np.float32)
    b = ora.update(lev, fields, _uniform_variation_tfs(), [0, 0], [1, 1], 64, p, 0.025,
                   level_scale=1 if scale == 2 else 3, keep_cells=True)
    w = (float(scale) ** lev.astype(np.float64)) ** p
    assert np.array_equal(b.cell_f, w)
    assert np.array_equal(b.cell_e, np.concatenate([[0.0], np.cumsum(w)]))
    assert b.f_total == w.sum()


def test_single_field_has_no_variation(ora):
    """M = 1: V = 0 everywhere, so every cell gets the minimum importance
    and the map is linear again (with P > 0)."""
    n, W = 1 << 12, 1 << 6
    rng = np.random.default_rng(3)
    x = rng.random((1, n), dtype=np.float32)
    lev = rng.integers(0, 3, n).astype(np.uint8)
    alpha = rng.random((1, 256), dtype=np.float32)
    b = ora.update(lev, x, alpha, [0], [1], W, 1.0, 0.03125, keep_cells=True)
    assert np.all(b.cell_f == 0.03125)
    assert np.array_equal(b.first, np.arange(W, dtype=np.uint32) * (n // W))


def test_identical_fields_have_no_variation(ora):
    n = 1000
    rng = np.random.default_rng(4)
    x = rng.random(n, dtype=np.float32)
    alpha = rng.random(256, dtype=np.float32)
    b = ora.update(np.zeros(n, np.uint8), np.stack([x, x, x]), np.stack([alpha] * 3),
                   [0] * 3, [1] * 3, 10, 1.0, 0.025, keep_cells=True)
    assert np.all(b.cell_f == 0.025)


def test_exponent_zero_is_linear(ora):
    """P = 0: (anything)^0 = 1 >= minimum importance, so every f = 1."""
    rng = np.random.default_rng(5)
    n = 2000
    lev = rng.integers(0, 4, n).astype(np.uint8)
    f = rng.random((3, n), dtype=np.float32)
    b = ora.update(lev, f, rng.random((3, 256), dtype=np.float32), [0] * 3, [1] * 3, 100, 0.0,
                   0.025, keep_cells=True)
    assert np.all(b.cell_f == 1.0)
    assert np.array_equal(b.first, np.arange(100, dtype=np.uint32) * 20)


def test_zero_total_width_falls_back_to_linear(ora):
    n = 300
    x = np.full((1, n), 0.5, np.float32)
    b = ora.update(np.zeros(n, np.uint8), x, np.full((1, 8), 0.5, np.float32), [0], [1], 3, 1.0, 0.0)
    assert b.degenerate
    assert b.f_total == n
    assert b.count.tolist() == [100, 100, 100]


# ---------------------------------------------------------------- invariants

def _small_volume(seed, base=8):
    import synth
    import oracle
    v = synth.make_amr(base, (0.4, 0.3), 4, seed, octaves=3, field_octaves=2)
    o = oracle.build_order(v.x.numpy(), v.y.numpy(), v.z.numpy(), v.level.numpy())
    F = np.stack([f.numpy()[o.perm] for f in v.fields])
    L = v.level.numpy()[o.perm]
    A = np.stack([t.numpy() for t in synth.make_tfs(seed, 4, (4, 8))])
    lo, hi = oracle.default_windows(F)
    return L, F, A, lo, hi


@pytest.mark.parametrize("seed,W,p,fmin", [(11, 64, 1.0, 0.025), (12, 257, 2.0, 0.025),
                                           (13, 1000, 3.0, 0.0), (14, 31, 0.5, 0.1)])
def test_structural_invariants(ora, seed, W, p, fmin):
    L, F, A, lo, hi = _small_volume(seed)
    n = L.size
    b = ora.update(L, F, A, lo, hi, W, p, fmin, keep_cells=True)
    # the last inclusive prefix is the total width
    assert b.cell_e[-1] == b.f_total
    assert np.all(np.diff(b.cell_e) >= 0)
    # every bin holds a contiguous, non-empty range of sorted cells
    assert np.all(b.count >= 1)
    assert np.array_equal(b.count.astype(np.int64), b.last.astype(np.int64) - b.first + 1)
    assert b.first[0] == 0 and b.last[-1] == n - 1
    # consecutive bins share at most the one straddling cell
    d = b.first[1:].astype(np.int64) - b.last[:-1]
    assert np.all((d == 0) | (d == 1))
    assert b.count.sum() == n + np.sum(d == 0)
    # the statistics are consistent
    assert np.all(b.vmin <= b.mean + 1e-12 * np.abs(b.mean)) and np.all(b.mean <= b.vmax + 1e-12 * np.abs(b.mean))
    for k in range(0, W, max(1, W // 17)):
        sl = slice(int(b.first[k]), int(b.last[k]) + 1)
        assert np.array_equal(b.vmin[:, k], F[:, sl].min(axis=1))
        assert np.array_equal(b.vmax[:, k], F[:, sl].max(axis=1))
        assert np.allclose(b.mean[:, k], F[:, sl].astype(np.float64).mean(axis=1), rtol=1e-13)


def test_whole_path_independent_of_input_order(ora):
    import synth
    import oracle
    v = synth.make_amr(6, (0.4, 0.3), 3, 21, octaves=3, field_octaves=2)
    A = np.stack([t.numpy() for t in synth.make_tfs(21, 3)])

    def run(sh):
        x, y, z, lev = (t.numpy()[sh] for t in (v.x, v.y, v.z, v.level))
        o = oracle.build_order(x, y, z, lev)
        F = np.stack([f.numpy()[sh][o.perm] for f in v.fields])
        lo, hi = oracle.default_windows(F)
        return oracle.update(lev[o.perm], F, A, lo, hi, 50)

    a = run(np.arange(v.n))
    bb = run(np.random.default_rng(0).permutation(v.n))
    for k in ("first", "last", "count", "mean", "vmin", "vmax", "y"):
        assert np.array_equal(getattr(a, k), getattr(bb, k)), k


def test_prefix_matches_correctly_rounded_sums(ora):
    """The compensated prefix stays within 2 ulp of the exactly rounded
    partial sums (math.fsum) over a skewed importance distribution."""
    rng = np.random.default_rng(6)
    n = 200_000
    lev = rng.integers(0, 5, n).astype(np.uint8)
    F = rng.random((3, n), dtype=np.float32)
    A = rng.random((3, 256), dtype=np.float32)
    b = ora.update(lev, F, A, [0] * 3, [1] * 3, 16, 2.5, 0.001, keep_cells=True)
    for h in list(range(0, n + 1, 9973)) + [n]:
        ref = math.fsum(b.cell_f[:h].tolist())
        assert abs(b.cell_e[h] - ref) <= 2 * np.spacing(ref) + 0.0


# ---------------------------------------------------------------- TF and max(V)

def test_quantiser_exact_window(ora):
    s, bb = ora.quantiser(4, 0.0, 4.0)
    assert (s, bb) == (1.0, 0.0)
    assert [ora.tf_index(v, s, bb, 4) for v in (-1.0, 0.0, 0.99, 1.0, 3.99, 4.0, 100.0)] == [0, 0, 0, 1, 3, 3, 3]


def test_quantiser_matches_exact_floor_away_from_edges(ora):
    rng = np.random.default_rng(8)
    for _ in range(200):
        lo = float(np.float32(rng.normal() * 10))
        hi = float(np.float32(lo + rng.random() * 100 + 1e-3))
        n_tf = int(rng.choice([2, 16, 256, 4096]))
        s, bb = ora.quantiser(n_tf, lo, hi)
        for x in np.float32(lo + (hi - lo) * rng.random(20)):
            t = (Q(float(x)) - Q(lo)) * n_tf / (Q(hi) - Q(lo))
            frac = t - (t.numerator // t.denominator)
            if min(frac, 1 - frac) < Q(1, 10 ** 4):
                continue
            assert ora.tf_index(float(x), s, bb, n_tf) == entry(float(x), lo, hi, n_tf)


def test_vmax_range_literal(ora):
    """Eqs. 5-6 on hand TFs: fields use entries [1,2] and [2,3]; the global
    range is [1,3]; V_a = |A0[a] - A1[a]| = .5, .25, .75 -> .75."""
    A = np.array([[0.0, 0.5, 0.5, 1.0], [1.0, 0.0, 0.25, 0.25]], np.float32)
    assert ora.vmax_tf(ora.VMAX_TF_RANGE, A, [1, 2], [2, 3]) == 0.75
    # bound: largest alpha inside each field's own range (A0[1..2] = .5,
    # A1[2..3] = .25) minus the smallest (.25); it can be below the literal
    # value, which also visits entries outside a field's own range
    assert ora.vmax_tf(ora.VMAX_TF_BOUND, A, [1, 2], [2, 3]) == 0.25


def test_vmax_range_is_not_an_upper_bound(ora):
    """Identical TFs give V_a = 0 at every entry although the two fields
    can sit at different entries (V_h > 0): the approximation falls back to
    the bound (a documented reading of the paper)."""
    A = np.array([[0.0, 1.0], [0.0, 1.0]], np.float32)
    F = np.array([[0.1, 0.9], [0.9, 0.1]], np.float32)
    assert ora.vmax_tf(ora.VMAX_TF_RANGE, A, [0, 0], [1, 1]) == 0.0
    b = ora.update(np.zeros(2, np.uint8), F, A, [0, 0], [1, 1], 2, keep_cells=True)
    assert b.vmax_used == 1.0
    assert np.all(b.cell_f == 1.0)


def test_bound_dominates_exact(ora):
    rng = np.random.default_rng(9)
    for _ in range(30):
        M, n = int(rng.integers(2, 5)), 500
        F = rng.random((M, n), dtype=np.float32) * rng.random((M, 1), dtype=np.float32)
        A = rng.random((M, 64), dtype=np.float32)
        lo, hi = np.zeros(M, np.float32), np.ones(M, np.float32)
        ex = ora.update(np.zeros(n, np.uint8), F, A, lo, hi, 4, vmax_mode=ora.VMAX_EXACT).vmax_used
        bd = ora.update(np.zeros(n, np.uint8), F, A, lo, hi, 4, vmax_mode=ora.VMAX_TF_BOUND).vmax_used
        assert bd >= ex


# ---------------------------------------------------------------- brute force

def _tiny_case(rng):
    """Tiny random case with values at TF entry centres (so the fp32 index
    equals the exact one), dyadic alphas and an integer exponent."""
    M = int(rng.integers(1, 4))
    n = int(rng.integers(1, 40))
    n_tf = int(rng.choice([4, 8, 16]))
    lev = rng.integers(0, 3, n).astype(np.uint8)
    ent = rng.integers(0, n_tf, (M, n))
    lo = np.zeros(M, np.float32)
    hi = np.full(M, float(n_tf), np.float32)
    F = (ent + 0.5).astype(np.float32)
    A = (rng.integers(0, 17, (M, n_tf)) / 16.0).astype(np.float32)
    W = int(rng.integers(1, 24))
    p = int(rng.integers(0, 3))
    fmin = float(rng.choice([0.0, 1 / 32, 1 / 8]))
    return M, n, n_tf, lev, F, A, lo, hi, W, p, fmin


def _near_edge(E, F, W, tol=1e-9):
    for e in E:
        x = e * W / F
        fr = x - (x.numerator // x.denominator)
        if 0 < fr < tol or 1 - tol < fr < 1:
            return True
    return False


@pytest.mark.parametrize("seed", range(60))
def test_against_exact_rational_bruteforce(ora, seed):
    rng = np.random.default_rng(1000 + seed)
    M, n, n_tf, lev, F, A, lo, hi, W, p, fmin = _tiny_case(rng)
    mode = ["range", "exact"][seed % 2]
    clamp = ["importance", "ratio"][(seed // 2) % 2]
    ex = dvl_exact(lev.tolist(), F.tolist(), A.tolist(), lo.tolist(), hi.tolist(), W, p, fmin,
                   mode, clamp)
    b = ora.update(lev, F, A, lo, hi, W, float(p), fmin,
                   vmax_mode=ora.VMAX_EXACT if mode == "exact" else ora.VMAX_TF_RANGE,
                   clamp_mode=0 if clamp == "importance" else 1, keep_cells=True)
    assert b.vmax_used == float(ex["vmax"])
    assert np.allclose(b.cell_f, [float(v) for v in ex["f"]], rtol=1e-15, atol=0)
    assert b.f_total == pytest.approx(float(ex["F"]), rel=1e-14)
    if _near_edge(ex["E"], ex["F"], W):
        pytest.skip("a cell boundary sits within 1e-9 of a bin edge")
    for k in range(W):
        mem = ex["members"][k]
        assert b.count[k] == len(mem)
        if mem:
            assert (b.first[k], b.last[k]) == (mem[0], mem[-1])
            for m in range(M):
                assert b.mean[m, k] == pytest.approx(float(ex["mean"][m][k]), rel=1e-14)
                assert b.vmin[m, k] == float(ex["vmin"][m][k])
                assert b.vmax[m, k] == float(ex["vmax_bin"][m][k])
                assert b.y[m, k] == float(ex["y"][m][k])
