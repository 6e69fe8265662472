"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Keys and the permutation must match bit-exactly; bins are reconciled as
described in parity.py (edge tolerance 1e-6 on the normalised axis, mean
relative 1e-5, min/max bitwise)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import check_order, dvl, random_amr, run_case, subset, tfs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


# ---------------------------------------------------------------- ordering

@pytest.mark.parametrize("seed,base,levels", [(0, 4, 3), (1, 6, 4), (2, 3, 2), (3, 8, 3)])
def test_order_random_amr(seed, base, levels):
    D = dvl()
    vol = random_amr(seed, base, levels)
    dev = vol.to("cuda")
    print(f"[order] seed={seed} n={vol.n}", flush=True)
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        check_order(V, vol)
    finally:
        V.close()


@pytest.mark.parametrize("n", [1, 2, 63, 4095, 4097, 12345])
def test_order_ragged_sizes(n):
    D = dvl()
    vol = subset(random_amr(7, 16, 3, 0.3), n, seed=n)
    dev = vol.to("cuda")
    print(f"[order] n={n}", flush=True)
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        check_order(V, vol)
        lev, fl = V.export_sorted()
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        assert np.array_equal(lev.cpu().numpy(), vol.level.numpy()[p])
        for m in range(vol.m):
            assert np.array_equal(fl[m].cpu().numpy(), vol.fields[m].numpy()[p])
    finally:
        V.close()


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_order_from_offset_views(offset):
    """Coordinates and levels passed as views that start `offset` elements into
    larger buffers: unaligned starts take the one-cell-per-thread key and extent
    kernels, aligned ones the four-cell kernels; the order is the same."""
    D = dvl()
    vol = subset(random_amr(11, 12, 3, 0.3), 9001, seed=offset)
    n = vol.n
    def shifted(t):
        big = torch.zeros(n + 8, dtype=t.dtype, device="cuda")
        big[offset:offset + n] = t.to("cuda")
        return big[offset:offset + n]
    x, y, z, lev = (shifted(t) for t in (vol.x, vol.y, vol.z, vol.level))
    assert (x.data_ptr() % 16 == 0) == (offset == 0)
    fields = [f.to("cuda") for f in vol.fields]
    print(f"[order] offset={offset} n={n}", flush=True)
    V = D.build_order(x, y, z, lev, fields)
    try:
        check_order(V, vol)
    finally:
        V.close()


def test_order_cfg1_grid():
    import synth
    D = dvl()
    vol = synth.cfg1()
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        o = check_order(V, vol)
        assert o.bits == 6
    finally:
        V.close()


# ---------------------------------------------------------------- update

def test_cfg1_grid_update():
    import synth
    vol = synth.cfg1()
    run_case(vol, tfs(synth.SEED + 1, 4, n_cp=(4, 4)), 1024, label="cfg1")


def _expected_level_segments(level_sorted: np.ndarray, n_pad: int):
    lv = np.zeros(n_pad, np.uint8)
    lv[: level_sorted.size] = level_sorted
    seg = lv.reshape(-1, 64)
    return seg.shape[0], int(np.sum(seg.min(1) != seg.max(1)))


@pytest.mark.parametrize("seed,frac,entry_cache", [(4, 0.4, 0), (5, 0.7, 1), (6, 0.2, 2)])
def test_level_segments_and_codes(seed, frac, entry_cache):
    """The per-step level codes (64-cell segments of one level) against the
    sorted levels, and an update that reads them against the oracle."""
    vol = random_amr(seed, base=8, levels=4, frac=frac, n_fields=3)
    D = dvl()
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        lev, _ = V.export_sorted()
        n_pad = -(-vol.n // 4096) * 4096
        got = V.level_segments()
        exp = _expected_level_segments(lev.cpu().numpy(), n_pad)
        assert got == exp, (got, exp)
        assert 0 < got[1] < got[0]      # both kinds present
    finally:
        V.close()
    run_case(vol, tfs(seed, 3), 300, label=f"codes seed {seed}", entry_cache=entry_cache)
    run_case(vol, tfs(seed + 1, 3), 300, level_scale=3, label=f"codes seed {seed} l3", entry_cache=entry_cache)


def test_uniform_nonzero_level():
    """Every cell at level 2 (a regular grid of 4-wide cells): every segment
    of real cells is uniform with a nonzero code."""
    import itertools
    import synth
    rng = np.random.default_rng(9)
    c = np.array(list(itertools.product(range(0, 64, 4), repeat=3)), np.int32)[:3000]
    n = c.shape[0]
    fields = [torch.from_numpy(rng.lognormal(0, 1, n).astype(np.float32)) for _ in range(2)]
    vol = synth.Volume(torch.from_numpy(c[:, 0].copy()), torch.from_numpy(c[:, 1].copy()),
                       torch.from_numpy(c[:, 2].copy()), torch.full((n,), 2, dtype=torch.uint8), fields,
                       ["a", "b"], 16, 1, [])
    D = dvl()
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        ns, nm = V.level_segments()
        assert ns == 4096 // 64 and nm == (1 if n % 64 else 0)   # the segment shared with the padding
    finally:
        V.close()
    for cache in (0, 1, 2):
        run_case(vol, tfs(9, 2), 100, label="all level 2", entry_cache=cache)
        run_case(vol, tfs(10, 2), 100, level_scale=3, exponent=2.0, label="all level 2, p=2", entry_cache=cache)


def test_uniform_variation_is_exactly_linear():
    """TFs constant 1 and 0 give V = max V at every cell: with N = 2^18 and
    W = 2^10 every GPU operation is exact, so bin b is cells 256b..256b+255."""
    import synth
    D = dvl()
    vol = synth.cfg1()
    A = np.stack([np.ones(256, np.float32), np.zeros(256, np.float32)] * 2)
    g, ob, rep = run_case(vol, A, 1024, label="uniform-variation")
    assert np.array_equal(g["first"], np.arange(1024, dtype=np.uint32) * 256)
    assert np.array_equal(g["count"], np.full(1024, 256, np.uint32))
    assert rep.edges_moved == 0


@pytest.mark.parametrize("exponent,fmin,vmax_mode,clamp,lscale,W", [
    (1.0, 0.025, 0, 0, 1, 1920),
    (1.0, 0.025, 1, 0, 1, 1024),
    (1.0, 0.025, 2, 0, 1, 1920),
    (2.0, 0.025, 0, 0, 1, 1920),
    (5.0, 0.025, 0, 0, 1, 3840),
    (0.0, 0.025, 0, 0, 1, 500),
    (0.5, 0.25, 0, 0, 1, 777),
    (3.0, 0.0, 0, 0, 1, 1920),
    (1.0, 0.025, 0, 1, 1, 1920),
    (1.0, 0.025, 0, 0, 3, 1920),
    (2.0, 0.1, 2, 1, 3, 257),
])
def test_small_amr_params(exponent, fmin, vmax_mode, clamp, lscale, W):
    import synth
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 31, octaves=3, field_octaves=2)
    run_case(vol, tfs(31, 4), W, exponent, fmin, vmax_mode, clamp, lscale,
             label=f"amr16 p={exponent}")


@pytest.mark.parametrize("exponent,fmin,vmax_mode,clamp,lscale,W,dtype", [
    (1.0, 0.025, 0, 0, 1, 1920, torch.float32),
    (2.0, 0.025, 2, 0, 1, 777, torch.float32),
    (0.5, 0.1, 1, 1, 3, 64, torch.float32),
    (1.0, 0.025, 0, 0, 1, 1920, torch.float16),
    (3.0, 0.0, 2, 0, 1, 300, torch.bfloat16),
])
def test_entry_cache_parity(exponent, fmin, vmax_mode, clamp, lscale, W, dtype):
    """Updates that read the cached TF entries (built on first use) instead of
    the values: same oracle parity."""
    import synth
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 33, octaves=3, field_octaves=2)
    run_case(vol, tfs(33, 4), W, exponent, fmin, vmax_mode, clamp, lscale, dtype=dtype, entry_cache=1,
             label="entry cache")


@pytest.mark.parametrize("n", [1, 255, 4097, 9000])
def test_entry_cache_ragged(n):
    vol = subset(random_amr(19, 16, 3, 0.3, n_fields=3), n, seed=n)
    run_case(vol, tfs(n + 1, 3), 64, entry_cache=1, label=f"entry cache ragged {n}")


def test_entry_cache_paths_agree_bitwise():
    """The same updates through the value path, the automatic cache (built by
    the second update with unchanged windows) and a cache rebuilt after a
    window change give bitwise equal bins."""
    import synth
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3), 4, 63, octaves=3, field_octaves=2).to("cuda")
    outs = {}
    for policy in (D.ENTRY_CACHE_NEVER, D.ENTRY_CACHE_AUTO, D.ENTRY_CACHE_ALWAYS):
        V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields, entry_cache=policy)
        try:
            res = []
            for k in range(5):
                A = tfs(700 + k, 4)
                for m in range(4):
                    lo, hi = V.field_range(m)
                    if k == 3:                      # a window change, then back
                        hi = hi * 0.5 + lo * 0.5
                    D.set_tf(V, m, A[m], lo, hi)
                b = D.Bins(1920, 4)
                V.update(b, exponent=2.0)
                res.append(V.read_bins(b))
            outs[policy] = res
        finally:
            V.close()
    for policy in (D.ENTRY_CACHE_AUTO, D.ENTRY_CACHE_ALWAYS):
        for k in range(5):
            for key in ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used"):
                a, b = np.asarray(outs[policy][k][key]), np.asarray(outs[D.ENTRY_CACHE_NEVER][k][key])
                assert a.tobytes() == b.tobytes(), (policy, k, key)


def test_entry_cache_follows_set_field(cfg2_base64):
    """A data change invalidates the cached entries."""
    import synth
    from parity import reconcile
    D = dvl()
    vol = cfg2_base64
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields, entry_cache=D.ENTRY_CACHE_ALWAYS)
    try:
        A = tfs(78, 4)
        lo0 = [V.field_range(m)[0] for m in range(4)]
        hi0 = [V.field_range(m)[1] for m in range(4)]
        for m in range(4):
            D.set_tf(V, m, A[m], lo0[m], hi0[m])
        b = D.Bins(32, 4)
        V.update(b)                      # builds the cache for these windows
        V.read_bins(b)
        new = dev.fields[1] * 0.5 + 0.25
        V.set_field(1, new)
        for m in range(4):               # same windows: a stale cache would be used if not invalidated
            D.set_tf(V, m, A[m], lo0[m], hi0[m])
        V.update(b)
        g = V.read_bins(b)
        fields = list(vol.fields)
        fields[1] = new.cpu()
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        F = np.stack([f.numpy()[p] for f in fields])
        lo, hi = np.array(lo0, np.float32), np.array(hi0, np.float32)
        ob = oracle.update(vol.level.numpy()[p], F, A, lo, hi, 32, keep_cells=True)
        reconcile(g, ob, F, A, lo, hi, 32)
    finally:
        V.close()


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_sixteen_bit_storage(dtype):
    import synth
    vol = synth.make_amr(16, (0.4, 0.3), 4, 41, octaves=3, field_octaves=2)
    run_case(vol, tfs(41, 4), 1920, dtype=dtype, label=str(dtype))


@pytest.mark.parametrize("scan_mode", [0, 1])
def test_carry_modes(scan_mode):
    import synth
    vol = synth.make_amr(24, (0.4, 0.3, 0.2), 4, 51, octaves=3, field_octaves=2)
    run_case(vol, tfs(51, 4), 1920, scan_mode=scan_mode, label=f"scan{scan_mode}")


@pytest.mark.parametrize("n", [1, 5, 255, 257, 4096, 4097, 9000])
def test_ragged_cell_counts(n):
    vol = subset(random_amr(9, 16, 3, 0.3, n_fields=2), n, seed=n)
    run_case(vol, tfs(n, 2), 64, label=f"ragged {n}")


@pytest.mark.parametrize("n_fields,n_tf", [(16, 1024), (4, 4096), (5, 256), (8, 256), (3, 300)])
def test_field_and_table_limits(n_fields, n_tf):
    """The most fields (16) and the largest tables (4096 entries; 16 * 1024 =
    16384 floats in all), field counts served by the general kernel variant
    (3, 5, 16) and by the fixed ones (8), tables too large for the entry cache."""
    vol = random_amr(17, 6, 3, 0.4, n_fields=n_fields)
    run_case(vol, tfs(n_fields * 7 + n_tf, n_fields, n_tf=n_tf), 500, exponent=1.5,
             label=f"M={n_fields} n_tf={n_tf}")


def test_most_bins():
    """W = 2^20 bins over ~2.6 k cells: every cell spans hundreds of bins."""
    vol = random_amr(18, 4, 3, 0.4, n_fields=2)
    g, _, _ = run_case(vol, tfs(18, 2), 1 << 20, label="W=2^20")
    assert np.all(g["count"] >= 1)


def test_more_bins_than_cells():
    """Cells wider than a pixel: interior bins hold exactly one cell."""
    vol = random_amr(11, 6, 3, 0.4, n_fields=3)
    g, ob, rep = run_case(vol, tfs(11, 3), 3840, exponent=2.0, label="wide cells")
    assert np.any(g["count"] == 1)


def test_single_bin():
    vol = random_amr(12, 8, 3, 0.4, n_fields=2)
    g, _, _ = run_case(vol, tfs(12, 2), 1, label="W=1")
    assert g["first"][0] == 0 and g["last"][0] == vol.n - 1


def test_zero_total_width_is_linear():
    """One field: V = 0 everywhere; with minimum importance 0 every f is 0
    and the update falls back to the linear map."""
    vol = random_amr(13, 8, 3, 0.4, n_fields=1)
    g, ob, rep = run_case(vol, tfs(13, 1), 100, fmin=0.0, label="degenerate")
    assert ob.degenerate
    assert g["f_total"] == vol.n


def test_determinism():
    import synth
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3), 4, 61, octaves=3, field_octaves=2).to("cuda")
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        A = tfs(61, 4)
        for m in range(4):
            V.set_tf(m, A[m])
        outs = []
        for _ in range(3):
            b = D.Bins(1920, 4)
            V.update(b, exponent=2.0)
            outs.append(V.read_bins(b))
        for k in ("first", "last", "mean", "vmin", "vmax", "y"):
            assert np.array_equal(outs[0][k], outs[1][k]) and np.array_equal(outs[0][k], outs[2][k]), k
    finally:
        V.close()


@pytest.fixture(scope="module")
def cfg2_base64():
    import synth
    return synth.cfg2(device="cuda", base=64).to("cpu")


@pytest.mark.parametrize("W,exponent", [(1920, 1.0), (64, 1.0), (7, 2.0), (1, 1.0), (300, 0.0)])
def test_cfg2_scaled(cfg2_base64, W, exponent):
    """The 3-level AMR workload at base 64 (about 1.5 M cells).  With few
    bins most 4096-cell tiles fall inside one bin and take their statistics
    from the per-tile precomputation instead of a rescan."""
    import synth
    run_case(cfg2_base64, tfs(synth.SEED + 2, 4, n_cp=(4, 4)), W, exponent=exponent,
             label=f"cfg2/base64 W={W}")


@pytest.mark.parametrize("W", [16, 48, 300])
def test_entry_cache_projection_paths(cfg2_base64, W):
    """The projection from cached entries (few bins: most tiles take their
    precomputed statistics, the rest are rescanned from entries) and from the
    importance the first pass stored (bins >= a quarter of the tiles)."""
    import synth
    run_case(cfg2_base64, tfs(synth.SEED + 5, 4, n_cp=(4, 8)), W, exponent=1.5, entry_cache=1,
             label=f"cfg2/base64 entries W={W}")


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_sixteen_bit_few_bins(cfg2_base64, dtype):
    import synth
    run_case(cfg2_base64, tfs(synth.SEED + 2, 4, n_cp=(4, 4)), 48, dtype=dtype, label=f"{dtype} W=48")


def test_set_field_refreshes_tile_statistics(cfg2_base64):
    """A data change through dvl_set_field: ordering kept, ranges and per-tile
    statistics refreshed, update equal to a volume built with the new data."""
    import synth
    D = dvl()
    vol = cfg2_base64
    dev = vol.to("cuda")
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, dev.fields)
    try:
        new = dev.fields[2] * 3.0 + 1.0
        V.set_field(2, new)
        fields = list(vol.fields)
        fields[2] = new.cpu()
        vol2 = synth.Volume(vol.x, vol.y, vol.z, vol.level, fields)
        A = tfs(77, 4)
        _, perm = V.export_order()
        p = perm.cpu().numpy().view(np.uint32)
        F = np.stack([f.numpy()[p] for f in fields])
        lo, hi = oracle.default_windows(F)
        for m in range(4):
            assert V.field_range(m) == (float(lo[m]), float(hi[m]))
            D.set_tf(V, m, A[m], float(lo[m]), float(hi[m]))
        W = 32
        bins = D.Bins(W, 4)
        V.update(bins)
        g = V.read_bins(bins)
        ob = oracle.update(vol2.level.numpy()[p], F, A, lo, hi, W, keep_cells=True)
        from parity import reconcile
        reconcile(g, ob, F, A, lo, hi, W)
    finally:
        V.close()


# ---------------------------------------------------------------- errors

def test_error_paths():
    D = dvl()
    vol = random_amr(21, 4, 2).to("cuda")
    # overlapping cells: a coarse cell and one of its own sub-cells
    x = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    lv = torch.tensor([1, 0], dtype=torch.uint8, device="cuda")
    f = torch.ones(2, device="cuda")
    with pytest.raises(D.DvlError) as e:
        D.build_order(x, x, x, lv, [f])
    assert e.value.status == 5
    with pytest.raises(D.DvlError) as e:
        D.build_order(-x - 1, x, x, torch.zeros_like(lv), [f])
    assert e.value.status == 6
    with pytest.raises(D.DvlError) as e:
        D.build_order(x, x, x, torch.full_like(lv, 21), [f])
    assert e.value.status == 6
    nanf = vol.fields[0].clone()
    nanf[3] = float("nan")
    with pytest.raises(D.DvlError) as e:
        D.build_order(vol.x, vol.y, vol.z, vol.level, [nanf])
    assert e.value.status == 6
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        b = D.Bins(16, vol.m)
        with pytest.raises(D.DvlError) as e:
            V.update(b)
        assert e.value.status == 4            # no TF yet
        for m in range(vol.m):
            V.set_tf(m, np.linspace(0, 1, 256))
        with pytest.raises(D.DvlError) as e:
            D.set_tf(V, 0, np.ones(4), 1.0, 1.0)
        assert e.value.status == 1
        with pytest.raises(D.DvlError) as e:
            D.set_tf(V, 9, np.ones(4), 0.0, 1.0)
        assert e.value.status == 1
        for bad in (dict(exponent=-1.0), dict(exponent=17.0), dict(min_importance=-0.1),
                    dict(vmax_mode=3), dict(level_scale=2), dict(scan_mode=7)):
            with pytest.raises(D.DvlError) as e:
                V.update(b, **bad)
            assert e.value.status == 1, bad
        V.update(b)
        g = V.read_bins(b)
        assert g["count"].sum() >= vol.n
    finally:
        V.close()
