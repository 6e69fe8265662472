"""GPU parity of the views beyond the lines, through the C ABI, against the
oracle: brushing (bins -> sorted cell range -> Hilbert key range; the cell
mask a key range selects), zoom (an update over a sorted sub-range with its
own width), per-bin histograms (histogram heatmap) and the line raster
(RasterizeLines)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, random_amr, tfs
from parity import reconcile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


@pytest.fixture(scope="module")
def amr():
    """A 5-level synthetic AMR volume (~90 k cells), built once, with the
    oracle's ordering and the oracle inputs in sorted order."""
    import synth
    D = dvl()
    vol = synth.make_amr(16, (0.4, 0.3, 0.2), 4, 901, octaves=3, field_octaves=2)
    d = vol.to("cuda")
    V = D.build_order(d.x, d.y, d.z, d.level, d.fields)
    o = oracle.build_order(vol.x.numpy(), vol.y.numpy(), vol.z.numpy(), vol.level.numpy())
    F = np.stack([f.numpy()[o.perm] for f in vol.fields]).astype(np.float32)
    lev = vol.level.numpy()[o.perm]
    lo, hi = oracle.default_windows(F)
    A = tfs(901, vol.m)
    yield {"D": D, "vol": vol, "V": V, "o": o, "F": F, "lev": lev, "lo": lo, "hi": hi, "A": A}
    V.close()


def _update(st, W, **kw):
    D, V, A = st["D"], st["V"], st["A"]
    for m in range(V.m):
        D.set_tf(V, m, A[m], float(st["lo"][m]), float(st["hi"][m]))
    b = D.Bins(W, V.m)
    V.update(b, **kw)
    g = V.read_bins(b)
    ob = oracle.update(st["lev"], st["F"], A, st["lo"], st["hi"], W, keep_cells=True)
    rep = reconcile(g, ob, st["F"], A, st["lo"], st["hi"], W)
    return b, g, ob, rep


def test_select_bins_and_key_ranges(amr):
    st = amr
    V, o = st["V"], st["o"]
    b, g, ob, rep = _update(st, 480)
    keys_sorted = o.keys[o.perm]
    for b0, b1 in ((0, 0), (17, 40), (100, 479), (479, 479), (0, 479)):
        first, last, klo, khi = V.select_bins(b, b0, b1)
        assert (first, last) == (int(g["first"][b0]), int(g["last"][b1]))
        # the oracle's bins agree on these edges (checked by the reconciliation above when no edge moved)
        if rep.edges_moved == 0:
            assert (first, last) == (int(ob.first[b0]), int(ob.last[b1]))
        assert (klo, khi) == (int(keys_sorted[first]), int(keys_sorted[last]))
        # exactly the region's cells have keys in [klo, khi] (keys increase along the order)
        inside = (keys_sorted >= klo) & (keys_sorted <= khi)
        assert np.flatnonzero(inside).tolist() == list(range(first, last + 1))
    D = st["D"]
    with pytest.raises(D.DvlError) as e:
        V.select_bins(b, 5, 4)
    assert e.value.status == D.E_INVALID


def test_select_mask_matches_oracle_keys(amr):
    st = amr
    V, o = st["V"], st["o"]
    ks = np.sort(o.keys)
    rng = np.random.default_rng(5)
    cases = [[(int(ks[0]), int(ks[-1]))],                       # everything
             [(int(ks[10]), int(ks[10]))],                       # one cell
             [(int(ks[-1]) + 1, int(ks[-1]) + 5)]]               # nothing
    for _ in range(3):
        picks = np.sort(rng.choice(ks.size, 6, replace=False))
        cases.append([(int(ks[picks[i]]), int(ks[picks[i + 1]])) for i in (0, 2, 4)])
    cases.append([(int(ks[i]), int(ks[i + 3])) for i in range(0, 128 * 7, 7)])   # 128 ranges
    for ranges in cases:
        got = V.select_mask(ranges).cpu().numpy()
        want = np.zeros(o.keys.size, np.uint8)
        for lo, hi in ranges:
            want |= ((o.keys >= lo) & (o.keys <= hi)).astype(np.uint8)
        assert np.array_equal(got, want), f"{len(ranges)} ranges"


@pytest.mark.parametrize("W_zoom,exponent", [(1920, 1.0), (64, 2.0), (7, 0.5)])
def test_zoom_update_matches_oracle_on_the_subrange(amr, W_zoom, exponent):
    st = amr
    D, V, o, A = st["D"], st["V"], st["o"], st["A"]
    b, g, ob0, rep0 = _update(st, 96)
    first, last = int(ob0.first[20]), int(ob0.last[41])       # the region, as the oracle's bins give it
    if rep0.edges_moved == 0:
        assert V.select_bins(b, 20, 41)[:2] == (first, last)
    Z = V.zoom(first, last)
    try:
        n = last - first + 1
        assert Z.n == n and Z.m == V.m
        keys, perm = Z.export_order()
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), o.keys[o.perm][first:last + 1])
        assert np.array_equal(perm.cpu().numpy().view(np.uint32), np.arange(n, dtype=np.uint32))
        F = st["F"][:, first:last + 1]
        lev = st["lev"][first:last + 1]
        lo, hi = oracle.default_windows(F)
        for m in range(Z.m):
            assert Z.field_range(m) == (float(lo[m]), float(hi[m]))
            D.set_tf(Z, m, A[m], float(lo[m]), float(hi[m]))
        bz = D.Bins(W_zoom, Z.m)
        Z.update(bz, exponent=exponent)
        gz = Z.read_bins(bz)
        ob = oracle.update(lev, F, A, lo, hi, W_zoom, exponent, keep_cells=True)
        rep = reconcile(gz, ob, F, A, lo, hi, W_zoom)
        assert abs(gz["f_total"] - ob.f_total) <= 1e-5 * ob.f_total
        print(f"[zoom] cells {first}..{last} W={W_zoom}: edges moved {rep.edges_moved}", flush=True)
    finally:
        Z.close()


@pytest.mark.parametrize("W,H,dtype", [(480, 64, torch.float32), (4000, 16, torch.float32),
                                       (96, 256, torch.bfloat16), (1, 1000, torch.float16)])
def test_bin_histograms_match_oracle(amr, W, H, dtype):
    st = amr
    D, vol = st["D"], st["vol"]
    A = st["A"]
    if dtype == torch.float32:
        V, F, lo, hi = st["V"], st["F"], st["lo"], st["hi"]
        own = False
    else:
        d = vol.to("cuda")
        fields = [f.to(dtype) for f in d.fields]
        V = D.build_order(d.x, d.y, d.z, d.level, fields)
        F = np.stack([f.float().cpu().numpy()[st["o"].perm] for f in fields]).astype(np.float32)
        lo, hi = oracle.default_windows(F)
        own = True
    try:
        for m in range(V.m):
            D.set_tf(V, m, A[m], float(lo[m]), float(hi[m]))
        b = D.Bins(W, V.m)
        V.update(b)
        g = V.read_bins(b)
        ob = oracle.update(st["lev"], F, A, lo, hi, W, keep_cells=True)
        rep = reconcile(g, ob, F, A, lo, hi, W)
        for m in range(V.m):
            wlo, whi = float(lo[m]), float(hi[m]) * 1.01 + 0.01     # a window slightly past the data
            got = V.bin_histograms(b, m, H, wlo, whi).cpu().numpy().view(np.uint32)
            want = oracle.bin_histograms(F[m], ob.first, ob.last, H, wlo, whi)
            same = (g["first"] == ob.first) & (g["last"] == ob.last)
            assert rep.edges_moved > 0 or same.all()
            assert np.array_equal(got[same], want[same]), f"field {m}"
            assert np.array_equal(got.sum(axis=1), g["count"]), f"field {m}: counts"
    finally:
        if own:
            V.close()


def test_rasterize_matches_oracle(amr):
    st = amr
    D = st["D"]
    ob = oracle.update(st["lev"], st["F"], st["A"], st["lo"], st["hi"], 333)
    rng = np.random.default_rng(8)
    lines = [ob.y.astype(np.float32),
             rng.random((3, 333)).astype(np.float32),
             np.array([[0.0, 1.0, 0.5, 0.25, 0.999999, 1e-7] * 5], np.float32)]
    for Y in lines:
        for H in (1, 7, 100, 1024):
            for mode in (D.RASTER_POLYLINE, D.RASTER_BARS):
                got = D.rasterize(torch.from_numpy(Y).cuda(), H, mode).cpu().numpy()
                for l in range(Y.shape[0]):
                    want = oracle.rasterize(Y[l], H, mode)
                    assert np.array_equal(got[l], want), (Y.shape, H, mode, l)


def test_view_errors(amr):
    st = amr
    D, V = st["D"], st["V"]
    b = D.Bins(16, V.m)
    for call in (lambda: V.bin_histograms(b, 9, 16, 0.0, 1.0), lambda: V.bin_histograms(b, 0, 0, 0.0, 1.0),
                 lambda: V.bin_histograms(b, 0, 16, 1.0, 1.0), lambda: V.select_mask([(5, 1)]),
                 lambda: V.zoom(10, 5), lambda: V.zoom(0, V.n),
                 lambda: D.rasterize(torch.zeros(2, 8, device="cuda"), 0)):
        with pytest.raises(D.DvlError) as e:
            call()
        assert e.value.status == D.E_INVALID
