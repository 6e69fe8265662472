"""Parity at the full size of the benchmark workload (5-level AMR, about
501 M cells, 4 fields, W = 1920), in the launch configuration bench.py times:
default layout, two TF sets alternated with unchanged windows, so the timed
updates read the cached TF entries.

Ordering: every one of the ~501 M keys is compared with the oracle's key of
that cell (computed in chunks on the host); the permutation is checked to be
one and to make the keys strictly increasing, which, the keys being
distinct, makes it the oracle's stable sort.  Updates: the cached-entry path
(bench.py's), the value path, the compensated fp32 carry and bf16 storage are
each reconciled against the oracle's full update (about 20-40 s of
single-threaded C each).  The tests share one generated volume (module
fixture); each stays well under two minutes."""
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

W = 1920
KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


def log(msg):
    print(f"[full] {msg}", flush=True)


@pytest.fixture(scope="module")
def full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import synth
    D = dvl()
    t0 = time.time()
    vol = synth.cfg3(device="cuda")
    torch.cuda.synchronize()
    log(f"generated {vol.n} cells in {time.time() - t0:.1f} s")
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    keys, perm_t = V.export_order()
    torch.cuda.synchronize()
    M = vol.m
    A = [np.stack([t.numpy() for t in synth.make_tfs(synth.SEED + 3 + k, M, (4, 4))]) for k in range(2)]
    win = [V.field_range(m) for m in range(M)]
    st = {"D": D, "vol": vol, "V": V, "keys": keys, "perm_t": perm_t, "A": A, "win": win,
          "perm": perm_t.cpu().numpy().view(np.uint32)}
    st["lev"] = vol.level.cpu().numpy()[st["perm"]]
    st["lo"] = np.array([w[0] for w in win], np.float32)
    st["hi"] = np.array([w[1] for w in win], np.float32)
    yield st
    V.close()


def _oracle_f32(full):
    """The oracle's update of TF set 0 on the fp32 data (computed once)."""
    if "ob" not in full:
        perm = full["perm"]
        F = np.stack([f.cpu().numpy()[perm] for f in full["vol"].fields])
        t0 = time.time()
        full["ob"] = oracle.update(full["lev"], F, full["A"][0], full["lo"], full["hi"], W, keep_cells=True)
        full["F"] = F
        log(f"oracle update in {time.time() - t0:.1f} s")
    return full["ob"], full["F"]


def _reconcile(full, g, ob, F, label):
    from parity import reconcile
    rep = reconcile(g, ob, F, full["A"][0], full["lo"], full["hi"], W)
    assert abs(g["f_total"] - ob.f_total) <= 1e-5 * ob.f_total, (g["f_total"], ob.f_total)
    log(f"{label}: edges moved {rep.edges_moved}, ambiguous cells {rep.ambiguous_cells}, "
        f"max mean rel {rep.max_mean_rel:.2e}")
    return rep


def test_full_ordering_every_key(full):
    vol, V = full["vol"], full["V"]
    n = vol.n
    perm_t, keys = full["perm_t"], full["keys"]
    counts = torch.bincount(perm_t.long(), minlength=n)
    assert int(counts.min()) == 1 and int(counts.max()) == 1, "not a permutation"
    del counts
    ks = keys[perm_t.long()]
    assert bool((ks[1:] > ks[:-1]).all()), "keys not strictly increasing in sorted order"
    del ks
    x, y, z, lv = (t.cpu().numpy() for t in (vol.x, vol.y, vol.z, vol.level))
    bits = oracle.grid_bits(x, y, z, lv)
    assert bits == V.bits
    got = keys.cpu().numpy().view(np.uint64)
    t0 = time.time()
    step = 50_000_000
    for a in range(0, n, step):
        b = min(n, a + step)
        ok = oracle.cell_keys(x[a:b], y[a:b], z[a:b], lv[a:b], bits)
        bad = np.flatnonzero(got[a:b] != ok)
        assert bad.size == 0, f"{bad.size} keys differ in cells [{a}, {b}), first at {a + bad[0]}"
    log(f"all {n} keys equal the oracle's ({bits} bits per axis) in {time.time() - t0:.1f} s")


def test_full_update_cached_entries(full):
    D, V, A, win = full["D"], full["V"], full["A"], full["win"]
    M = V.m
    b = D.Bins(W, M)
    for k in range(3):
        for m in range(M):
            D.set_tf(V, m, A[k & 1][m], *win[m])
        V.update(b)
    g = V.read_bins(b)                      # the third update: TF set 0
    assert V.entry_cache_info() is not None, "the timed path reads cached entries"
    full["g_entries"] = g
    ob, F = _oracle_f32(full)
    _reconcile(full, g, ob, F, "cached entries")


def test_full_update_values_and_kahan_carry(full):
    D, V, A, win = full["D"], full["V"], full["A"], full["win"]
    M = V.m
    ob, F = _oracle_f32(full)
    V.set_entry_cache(D.ENTRY_CACHE_NEVER)
    try:
        for m in range(M):
            D.set_tf(V, m, A[0][m], *win[m])
        b = D.Bins(W, M)
        V.update(b)
        g = V.read_bins(b)
        _reconcile(full, g, ob, F, "values")
        if "g_entries" in full:
            for k in KEYS:
                assert np.asarray(g[k]).tobytes() == np.asarray(full["g_entries"][k]).tobytes(), k
        V.update(b, scan_mode=D.SCAN_KAHAN_FP32)
        gk = V.read_bins(b)
        _reconcile(full, gk, ob, F, "values, compensated fp32 carry")
    finally:
        V.set_entry_cache(D.ENTRY_CACHE_AUTO)


def test_full_update_bf16_storage(full):
    D, vol, A = full["D"], full["vol"], full["A"]
    full.pop("F", None)
    full.pop("ob", None)
    fields = [f.to(torch.bfloat16) for f in vol.fields]
    V16 = D.build_order(vol.x, vol.y, vol.z, vol.level, fields)
    try:
        _, perm_t = V16.export_order()
        assert torch.equal(perm_t, full["perm_t"])
        perm = full["perm"]
        F = np.stack([f.float().cpu().numpy()[perm] for f in fields])
        del fields
        lo, hi = oracle.default_windows(F)
        M = vol.m
        for m in range(M):
            assert V16.field_range(m) == (float(lo[m]), float(hi[m]))
            D.set_tf(V16, m, A[0][m], float(lo[m]), float(hi[m]))
        b = D.Bins(W, M)
        V16.update(b)
        g = V16.read_bins(b)
        t0 = time.time()
        ob = oracle.update(full["lev"], F, A[0], lo, hi, W, keep_cells=True)
        log(f"oracle update (bf16 data) in {time.time() - t0:.1f} s")
        from parity import reconcile
        rep = reconcile(g, ob, F, A[0], lo, hi, W)
        assert abs(g["f_total"] - ob.f_total) <= 1e-5 * ob.f_total
        log(f"bf16: edges moved {rep.edges_moved}, max mean rel {rep.max_mean_rel:.2e}")
    finally:
        V16.close()
