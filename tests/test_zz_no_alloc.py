"""The allocation-free update (dvl_update_noalloc) against dvl_update through
the C ABI: bitwise equal results on two calls in a row, the second on a
smaller volume (the shared scratch keeps the first call's contents), with and
without the TF entry cache, and reconciled against the oracle; no device
memory is taken from PyTorch's allocator or anywhere else."""
import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl, random_amr, tfs
from parity import reconcile

pytestmark = pytest.mark.gpu

KEYS = ("first", "last", "mean", "vmin", "vmax", "y", "f_total", "vmax_used")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def _oracle_of(V, vol, A, W):
    _, perm = V.export_order()
    p = perm.cpu().numpy().view(np.uint32)
    F = np.stack([f.numpy()[p] for f in vol.fields]).astype(np.float32)
    lo, hi = oracle.default_windows(F)
    return oracle.update(vol.level.numpy()[p], F, A, lo, hi, W, keep_cells=True), F, lo, hi


def test_noalloc_matches_update_bigger_then_smaller():
    D = dvl()
    big = random_amr(41, 24, 3, 0.4, n_fields=4)       # ~175 k cells, 43 tiles
    small = random_amr(42, 6, 2, 0.3, n_fields=4)      # ~1.1 k cells, one ragged tile
    assert big.n > 40 * small.n
    A = tfs(41, 4)
    cases = [(big, 1920), (small, 96)]
    vols = []
    try:
        for vol, W in cases:
            d = vol.to("cuda")
            V = D.build_order(d.x, d.y, d.z, d.level, d.fields)
            for m in range(4):
                V.set_tf(m, A[m])
            vols.append(V)
        for rnd in range(2):                      # second round: the entry cache of both volumes
            for (vol, W), V in zip(cases, vols):
                out = D.Bins(W, 4)
                torch.cuda.synchronize()
                used = torch.cuda.memory_allocated()
                D.update_noalloc(V, D.params(W), out)
                torch.cuda.synchronize()
                assert torch.cuda.memory_allocated() == used
                got = V.read_bins(out)
                ref_b = D.Bins(W, 4)
                V.update(ref_b)
                V.update(ref_b)                   # the second use of the windows builds the cache
                ref = V.read_bins(ref_b)
                for k in KEYS:
                    assert np.asarray(got[k]).tobytes() == np.asarray(ref[k]).tobytes(), (rnd, vol.n, k)
                if rnd == 0:
                    ob, F, lo, hi = _oracle_of(V, vol, A, W)
                    rep = reconcile(got, ob, F, A, lo, hi, W)
                    print(f"[noalloc] n={vol.n} W={W}: edges moved {rep.edges_moved}", flush=True)
        assert all(V.entry_cache_info() is not None for V in vols)
    finally:
        for V in vols:
            V.close()


def test_noalloc_limit_is_stated():
    D = dvl()
    assert D.lib().dvl_update_noalloc_max_bytes() == 64 << 20
