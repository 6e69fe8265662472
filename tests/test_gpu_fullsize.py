"""Parity at the full size of the benchmark workload (5-level AMR, about
501 M cells, 4 fp32 fields, W = 1920), in the launch configuration bench.py
times: default layout, two TF sets alternated with unchanged windows, so the
timed updates read the cached TF entries.

The ordering is checked through properties that hold at any size (the
permutation is one, the exported keys are strictly increasing along it) and
through the oracle's keys of a sample of one million cells computed one by
one; the bins of one update are reconciled against the oracle's full update
(about 30-60 s of single-threaded C)."""
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_cases import dvl

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dvl()


def test_full_size_amr5_500m():
    import synth
    from parity import reconcile
    D = dvl()
    t0 = time.time()
    vol = synth.cfg3(device="cuda")
    torch.cuda.synchronize()
    n, M = vol.n, vol.m
    print(f"[full] generated {n} cells in {time.time() - t0:.1f} s", flush=True)
    V = D.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    try:
        keys, perm_t = V.export_order()
        torch.cuda.synchronize()
        # ordering: a permutation, keys strictly increasing along it
        counts = torch.bincount(perm_t.long(), minlength=n)
        assert int(counts.min()) == 1 and int(counts.max()) == 1
        ks = keys[perm_t.long()]
        assert bool((ks[1:] > ks[:-1]).all()), "keys not strictly increasing in sorted order"
        del counts, ks
        # sampled keys against the oracle, cell by cell
        x, y, z, lv = (t.cpu().numpy() for t in (vol.x, vol.y, vol.z, vol.level))
        bits = oracle.grid_bits(x, y, z, lv)
        assert bits == V.bits
        rng = np.random.default_rng(5)
        sample = rng.choice(n, 1_000_000, replace=False)
        ok = oracle.cell_keys(x[sample], y[sample], z[sample], lv[sample], bits)
        got = keys.cpu().numpy().view(np.uint64)[sample]
        assert np.array_equal(got, ok), f"{np.sum(got != ok)} sampled keys differ"
        del keys, x, y, z
        print(f"[full] ordering checked ({bits} bits per axis)", flush=True)

        # the bench's update loop: two TF sets, windows = data ranges
        A = [np.stack([t.numpy() for t in synth.make_tfs(synth.SEED + 3 + k, M, (4, 4))]) for k in range(2)]
        win = [V.field_range(m) for m in range(M)]
        b = D.Bins(1920, M)
        for k in range(3):
            for m in range(M):
                D.set_tf(V, m, A[k & 1][m], *win[m])
            V.update(b)
        g = V.read_bins(b)                      # the third update: TF set 0
        assert V.entry_cache_info() is not None, "the timed path reads cached entries"
        perm = perm_t.cpu().numpy().view(np.uint32)
        lev = lv[perm]
        F = np.stack([f.cpu().numpy()[perm] for f in vol.fields])
        lo = np.array([w[0] for w in win], np.float32)
        hi = np.array([w[1] for w in win], np.float32)
        t0 = time.time()
        ob = oracle.update(lev, F, A[0], lo, hi, 1920, keep_cells=True)
        print(f"[full] oracle update in {time.time() - t0:.1f} s", flush=True)
        rep = reconcile(g, ob, F, A[0], lo, hi, 1920)
        assert abs(g["f_total"] - ob.f_total) <= 1e-5 * ob.f_total
        print(f"[full] ok: edges moved {rep.edges_moved}, ambiguous cells {rep.ambiguous_cells}, "
              f"max mean rel {rep.max_mean_rel:.2e}", flush=True)
    finally:
        V.close()
