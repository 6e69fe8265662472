"""Shared driver of the GPU parity tests: build the volume through the C ABI,
run one update, run the oracle on the same inputs and reconcile."""
from __future__ import annotations

import itertools

import numpy as np
import torch

import oracle
from parity import reconcile, to_np


def dvl():
    from paper_2306_11612_amd import dvl as D
    D.lib()
    return D


def random_amr(seed: int, base: int = 4, levels: int = 3, frac: float = 0.4, n_fields: int = 3,
               shuffle: bool = True):
    """Small random aligned AMR volume (CPU tensors) with random fields."""
    import synth
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
    lev = np.concatenate(lev).astype(np.uint8)
    if shuffle:
        p = rng.permutation(c.shape[0])
        c, lev = c[p], lev[p]
    n = c.shape[0]
    fields = [torch.from_numpy((rng.lognormal(0, 1 + m, n)).astype(np.float32)) for m in range(n_fields)]
    return synth.Volume(torch.from_numpy(c[:, 0].astype(np.int32)), torch.from_numpy(c[:, 1].astype(np.int32)),
                        torch.from_numpy(c[:, 2].astype(np.int32)), torch.from_numpy(lev), fields,
                        [f"f{m}" for m in range(n_fields)], base, levels, [])


def subset(vol, n: int, seed: int = 0):
    """First n cells of a random permutation (non-overlapping cells stay so)."""
    import synth
    p = torch.from_numpy(np.random.default_rng(seed).permutation(vol.n)[:n])
    return synth.Volume(vol.x[p], vol.y[p], vol.z[p], vol.level[p], [f[p] for f in vol.fields],
                        vol.names, vol.base, vol.n_levels, [])


def tfs(seed: int, M: int, n_tf: int = 256, n_cp=(4, 8)):
    import synth
    return np.stack([t.numpy() for t in synth.make_tfs(seed, M, n_cp, n_tf)])


def check_order(V, vol):
    """Keys (original order) and permutation bit-exact against the oracle."""
    keys, perm = V.export_order()
    torch.cuda.synchronize()
    keys = keys.cpu().numpy().view(np.uint64)
    perm = perm.cpu().numpy().view(np.uint32)
    o = oracle.build_order(vol.x.numpy(), vol.y.numpy(), vol.z.numpy(), vol.level.numpy())
    assert V.bits == o.bits, (V.bits, o.bits)
    assert np.array_equal(keys, o.keys), f"{np.sum(keys != o.keys)} keys differ"
    assert np.array_equal(perm, o.perm), f"{np.sum(perm != o.perm)} permutation entries differ"
    return o


def run_case(vol, alpha, W: int, exponent: float = 1.0, fmin: float = 0.025, vmax_mode: int = 0,
             clamp_mode: int = 0, level_scale: int = 1, scan_mode: int = 0,
             dtype=torch.float32, windows=None, label: str = "", check_order_too: bool = True,
             edge_tol: float = 1e-6, entry_cache: int = 0):
    D = dvl()
    print(f"[case] {label} n={vol.n} M={vol.m} W={W} p={exponent} fmin={fmin} vmax={vmax_mode} "
          f"clamp={clamp_mode} lscale={level_scale} scan={scan_mode} dtype={dtype} cache={entry_cache}",
          flush=True)
    dev = vol.to("cuda")
    fields = [f.to(dtype) for f in dev.fields]
    V = D.build_order(dev.x, dev.y, dev.z, dev.level, fields, entry_cache=entry_cache)
    try:
        if check_order_too:
            o = check_order(V, vol)
            perm = o.perm
        else:
            _, perm_t = V.export_order()
            perm = perm_t.cpu().numpy().view(np.uint32)
        F = np.stack([to_np(f.cpu())[perm] for f in fields]).astype(np.float32)
        lev = vol.level.numpy()[perm]
        M = vol.m
        if windows is None:
            lo, hi = oracle.default_windows(F)
            for m in range(M):
                glo, ghi = V.field_range(m)
                assert (glo, ghi) == (float(lo[m]), float(hi[m])), (m, glo, ghi, lo[m], hi[m])
                if not hi[m] > lo[m]:
                    hi[m] = np.nextafter(lo[m], np.float32(np.inf))
        else:
            lo, hi = (np.asarray(w, np.float32) for w in windows)
        A = np.asarray(alpha, np.float32)
        for m in range(M):
            D.set_tf(V, m, A[m], float(lo[m]), float(hi[m]))
        bins = D.Bins(W, M)
        V.update(bins, exponent=exponent, min_importance=fmin, vmax_mode=vmax_mode, clamp_mode=clamp_mode,
                 level_scale=level_scale, scan_mode=scan_mode)
        g = V.read_bins(bins)
        ob = oracle.update(lev, F, A, lo, hi, W, exponent, fmin, vmax_mode, clamp_mode, level_scale,
                           keep_cells=True)
        rep = reconcile(g, ob, F, A, lo, hi, W, edge_tol=edge_tol)
        assert abs(g["f_total"] - ob.f_total) <= 1e-5 * ob.f_total, (g["f_total"], ob.f_total)
        assert abs(g["vmax_used"] - ob.vmax_used) <= 1e-6 * max(ob.vmax_used, 1e-30), (g["vmax_used"], ob.vmax_used)
        print(f"[ok] edges moved {rep.edges_moved}, ambiguous cells {rep.ambiguous_cells}, "
              f"max mean rel {rep.max_mean_rel:.2e}, heights skipped {rep.y_skipped}", flush=True)
        return g, ob, rep
    finally:
        V.close()
