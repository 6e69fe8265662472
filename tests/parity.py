"""Parity helpers: run the GPU library and the CPU oracle on the same seeded
inputs and reconcile their bins.

Reading of "within 1e-6 of a bin edge" (the paper gives no precision): the
distance is measured on the normalised axis u = E / F_tot, i.e. 1e-6 * W
pixels.  A bin's first/last cell may differ from the oracle's only where
every cell boundary between the two candidates lies within that distance of
the bin edge.  With the GPU's membership, min/max must be bitwise equal, the
mean within a relative 1e-5 (floor 1e-3 of the field's largest magnitude),
and the height equal unless the mean sits within 1e-5 (relative) of a TF
entry edge.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EDGE_TOL = 1e-6
MEAN_RTOL = 1e-5


@dataclass
class Report:
    edges_moved: int = 0
    ambiguous_cells: int = 0
    max_mean_rel: float = 0.0
    y_skipped: int = 0
    notes: list = field(default_factory=list)


def to_np(t):
    import torch
    if t.dtype == torch.bfloat16 or t.dtype == torch.float16:
        return t.float().cpu().numpy()
    return t.cpu().numpy()


def oracle_inputs(vol, perm):
    """Sorted level and fp32 (upcast) fields for the oracle."""
    lev = to_np(vol.level)[perm]
    F = np.stack([to_np(f)[perm] for f in vol.fields]).astype(np.float32)
    return lev, F


def reconcile(g: dict, o, F: np.ndarray, alpha: np.ndarray, lo, hi, W: int,
              edge_tol: float = EDGE_TOL, mean_rtol: float = MEAN_RTOL) -> Report:
    """Compare GPU bins ``g`` (dict from read_bins) with oracle bins ``o``
    (oracle.Bins with cell_e).  Raises AssertionError on a mismatch."""
    import oracle
    rep = Report()
    n = F.shape[1]
    M = F.shape[0]
    u = o.cell_e / o.f_total                      # boundaries, length n + 1
    gf, gl = g["first"].astype(np.int64), g["last"].astype(np.int64)
    of, ol = o.first.astype(np.int64), o.last.astype(np.int64)
    assert gf[0] == 0, f"first[0] = {gf[0]}"
    assert gl[W - 1] == n - 1, f"last[W-1] = {gl[W - 1]} != {n - 1}"
    assert np.all(gf <= gl), "a bin with first > last"
    d = gf[1:] - gl[:-1]
    assert np.all((d == 0) | (d == 1)), "bins are not a chain of contiguous cell ranges"
    amb = set()

    def check(k_edge, a, b, what):
        lo_i, hi_i = min(a, b), max(a, b)
        js = np.arange(lo_i + 1, hi_i + 1)
        dist = np.abs(u[js] - k_edge / W)
        if np.any(dist > edge_tol):
            bad = js[dist > edge_tol][0]
            raise AssertionError(f"{what} at edge {k_edge}: gpu {a} vs oracle {b}; boundary {bad} "
                                 f"is {dist.max():.3e} from the edge (tolerance {edge_tol})")
        amb.update(range(lo_i, hi_i + 1))

    for k in range(1, W):
        if gf[k] != of[k]:
            check(k, gf[k], of[k], "first")
            rep.edges_moved += 1
        if gl[k - 1] != ol[k - 1]:
            check(k, gl[k - 1], ol[k - 1], "last")
            rep.edges_moved += 1
    rep.ambiguous_cells = len(amb)

    # statistics over the GPU's membership
    cs = np.concatenate([np.zeros((M, 1)), np.cumsum(F.astype(np.float64), axis=1)], axis=1)
    cnt = (gl - gf + 1).astype(np.float64)
    ref_mean = (cs[:, gl + 1] - cs[:, gf]) / cnt
    starts = gf
    mn = np.minimum.reduceat(F, starts, axis=1)
    mx = np.maximum.reduceat(F, starts, axis=1)
    straddle = np.zeros(W, bool)
    straddle[:-1] = gl[:-1] == gf[1:]
    if straddle.any():
        idx = gl[:-1][straddle[:-1]]
        mn[:, :-1][:, straddle[:-1]] = np.minimum(mn[:, :-1][:, straddle[:-1]], F[:, idx])
        mx[:, :-1][:, straddle[:-1]] = np.maximum(mx[:, :-1][:, straddle[:-1]], F[:, idx])
    assert np.array_equal(g["vmin"], mn), f"min differs in {np.sum(g['vmin'] != mn)} bins"
    assert np.array_equal(g["vmax"], mx), f"max differs in {np.sum(g['vmax'] != mx)} bins"
    scale = np.maximum(np.abs(ref_mean), 1e-3 * np.abs(F).max(axis=1, keepdims=True))
    rel = np.abs(g["mean"].astype(np.float64) - ref_mean) / scale
    rep.max_mean_rel = float(rel.max())
    assert rep.max_mean_rel <= mean_rtol, f"mean relative error {rep.max_mean_rel:.3e} > {mean_rtol}"
    # heights: same TF entry unless the mean sits on an entry edge
    for m in range(M):
        s, b = oracle.quantiser(alpha.shape[1], float(lo[m]), float(hi[m]))
        n_tf = alpha.shape[1]
        span = float(hi[m]) - float(lo[m])
        t = (ref_mean[m] - float(lo[m])) * n_tf / span
        frac = np.abs(t - np.round(t))
        near = frac <= 2.0 * mean_rtol * scale[m] * n_tf / span + 1e-6
        ent = np.array([oracle.tf_index(float(x), s, b, n_tf) for x in ref_mean[m].astype(np.float32)])
        expect_y = alpha[m][ent]
        bad = (g["y"][m] != expect_y) & ~near
        rep.y_skipped += int(near.sum())
        assert not bad.any(), f"field {m}: height differs in {bad.sum()} bins"
    return rep


def compare_oracle_bins(g: dict, o, W: int):
    """Strict comparison used where the two sides must agree exactly
    (closed-form cases): membership bit-exact."""
    assert np.array_equal(g["first"], o.first), "first differs"
    assert np.array_equal(g["last"], o.last), "last differs"
