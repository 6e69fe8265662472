"""Precision study of the GPU path against the FP64 oracle on the full
5-level AMR workload (about 501 M cells, 4 fields, W = 1920).

For every variant (fp32 storage with the fp64, compensated-fp32 and naive-fp32
carry; bf16 and fp16 storage with the fp64 carry) one update is compared with
the oracle run on

  (i)  the data the GPU reads (the 16-bit values upcast): the parity bar,
       reconciled as in the parity tests (edges within 1e-6 of the normalised
       axis, min/max bitwise, mean within 1e-5 relative);
  (ii) the original fp32 data: error of every output, reported only.

    python tests/precision_study.py [--base 256] [--out precision_amr5_500m.json]

Run on a GPU; it holds the sorted fields on the host (about 9 GB at full size)
and runs the oracle once per distinct input (about 20-40 s each).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from parity import reconcile  # noqa: E402


def log(m):
    print(f"[precision] {m}", flush=True)


def output_errors(g: dict, o, F: np.ndarray, alpha: np.ndarray, lo, hi, W: int) -> dict:
    """Errors of the GPU bins g against oracle bins o (keep_cells) on data F."""
    n = F.shape[1]
    u = o.cell_e / o.f_total
    gf = g["first"].astype(np.int64)
    of = o.first.astype(np.int64)
    moved = np.nonzero(gf[1:] != of[1:])[0] + 1
    # how far (normalised axis) each moved edge's GPU boundary lies from the edge k / W
    dist = [abs(u[gf[k]] - k / W) for k in moved]
    cnt_g = g["last"].astype(np.int64) - gf + 1
    cnt_o = o.last.astype(np.int64) - of + 1
    # statistics with the oracle's membership vs the GPU's own output
    rel = np.abs(g["mean"].astype(np.float64) - o.mean) / np.maximum(np.abs(o.mean), 1e-30)
    out = {
        "edges_moved": int(moved.size),
        "max_edge_shift_cells": int(np.max(np.abs(gf[moved] - of[moved]))) if moved.size else 0,
        "max_moved_edge_distance_normalised": float(max(dist)) if dist else 0.0,
        "bins_count_differs": int(np.sum(cnt_g != cnt_o)),
        "mean_rel_max": float(rel.max()), "mean_rel_p99": float(np.quantile(rel, 0.99)),
        "vmin_max_abs": float(np.max(np.abs(g["vmin"].astype(np.float64) - o.vmin))),
        "vmax_max_abs": float(np.max(np.abs(g["vmax"].astype(np.float64) - o.vmax))),
        "y_differs": int(np.sum(g["y"] != o.y.astype(np.float32))),
        "f_total_rel": abs(g["f_total"] - o.f_total) / o.f_total,
        "vmax_used_rel": abs(g["vmax_used"] - o.vmax_used) / max(o.vmax_used, 1e-30),
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--base", type=int, default=256)
    ap.add_argument("--bins", type=int, default=1920)
    ap.add_argument("--out", default="precision_amr5_500m.json")
    args = ap.parse_args()
    import synth
    from paper_2306_11612_amd import dvl
    dvl.lib()
    W = args.bins
    t0 = time.time()
    vol = synth.cfg3(device="cuda", base=args.base)
    torch.cuda.synchronize()
    log(f"generated {vol.n} cells in {time.time() - t0:.1f} s")
    M = vol.m
    A = np.stack([t.numpy() for t in synth.make_tfs(synth.SEED + 3, M, (4, 4))])

    V = dvl.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    _, perm_t = V.export_order()
    perm = perm_t.cpu().numpy().view(np.uint32)
    lev = vol.level.cpu().numpy()[perm]
    F32 = np.stack([f.cpu().numpy()[perm] for f in vol.fields])
    V.close()
    lo32, hi32 = oracle.default_windows(F32)
    t0 = time.time()
    o32 = oracle.update(lev, F32, A, lo32, hi32, W, keep_cells=True)
    log(f"oracle fp32: {time.time() - t0:.1f} s")

    report = {"workload": "amr5_500m", "n_cells": int(vol.n), "n_fields": M, "n_bins": W, "variants": []}
    variants = [("f32", 0), ("f32", 1), ("f32", 2), ("bf16", 0), ("f16", 0)]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
    cur_dt, Vd, o_up, F_up, lo_up, hi_up = None, None, None, None, None, None
    for dt, scan in variants:
        if dt != cur_dt:
            if Vd is not None:
                Vd.close()
            fields = [f.to(tdt[dt]) for f in vol.fields]
            Vd = dvl.build_order(vol.x, vol.y, vol.z, vol.level, fields)
            if dt == "f32":
                F_up, o_up, lo_up, hi_up = F32, o32, lo32, hi32
            else:
                F_up = np.stack([f.float().cpu().numpy()[perm] for f in fields])
                lo_up, hi_up = oracle.default_windows(F_up)
                t0 = time.time()
                o_up = oracle.update(lev, F_up, A, lo_up, hi_up, W, keep_cells=True)
                log(f"oracle on upcast {dt}: {time.time() - t0:.1f} s")
            del fields
            torch.cuda.empty_cache()
            cur_dt = dt
        for m in range(M):
            dvl.set_tf(Vd, m, A[m], float(lo_up[m]), float(hi_up[m]))
        b = dvl.Bins(W, M)
        Vd.update(b, scan_mode=scan)
        g = Vd.read_bins(b)
        rec = {"storage": dt, "carry": ["fp64", "kahan_fp32", "naive_fp32"][scan]}
        try:
            rep = reconcile(g, o_up, F_up, A, lo_up, hi_up, W)
            rec["parity_on_data_read"] = {"pass": True, "edges_moved": rep.edges_moved,
                                          "ambiguous_cells": rep.ambiguous_cells,
                                          "max_mean_rel": rep.max_mean_rel, "heights_skipped": rep.y_skipped}
        except AssertionError as e:
            rec["parity_on_data_read"] = {"pass": False, "reason": str(e)[:300]}
        rec["vs_data_read"] = output_errors(g, o_up, F_up, A, lo_up, hi_up, W)
        if dt != "f32":
            # the 16-bit path against the oracle on the original fp32 values and windows
            for m in range(M):
                dvl.set_tf(Vd, m, A[m], float(lo32[m]), float(hi32[m]))
            Vd.update(b, scan_mode=scan)
            g32 = Vd.read_bins(b)
            rec["vs_fp32_original"] = output_errors(g32, o32, F32, A, lo32, hi32, W)
        log(json.dumps(rec))
        report["variants"].append(rec)
    Vd.close()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(report, fh, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
