"""The paper's three evaluations, on the synthetic stand-in workloads.

Evaluation section of the paper (its Figs. 4-6, whose images are not in the
text): (1) the time of the projection as the exponent P of Eq. 3 goes from 0
to 5 and the minimum importance from 0 to 0.25; (2) how evenly the cells
spread over the bins under the same sweeps (the paper reports that more
compression makes the projection slightly faster, 1-2 %); (3) the
approximate max(V_h) of Eqs. 5-6 against the exact maximum over 107 random
transfer-function configurations.

    python -m paper_2306_11612_amd.evaluate --workload amr3_12m [--out FILE.md]

Every number comes from the library through the C ABI (dvl_update,
dvl_kernel_times, dvl_read_bins).  Projection time = the tile classification
and rescan (phase 3) plus the per-bin statistics (phase 4); the importance
pass is listed beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

P_SWEEP = (0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0)
FMIN_SWEEP = (0.0, 0.025, 0.05, 0.1, 0.15, 0.2, 0.25)
N_TF_CONFIGS = 107


def count_stats(first, last) -> dict:
    """Cells per bin (last - first + 1): min, quartiles (lower order
    statistics), max, mean and the coefficient of variation."""
    c = np.sort((np.asarray(last, np.int64) - np.asarray(first, np.int64) + 1))
    q = lambda p: int(c[int(np.floor(p * (c.size - 1)))])
    return {"min": int(c[0]), "q1": q(0.25), "median": q(0.5), "q3": q(0.75), "max": int(c[-1]),
            "mean": float(c.mean()), "cv": float(c.std() / c.mean()) if c.mean() > 0 else 0.0}


def _set_tfs(V, alpha, windows):
    from . import dvl
    for m in range(V.m):
        lo, hi = windows[m]
        dvl.set_tf(V, m, alpha[m], lo, hi)


def windows_of(V):
    out = []
    for m in range(V.m):
        lo, hi = V.field_range(m)
        if not hi > lo:
            hi = float(np.nextafter(np.float32(lo), np.float32(np.inf)))
        out.append((lo, hi))
    return out


def timed_update(V, alpha, W: int, reps: int = 10, warmup: int = 3, **kw) -> dict:
    """Per-phase milliseconds (mean over `reps` updates) and the bins of the
    last update."""
    import torch
    from . import dvl
    win = windows_of(V)
    _set_tfs(V, alpha, win)
    bins = dvl.Bins(W, V.m)
    for _ in range(warmup):
        V.update(bins, **kw)
    torch.cuda.synchronize()
    V.set_timing(True)
    V.kernel_times()
    for _ in range(reps):
        V.update(bins, **kw)
    phases, n = V.kernel_times()
    V.set_timing(False)
    ms = {k: v / max(n, 1) for k, v in phases.items()}
    g = V.read_bins(bins)
    # the projection: classification (sharing its kernel with the carry scan),
    # rescan and bin statistics
    return {"ms": ms, "projection_ms": ms["carry"] + ms["bin"] + ms["bin_stats"], "bins": g}


def sweep(V, alpha, W: int, name: str, values, fixed: dict, reps: int = 10, log=None) -> list[dict]:
    rows = []
    for x in values:
        kw = dict(fixed)
        kw[name] = float(x)
        r = timed_update(V, alpha, W, reps=reps, **kw)
        row = {name: float(x), "projection_ms": r["projection_ms"], "importance_ms": r["ms"]["tile_sums"],
               "update_ms": sum(r["ms"].values()), "counts": count_stats(r["bins"]["first"], r["bins"]["last"])}
        rows.append(row)
        if log:
            log(f"{name}={x}: projection {row['projection_ms']:.4f} ms, counts {row['counts']}")
    return rows


def random_tf_configs(seed: int, M: int, n: int = N_TF_CONFIGS, n_tf: int = 256):
    """`n` seeded configurations of M piecewise-linear alpha TFs with 4-8
    control points each."""
    import synth
    return [np.stack([t.numpy() for t in synth.make_tfs(seed + 7 * k, M, (4, 8), n_tf)]) for k in range(n)]


def vmax_study(V, configs, W: int = 64, log=None) -> list[dict]:
    """max(V_h) used by the update under the exact mode and both
    approximations, per configuration."""
    from . import dvl
    win = windows_of(V)
    bins = dvl.Bins(W, V.m)
    rows = []
    for k, A in enumerate(configs):
        _set_tfs(V, A, win)
        row = {"config": k}
        for mode, key in ((dvl.VMAX_EXACT, "exact"), (dvl.VMAX_TF_RANGE, "tf_range"), (dvl.VMAX_TF_BOUND, "tf_bound")):
            V.update(bins, vmax_mode=mode)
            row[key] = V.read_bins(bins)["vmax_used"]
        rows.append(row)
    if log:
        r = np.array([[x["tf_range"] / x["exact"], x["tf_bound"] / x["exact"]] for x in rows if x["exact"] > 0])
        log(f"approx / exact over {len(rows)} configs: tf_range median {np.median(r[:, 0]):.3f}, "
            f"tf_bound median {np.median(r[:, 1]):.3f}")
    return rows


def summarise_vmax(rows) -> dict:
    ex = np.array([r["exact"] for r in rows])
    out = {"configs": len(rows)}
    for key in ("tf_range", "tf_bound"):
        a = np.array([r[key] for r in rows])
        ok = ex > 0
        ratio = a[ok] / ex[ok]
        out[key] = {"ratio_min": float(ratio.min()), "ratio_median": float(np.median(ratio)),
                    "ratio_max": float(ratio.max()), "below_exact": int(np.sum(a < ex)),
                    "mean_abs_diff": float(np.mean(np.abs(a - ex)))}
    return out


def markdown(res: dict) -> str:
    L = [f"# Evaluation on {res['workload']} ({res['n_cells']} cells, {res['n_fields']} fields, W = {res['n_bins']})",
         "", "Command:", "", f"    {res['command']}", "",
         "Projection = carry scan with tile classification (one kernel), rescan and per-bin statistics (ms per update, mean of "
         f"{res['reps']} updates, TF entry cache on); counts = cells per bin.", ""]
    for name, rows in (("exponent", res["exponent_sweep"]), ("min_importance", res["min_importance_sweep"])):
        L += [f"## Sweep of {name}", "",
              f"| {name} | projection ms | importance ms | update ms | min | q1 | median | q3 | max | cv |",
              "|---|---|---|---|---|---|---|---|---|---|"]
        for r in rows:
            c = r["counts"]
            L.append(f"| {r[name]:g} | {r['projection_ms']:.4f} | {r['importance_ms']:.4f} | {r['update_ms']:.4f} | "
                     f"{c['min']} | {c['q1']} | {c['median']} | {c['q3']} | {c['max']} | {c['cv']:.3f} |")
        L.append("")
    v = res["vmax"]
    L += [f"## Approximate vs exact max(V_h), {v['configs']} random TF configurations", "",
          "| approximation | min ratio | median ratio | max ratio | configs below exact | mean abs diff |",
          "|---|---|---|---|---|---|"]
    for key in ("tf_range", "tf_bound"):
        s = v[key]
        L.append(f"| {key} | {s['ratio_min']:.4f} | {s['ratio_median']:.4f} | {s['ratio_max']:.4f} | "
                 f"{s['below_exact']} | {s['mean_abs_diff']:.4f} |")
    L.append("")
    return "\n".join(L)


def main(argv=None):
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    from . import dvl
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="amr3_12m", choices=["amr3_12m", "amr5_500m"])
    ap.add_argument("--bins", type=int, default=1920)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--configs", type=int, default=N_TF_CONFIGS)
    ap.add_argument("--out", default=None, help="markdown summary (default: print only)")
    args = ap.parse_args(argv)

    def log(m):
        print(f"[evaluate] {m}", file=sys.stderr, flush=True)

    dvl.lib()
    t0 = time.perf_counter()
    vol = synth.cfg2(device="cuda") if args.workload == "amr3_12m" else synth.cfg3(device="cuda")
    seed = synth.SEED + (2 if args.workload == "amr3_12m" else 3)
    V = dvl.build_order(vol.x, vol.y, vol.z, vol.level, vol.fields)
    n, M = vol.n, vol.m
    del vol
    torch.cuda.empty_cache()
    log(f"{args.workload}: {n} cells resident in {time.perf_counter() - t0:.1f} s")
    try:
        alpha = np.stack([t.numpy() for t in synth.make_tfs(seed, M, (4, 4))])
        res = {"workload": args.workload, "n_cells": n, "n_fields": M, "n_bins": args.bins, "reps": args.reps,
               "command": "python -m paper_2306_11612_amd.evaluate " + " ".join(sys.argv[1:] if argv is None else argv)}
        res["exponent_sweep"] = sweep(V, alpha, args.bins, "exponent", P_SWEEP, {"min_importance": 0.025},
                                      args.reps, log)
        res["min_importance_sweep"] = sweep(V, alpha, args.bins, "min_importance", FMIN_SWEEP, {"exponent": 1.0},
                                            args.reps, log)
        rows = vmax_study(V, random_tf_configs(seed + 1000, M, args.configs), log=log)
        res["vmax"] = summarise_vmax(rows)
        res["vmax_rows"] = rows
    finally:
        V.close()
    print(json.dumps(res), flush=True)
    md = markdown(res)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(md)
    print(md, file=sys.stderr)


if __name__ == "__main__":
    main()
