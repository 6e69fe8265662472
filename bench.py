#!/usr/bin/env python3
"""DVL update throughput on one MI355X.

A step is one volume-line update of the resident volume after a transfer
function change (dvl_set_tf + dvl_update: TF lookup, variation, importance,
prefix sum, projection and bin reduction of every cell).  The one-time
Hilbert ordering is timed once and reported separately under "ordering".

Default workload: synthetic 5-level AMR, base 256^3, refinement of the top
40/30/20/10 % of cells by seeded fBm noise (about 500 M leaf cells), four
fp32 fields (log-normal density, temperature, pressure, velocity
magnitude), 4-control-point alpha TFs, W = 1920 bins, P = 1, minimum
importance 0.025.  Inputs are generated on the GPU and resident in HBM
before the timed region.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DVL update throughput (cells/s, ms/update) and achieved HBM GB/s; p99 latency served"
HBM_PEAK_GBPS = 8000.0


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name: str, base: int | None, device: str):
    import synth
    if name == "amr5_500m":
        return synth.cfg3(device=device, base=base or 256), synth.SEED + 3, \
            "5-level AMR, base {b}^3, refine top 40/30/20/10% by fBm".format(b=base or 256)
    if name == "amr3_12m":
        return synth.cfg2(device=device, base=base or 128), synth.SEED + 2, \
            "3-level AMR, base {b}^3, refine top 30/15% by fBm".format(b=base or 128)
    if name == "grid64":
        return synth.cfg1(device=device), synth.SEED + 1, "single-level 64^3 grid, blob fields"
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash() -> str:
    """sha256 over the device-code sources (the kernels and what they include)
    and the build script's flags; profiles record it next to their counters.
    Host-side launch code (api.hip) is not part of it: it does not change the
    bytes a kernel moves."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2306_11612_amd", "csrc")
    files = sorted(f for f in glob.glob(os.path.join(csrc, "*")) if os.path.basename(f) != "api.hip")
    files += [os.path.join(ROOT, "paper_2306_11612_amd", "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload: str, dtype: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if there is none or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{dtype}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_launch", {}).get("k_" + kernel)


def host_cpu() -> dict:
    """CPU model and logical CPU count of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(upd_inputs, alphas, n_bins: int, exponent: float, fmin: float, order_inputs=None):
    """The oracle (single-threaded C, fp64) timed on the GPU machine's host: one
    update over a sample of the workload's cells (`upd_inputs`: levels and
    fields of the first cells in generation order; the oracle's cost per cell
    does not depend on the order) and its ordering step (keys + sort) over the
    first cells of `order_inputs` (x, y, z, level)."""
    import numpy as np
    import oracle
    L, F = upd_inputs
    n = L.shape[0]
    lo, hi = oracle.default_windows(F)
    hi = np.where(hi > lo, hi, np.nextafter(lo, np.float32(np.inf))).astype(np.float32)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.update(L, F, alphas, lo, hi, n_bins, exponent, fmin)
    dt = time.perf_counter() - t0
    out = {"value": n / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n} cells of the same volume (generation order), one update "
                     f"(W={n_bins}), {dt:.2f} s single-threaded fp64",
           "threads": 1, **host_cpu()}
    if order_inputs is not None:
        xs, ys, zs, ls = (np.ascontiguousarray(a) for a in order_inputs)
        k = xs.shape[0]
        bits = oracle.grid_bits(xs, ys, zs, ls)
        t0 = time.perf_counter()
        keys = oracle.cell_keys(xs, ys, zs, ls, bits)
        t1 = time.perf_counter()
        oracle.sort_order(keys)
        t2 = time.perf_counter()
        out["ordering"] = {"cells": k, "keys_s": t1 - t0, "sort_s": t2 - t1,
                           "cells_per_s": k / (t2 - t0),
                           "sample": f"first {k} cells in original order: Hilbert keys + qsort of "
                                     f"(key, index), single-threaded"}
    return out


def bench_batch32(args, dt):
    """32 resident volumes of 1-20 M cells (8 fields, W = 2048), every volume
    updated after a TF change each step: as 32 sequential dvl_update calls, as
    one dvl_update_batch, and as one captured graph (dvl_graph_launch);
    `value` is the faster of the two batched forms."""
    import numpy as np
    import torch
    import synth
    from synth.configs import config_seed
    from paper_2306_11612_amd import dvl

    from paper_2306_11612_amd import tune
    W, n_vol = 2048, 32
    t0 = time.perf_counter()
    vols, layouts = [], []
    for k in range(n_vol):
        v = synth.cfg4_volume(k, "cuda", n_vol)
        fields = [f.to(dt) for f in v.fields]
        # the layout autotuner (cached per shape class: cell count and width
        # rounded to powers of two, field count, storage)
        lay = tune.best_layout(v.x, v.y, v.z, v.level, fields, W)
        layouts.append((lay["tile_steps"], lay["run_waves"]))
        vols.append(dvl.build_order(v.x, v.y, v.z, v.level, fields, tile_steps=lay["tile_steps"],
                                    run_waves=lay["run_waves"]))
        del v, fields
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    gen_s = time.perf_counter() - t0
    cells = sum(V.n for V in vols)
    M = vols[0].m
    log(f"{n_vol} volumes, {cells} cells, resident in {gen_s:.1f} s")
    tfs = [[np.stack([t.numpy() for t in synth.make_tfs(config_seed(4) * 1000 + k + 101 * s, M, (4, 4))])
            for s in range(2)] for k in range(n_vol)]
    kw = dict(exponent=args.exponent, min_importance=args.min_importance)

    gc.collect()
    gc.freeze()

    def timed(step, label):
        """Pipelined wall-clock ms per step (the host runs ahead), then the
        median per-step latency with the host waiting for each step (events
        on the current stream around one step).  Each form first runs the
        warm-up and one untimed pass of the timed length: a captured batch
        captures its graphs on its first launches, and the first pass after
        them ran slower than later ones."""
        for k in range(args.warmup + args.steps):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(k)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        lat = pct(event_times(step, max(args.steps, 10)))
        log(f"{label}: {ms:.3f} ms per step of {n_vol} updates, latency p50 {lat['p50']:.3f} ms")
        return ms, lat

    bins = [dvl.Bins(W, M) for _ in vols]

    def seq(k):
        for i, V in enumerate(vols):
            A = tfs[i][k & 1]
            for m in range(M):
                V.set_tf(m, A[m])
            V.update(bins[i], **kw)
    ms_seq, lat_seq = timed(seq, "sequential dvl_update")

    ex = dvl.Executor()
    reqs = [dvl.Request(V, tfs[i][0], bins[i], **kw) for i, V in enumerate(vols)]

    def batch(k):
        for i, r in enumerate(reqs):
            r.alpha = np.ascontiguousarray(tfs[i][k & 1])
        ex.update_batch(reqs)
    ms_batch, lat_batch = timed(batch, "dvl_update_batch")
    ex.set_timing(True)
    ex.kernel_times()
    for k in range(args.steps):
        batch(k)
    phases, nb = ex.kernel_times()
    ex.set_timing(False)
    per_launch = {k: v / max(nb, 1) for k, v in phases.items()}

    g = dvl.Graph(reqs)

    alt = [[tfs[i][s] for i in range(n_vol)] for s in range(2)]

    def graph(k):
        g.set_tf_all(alt[k & 1])
        g.launch()
    ms_graph, lat_graph = timed(graph, "captured graph")
    cached = all(V.entry_cache_info() is not None for V in vols)
    dom = max(("tile_sums", "bin", "bin_stats"), key=lambda k: per_launch[k])
    elem = 4 if args.dtype == "f32" else 2
    segs = [V.level_segments() for V in vols]
    lbpc = sum(nm * 64 + (ns // 4) * 4 for ns, nm in segs) / cells   # level codes + mixed segments
    bpc = (M + lbpc) if cached else (M * elem + lbpc)
    # algorithmic bytes per launch of each candidate dominant kernel:
    #  tile_sums  every cell's M entries (or values) + level stream, plus 4 B
    #             per cell written where the pass stores f for the rescan
    #  bin        the rescanned tiles (at most min(T, W) per volume); with
    #             W >= T / 4 the importance pass stored f, which the rescan
    #             reads (4 B per cell), else it reads what the first pass read
    #  bin_stats  per bin, the values of its two partial end steps
    kbytes = {"tile_sums": cells * bpc, "bin": 0.0, "bin_stats": 0.0}
    for V, (ts, _) in zip(vols, layouts):
        tile_cells = 256 * ts
        T = -(-V.n // tile_cells)
        stored_f = W * 4 >= T
        if stored_f:
            kbytes["tile_sums"] += V.n * 4          # the importance pass writes f of every cell
        kbytes["bin"] += min(T, W) * tile_cells * (4 if stored_f else bpc)
        kbytes["bin_stats"] += W * 2 * 256 * M * elem
    achieved = kbytes[dom] / (per_launch[dom] * 1e-3) / 1e9
    ms_best = min(ms_batch, ms_graph)
    out = {
        "metric": METRIC, "value": cells / (ms_best * 1e-3), "unit": "cells/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_best, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "batch32: 32 AMR volumes of 1-20 M cells (log-uniform), 2-4 levels, 8 fields, "
                               "one TF change per volume per step", "n_volumes": n_vol, "n_cells": cells,
                   "n_fields": M, "n_bins": W, "exponent": args.exponent, "min_importance": args.min_importance},
        "roofline": {"bound": "hbm", "kernel": dom + ("[entries]" if cached and dom == "tile_sums" else ""),
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "bytes_per_launch": kbytes[dom],
                     "bytes_per_cell": kbytes[dom] / cells, "avg_launch_ms": per_launch[dom],
                     "byte_model": {"tile_sums": "M cached entry bytes (or M field values) + level stream per cell, + 4 B of stored f per cell of the dense-bin volumes",
                                    "bin": "rescanned tiles: stored f (4 B per cell) or the first pass's bytes",
                                    "bin_stats": "per bin: the values of its two partial end steps"}[dom],
                     "kernel_bytes": kbytes},
        "dominant_kernel": dom,
        "tuned_layouts": {f"tile_steps={a},run_waves={b or 'default'}": layouts.count((a, b))
                          for a, b in sorted(set(layouts))},
        "entry_cache": cached,
        "sequential_ms_per_step": ms_seq, "batch_ms_per_step": ms_batch, "graph_ms_per_step": ms_graph,
        "step_latency_ms": {"sequential": lat_seq, "batch": lat_batch, "graph": lat_graph},
        "speedup_vs_sequential": ms_seq / ms_best,
        "kernel_ms_per_batch": per_launch, "generation_s": gen_s,
    }
    g.close()
    ex.close()
    for V in vols:
        V.close()
    print(json.dumps(out), flush=True)


def sort_passes(bits: int) -> int:
    """8-bit LSD passes over the 3 * bits significant key bits."""
    return max(1, (3 * bits + 7) // 8)


def ordering_bytes_per_cell(bits: int, M: int, elem: int) -> float:
    """Algorithmic bytes of the one-time ordering per cell: keys (read x, y, z,
    level: 13 B; write the 8-byte key: 21 B per cell, the 4-byte starting index
    written beside it not counted), the sort (one 8 B digit read per pass for the counts plus 24 B of
    key and index read and written per pass), the gather of level and fields
    (read index, level, fields; write level and fields)."""
    p = sort_passes(bits)
    return 21 + 8 * p + 24 * p + (4 + 1 + M * elem) + (1 + M * elem)


def event_times(step, reps: int, flush=None):
    """Per-step GPU time (ms) between events on the current stream; `flush`,
    when given, runs before every step outside the events (it overwrites the
    Infinity Cache)."""
    import torch
    out = []
    s = torch.cuda.current_stream()
    for k in range(reps):
        if flush is not None:
            flush(k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        step(k)
        e1.record(s)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def pct(xs) -> dict:
    import numpy as np
    a = np.asarray(xs, np.float64)
    return {"p10": float(np.percentile(a, 10)), "p50": float(np.percentile(a, 50)),
            "p90": float(np.percentile(a, 90)), "n": int(a.size)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="amr5_500m", choices=["amr5_500m", "amr3_12m", "grid64", "batch32"])
    ap.add_argument("--entry-cache", default="auto", choices=["auto", "never"],
                    help="TF entry cache policy of the timed updates (auto: the library default)")
    ap.add_argument("--base", type=int, default=None, help="override the base grid side")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--bins", type=int, default=1920)
    ap.add_argument("--exponent", type=float, default=1.0)
    ap.add_argument("--min-importance", type=float, default=0.025)
    ap.add_argument("--cpu-sample", type=int, default=300_000_000)
    ap.add_argument("--cpu-order-sample", type=int, default=20_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-data-change", action="store_true")
    ap.add_argument("--flush-mb", type=int, default=512,
                    help="bytes written before each event-timed step to overwrite the Infinity Cache (0: none)")
    ap.add_argument("--copy-only", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES bytes (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.copy_only:
        import torch
        n = args.copy_only // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the update shards by "
              "contiguous Hilbert ranges, but no multi-GPU path is built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2306_11612_amd import dvl

    dvl.lib()   # raises if the HIP library is missing: there is no fallback
    torch.cuda.set_device(0)
    dt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]

    import synth.amr
    synth.amr.PROGRESS = log
    if args.workload == "batch32":
        return bench_batch32(args, dt)
    t0 = time.perf_counter()
    vol, seed, desc = make_workload(args.workload, args.base, "cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    n, M = vol.n, vol.m
    log(f"generated {n} cells, levels {vol.level_counts}, in {gen_s:.1f} s")

    fields = [f.to(dt) for f in vol.fields]
    del vol.fields
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V = dvl.build_order(vol.x, vol.y, vol.z, vol.level, fields)
    torch.cuda.synchronize()
    order_s = time.perf_counter() - t0
    log(f"ordering (Hilbert keys + radix sort + gather): {order_s * 1e3:.1f} ms")
    order_inputs = upd_inputs = None
    if not args.no_cpu_baseline:
        k = min(args.cpu_order_sample, n)
        order_inputs = tuple(t[:k].cpu().numpy() for t in (vol.x, vol.y, vol.z, vol.level))
        k = min(args.cpu_sample, n)
        upd_inputs = (vol.level[:k].cpu().numpy(), np.stack([f[:k].float().cpu().numpy() for f in fields]))
    del vol
    torch.cuda.empty_cache()

    # two TF sets, alternated every step: each update follows a TF change
    tf_sets = [np.stack([t.numpy() for t in synth.make_tfs(seed + k, M, (4, 4))]) for k in range(2)]
    bins = dvl.Bins(args.bins, M)
    kw = dict(exponent=args.exponent, min_importance=args.min_importance)

    def set_tfs(k):
        A = tf_sets[k & 1]
        for m in range(M):
            lo, hi = V.field_range(m)
            if not hi > lo:
                hi = float(np.nextafter(np.float32(lo), np.float32(np.inf)))
            dvl.set_tf(V, m, A[m], lo, hi)

    def step(k):
        set_tfs(k)
        V.update(bins, **kw)

    flush_buf = torch.empty(max(args.flush_mb, 1) << 18, dtype=torch.float32, device="cuda")

    def flush(k):
        flush_buf.fill_(float(k))

    # the interpreter's objects so far (torch, the workload) move to the
    # permanent generation: a full collection during a timed region would
    # otherwise walk them all (a host pause of tens of milliseconds)
    gc.collect()
    gc.freeze()

    def measure(policy):
        V.set_entry_cache(policy)
        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        # timed region: HIP events around the importance pass (the dominant
        # kernel) of every fourth update (each recorded event drains the
        # queue for a few microseconds, which the other updates are spared)
        V.kernel_times()   # reset
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            V.set_timing(2 if k % 4 == 0 else 0)
            step(k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        k1_phases, n_upd = V.kernel_times()
        # the other kernels, with events around each, over as many untimed steps
        V.set_timing(1)
        for k in range(args.steps):
            step(k)
        phases, n_all = V.kernel_times()
        V.set_timing(False)
        phases = {k: v / max(n_all, 1) * max(n_upd, 1) for k, v in phases.items()}
        phases["tile_sums"] = k1_phases["tile_sums"]
        ms = wall * 1e3 / args.steps
        cached = V.entry_cache_info() is not None
        log(f"entry cache {'on' if cached else 'off'}: {args.steps} steps in {wall:.3f} s: {ms:.3f} ms/update; "
            f"kernels {phases}")
        per_step = {"warm": pct(event_times(step, args.steps))}
        if args.flush_mb:
            per_step["flushed"] = pct(event_times(step, args.steps, flush))
        return ms, {k: v / max(n_upd, 1) for k, v in phases.items()}, cached, per_step

    # The value path first (every update reads the fields), then the library
    # default: from the second update with unchanged windows on, the importance
    # pass reads the cached TF entries (one byte per cell and field).
    elem = 4 if args.dtype == "f32" else 2
    ms_values, per_launch_values, _, steps_values = measure(dvl.ENTRY_CACHE_NEVER)
    if args.entry_cache == "never":
        ms_per_step, per_launch, cached, steps_default = ms_values, per_launch_values, False, steps_values
    else:
        ms_per_step, per_launch, cached, steps_default = measure(dvl.ENTRY_CACHE_AUTO)

    # Byte models.  The importance pass streams every cell's M field values
    # (or M cached entries) once, plus one 32-bit level code per 256 cells and
    # the level bytes of the 64-cell segments whose levels differ.  The
    # projection re-reads the tiles that contain a bin edge (at most
    # min(tiles, W) of them; cached entries or values, as the first pass) and,
    # per bin, the values of the partial 256-cell steps at its two ends.
    n_seg, n_mixed = V.level_segments()
    level_bytes = n_mixed * 64 + (n_seg // 4) * 4
    lam = level_bytes / n
    value_bpc = M * elem + lam
    entry_bpc = M + lam
    k1_bpc = entry_bpc if cached else value_bpc
    alg_bytes = n * k1_bpc
    dom = max(("tile_sums", "bin"), key=lambda k: per_launch[k])
    achieved = alg_bytes / (per_launch[dom] * 1e-3) / 1e9
    n_tiles = (n + 4095) // 4096

    def update_bytes_of(bpc):
        return n * bpc + min(n_tiles, args.bins) * 4096 * bpc + args.bins * 2 * 256 * M * elem

    update_bytes = update_bytes_of(k1_bpc)
    update_gbps = update_bytes / (ms_per_step * 1e-3) / 1e9
    values_update_bytes = update_bytes_of(value_bpc)
    values_gbps = n * value_bpc / (per_launch_values["tile_sums"] * 1e-3) / 1e9
    plain_bpc = 2 * (M * elem + 1)
    ord_bpc = ordering_bytes_per_cell(V.bits, M, elem)
    model = ("design, TF change with unchanged windows: importance pass over cached TF entries "
             "(M + level bytes per cell), rescan of the tiles holding a bin edge, bin end steps; per-tile "
             "and per-step field statistics and the entry cache are built at ordering / data-change time"
             if cached else
             "design, value path: importance pass over the field values (M*s + level bytes per cell), "
             "rescan of the tiles holding a bin edge, bin end steps")

    out = {
        "metric": METRIC,
        "value": n / (ms_per_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n_cells": n, "n_fields": M,
                   "field_storage": args.dtype, "n_bins": args.bins, "exponent": args.exponent,
                   "min_importance": args.min_importance, "tf_control_points": 4,
                   "step": "TF change (dvl_set_tf x M with the windows kept) + dvl_update",
                   "layout": "library default: 4096-cell tiles (16 steps of 256 cells), default runs per wave"},
        "roofline": {"bound": "hbm", "kernel": dom + ("[entries]" if cached and dom == "tile_sums" else ""),
                     "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": profiled_traffic(args.workload, args.dtype, dom + ("_entries" if cached else "")),
                     "bytes_per_launch": alg_bytes, "bytes_per_cell": k1_bpc,
                     "byte_model": ("importance pass: M cached entry bytes + level stream per cell" if cached
                                    else "importance pass: M field values + level stream per cell"),
                     "avg_launch_ms": per_launch[dom]},
        "whole_update": {"bytes": update_bytes, "bytes_per_cell": update_bytes / n, "byte_model": model,
                         "gbps": update_gbps, "frac": update_gbps / HBM_PEAK_GBPS, "target_frac": 0.6,
                         "meets_target": update_gbps / HBM_PEAK_GBPS >= 0.6,
                         "plain_two_pass_bytes_per_cell": plain_bpc,
                         "plain_two_pass_equivalent_gbps": n * plain_bpc / (ms_per_step * 1e-3) / 1e9},
        "per_step_ms": steps_default,
        "entry_cache": cached,
        "level_segments": {"segments_of_64_cells": n_seg, "mixed": n_mixed, "level_bytes_per_cell": lam},
        "no_entry_cache": {"ms_per_step": ms_values, "value": n / (ms_values * 1e-3),
                           "tile_sums_ms": per_launch_values["tile_sums"], "tile_sums_gbps": values_gbps,
                           "tile_sums_frac": values_gbps / HBM_PEAK_GBPS, "bytes_per_cell": value_bpc,
                           "whole_update_gbps": values_update_bytes / (ms_values * 1e-3) / 1e9,
                           "whole_update_frac": values_update_bytes / (ms_values * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                           "traffic": profiled_traffic(args.workload, args.dtype, "tile_sums"),
                           "per_step_ms": steps_values,
                           "kernel_ms_per_update": per_launch_values},
        "kernel_ms_per_update": per_launch,
        "ordering": {"ms": order_s * 1e3, "cells_per_s": n / order_s, "bits_per_axis": V.bits,
                     "sort_passes": sort_passes(V.bits), "bytes_per_cell": ord_bpc,
                     "gbps": n * ord_bpc / order_s / 1e9, "frac": n * ord_bpc / order_s / 1e9 / HBM_PEAK_GBPS},
        "generation_s": gen_s,
        "paper_context": "RTX A6000, 35.8 M-cell Molecular Cloud, 4 fields: ~58.4 ms/update "
                         "(Table 1 sum excluding line drawing), ~0.61 G cells/s; other data and hardware",
    }

    if not args.no_data_change:
        # A data change: new values for every field (two resident copies in
        # the original cell order, alternated), then the update.  The windows
        # follow the new data ranges, so no entry cache is built.
        alt = [(f.float() * (1.0 + 0.1 * torch.sin(fields[(m + 1) % M].float()))).to(dt)
               for m, f in enumerate(fields)]
        copies = (alt, fields)
        V.set_entry_cache(dvl.ENTRY_CACHE_AUTO)

        def data_step(k):
            for m in range(M):
                V.set_field(m, copies[k & 1][m])
            step(k)

        for k in range(args.warmup):
            data_step(k)
        torch.cuda.synchronize()
        t_set = 0.0
        t0 = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            for m in range(M):
                V.set_field(m, copies[k & 1][m])
            t_set += time.perf_counter() - ts
            step(k)
        torch.cuda.synchronize()
        ms_dc = (time.perf_counter() - t0) * 1e3 / args.steps
        # per field: data range of the new values (s B/cell), gather (4 B index,
        # s B random read, s B write), per-tile/step statistics (s B/cell read)
        set_bpc = M * (4 + 4 * elem)
        dc_bytes = n * set_bpc + values_update_bytes
        out["data_change"] = {
            "ms_per_step": ms_dc, "value": n / (ms_dc * 1e-3), "set_field_ms_per_step": t_set * 1e3 / args.steps,
            "entry_cache": V.entry_cache_info() is not None,
            "bytes_per_cell": dc_bytes / n,
            "byte_model": "dvl_set_field x M (range of the new values, gather into sorted order, per-tile and "
                          "per-step statistics) + value-path update",
            "gbps": dc_bytes / (ms_dc * 1e-3) / 1e9, "frac": dc_bytes / (ms_dc * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "step": "dvl_set_field for every field from one of two resident copies (original order), "
                    "dvl_set_tf x M with the new data ranges, dvl_update"}
        log(f"data change: {ms_dc:.3f} ms per step (set_field {t_set * 1e3 / args.steps:.3f} ms)")
        del alt, copies
    del fields
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log(f"oracle CPU baseline on up to {args.cpu_sample} cells ...")
        out["cpu_baseline"] = cpu_baseline(upd_inputs, tf_sets[0], args.bins, args.exponent,
                                           args.min_importance, order_inputs)
        del upd_inputs, order_inputs
        log(f"oracle: {out['cpu_baseline']['value']:.3e} cells/s")
    V.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
