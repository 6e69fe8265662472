"""Autotuning of a volume's update layout (tile size and importance-pass run
count, ``dvl_build_options``) by measurement on the device.

The best layout depends on the cell count, the field count and storage type
and the plot width (how many tiles hold a bin edge and are read again), so
results are cached per shape class in a JSON file (``DVL_TUNE_CACHE``, default
``~/.cache/dvl_tune.json``):

    from paper_2306_11612_amd import tune
    V = tune.build_tuned(x, y, z, level, fields, n_bins=1920)

Every candidate gives results within the parity tolerance of the oracle; they
differ only in the fp64 summation order of the prefix and in speed.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import dvl

# (tile_steps, run waves per compute unit; 0 = the library default of 32)
CANDIDATES = [(16, 0), (8, 0), (32, 0), (16, 16), (32, 16), (8, 16), (16, 48)]


def cache_path() -> str:
    return os.environ.get("DVL_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dvl_tune.json"))


def shape_key(n_cells: int, n_fields: int, dtype: torch.dtype, n_bins: int) -> str:
    """Shape class: cell count and width rounded to powers of two."""
    return (f"n2^{int(round(math.log2(max(n_cells, 1))))}_m{n_fields}_{str(dtype).split('.')[-1]}"
            f"_w2^{int(round(math.log2(max(n_bins, 1))))}")


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(rec: dict):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _n_cu() -> int:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count


def time_layout(x, y, z, level, fields, n_bins: int, tile_steps: int, run_waves: int, steps: int = 10,
                alphas=None) -> float:
    """Mean ms per update (TF change + update) of one layout."""
    V = dvl.build_order(x, y, z, level, fields, tile_steps=tile_steps, run_waves=run_waves)
    try:
        M = V.m
        if alphas is None:
            import synth
            alphas = [np.stack([t.numpy() for t in synth.make_tfs(synth.SEED + 11 + k, M, (4, 4))])
                      for k in range(2)]
        win = [V.field_range(m) for m in range(M)]
        bins = dvl.Bins(n_bins, M)

        def step(k):
            for m in range(M):
                lo, hi = win[m]
                if not hi > lo:
                    hi = float(np.nextafter(np.float32(lo), np.float32(np.inf)))
                dvl.set_tf(V, m, alphas[k & 1][m], lo, hi)
            V.update(bins)

        for k in range(3):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(k)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3
    finally:
        V.close()


def tune(x, y, z, level, fields, n_bins: int, candidates=CANDIDATES, steps: int = 10, log=None) -> dict:
    """Measure every candidate layout; returns {"tile_steps", "run_waves", "ms", "all"}."""
    n_cu = _n_cu()
    results = []
    for ts, wpc in candidates:
        rw = wpc * n_cu if wpc else 0
        ms = time_layout(x, y, z, level, fields, n_bins, ts, rw, steps)
        results.append({"tile_steps": ts, "run_waves": rw, "ms": ms})
        if log:
            log(f"tile_steps={ts} run_waves={rw or 'default'}: {ms:.3f} ms/update")
        torch.cuda.empty_cache()
    best = min(results, key=lambda r: r["ms"])
    return {"tile_steps": best["tile_steps"], "run_waves": best["run_waves"], "ms": best["ms"], "all": results}


def best_layout(x, y, z, level, fields, n_bins: int, retune: bool = False, log=None) -> dict:
    """The cached layout of this shape class, tuning (and caching) it first if needed."""
    key = shape_key(x.numel(), len(fields), fields[0].dtype, n_bins)
    rec = _load()
    if key in rec and not retune:
        return rec[key]
    res = tune(x, y, z, level, fields, n_bins, log=log)
    rec = _load()
    rec[key] = {"tile_steps": res["tile_steps"], "run_waves": res["run_waves"], "ms": res["ms"]}
    _store(rec)
    return rec[key]


def build_tuned(x, y, z, level, fields, n_bins: int, stream=None, log=None, **kw) -> "dvl.Volume":
    """dvl.build_order with the tuned layout of this shape class."""
    lay = best_layout(x, y, z, level, fields, n_bins, log=log)
    return dvl.build_order(x, y, z, level, fields, stream=stream, tile_steps=lay["tile_steps"],
                           run_waves=lay["run_waves"], **kw)
