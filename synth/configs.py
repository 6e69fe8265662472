"""The five synthetic workloads (and scaled-down variants used by tests).

1. ``grid64``      single-level regular 64^3 grid, 4 fp32 blob fields, W=1024.
2. ``amr3_12m``    3-level AMR, base 128^3, refine top 30 % then top 15 %
                   (about 12 M leaves), 4 fp32 astro fields, W=1920.
3. ``amr5_500m``   5-level AMR, base 256^3, refine top 40/30/20/10 %
                   (about 500 M leaves), 4 astro fields, W=1920.
4. ``batch32``     32 volumes of 1-20 M cells (log-uniform), 2-4 levels,
                   8 fp32 fields, W=2048.
5. ``serve4``      resident volumes of 10/50/150/300 M cells, 4 levels,
                   4 fp32 fields, W in {1024, 1920, 3840} per request.

All use p = 1 and minimum importance 0.025 (the paper's evaluation setting).
"""
from __future__ import annotations

import math

import torch

from .amr import (SEED, S_SIZES, Volume, base_side_for, make_amr, make_regular,
                  make_tfs)
from .noise import substream

P_DEFAULT = 1.0
FMIN_DEFAULT = 0.025

# refinement fractions per level, coarsest first
REFINE_CFG2 = (0.30, 0.15)
REFINE_CFG3 = (0.40, 0.30, 0.20, 0.10)


def config_seed(i: int) -> int:
    return SEED + i


def cfg1(device="cpu") -> Volume:
    return make_regular(64, 4, config_seed(1), device)


def cfg2(device="cpu", base: int = 128) -> Volume:
    return make_amr(base, REFINE_CFG2, 4, config_seed(2), device)


def cfg3(device="cpu", base: int = 256) -> Volume:
    # coarser noise octaves keep generation of ~500 M cells within seconds on a GPU
    return make_amr(base, REFINE_CFG3, 4, config_seed(3), device, octaves=5, field_octaves=3)


def cfg4_sizes(n_vol: int = 32, lo: float = 1e6, hi: float = 20e6, seed: int | None = None):
    """Log-uniform volume sizes and per-volume level counts (2-4 levels)."""
    s = substream(config_seed(4) if seed is None else seed, S_SIZES)
    g = torch.Generator().manual_seed(s)
    u = torch.rand(n_vol, generator=g, dtype=torch.float64)
    sizes = torch.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    levels = torch.randint(2, 5, (n_vol,), generator=g)
    return [float(v) for v in sizes], [int(v) for v in levels]


def cfg4_volume(k: int, device="cpu", n_vol: int = 32, scale: float = 1.0) -> Volume:
    """The k-th volume of the batch workload (8 fields)."""
    sizes, levels = cfg4_sizes(n_vol)
    fr = (0.3,) * (levels[k] - 1)
    b = base_side_for(sizes[k] * scale, fr)
    return make_amr(b, fr, 8, config_seed(4) * 1000 + k, device, octaves=4, field_octaves=2)


def cfg4(device="cpu", n_vol: int = 32, scale: float = 1.0):
    return [cfg4_volume(k, device, n_vol, scale) for k in range(n_vol)]


CFG5_SIZES = (10e6, 50e6, 150e6, 300e6)


def cfg5_volume(k: int, device="cpu", scale: float = 1.0, sizes=CFG5_SIZES) -> Volume:
    """The k-th resident volume of the serving workload (4 levels)."""
    fr = (0.3, 0.3, 0.3)
    b = base_side_for(sizes[k] * scale, fr)
    return make_amr(b, fr, 4, config_seed(5) * 1000 + k, device, octaves=4, field_octaves=2)


def cfg5(device="cpu", scale: float = 1.0, sizes=CFG5_SIZES):
    return [cfg5_volume(k, device, scale, sizes) for k in range(len(sizes))]


def tfs_for(i: int, n_fields: int, n_cp=(4, 4), n_tf: int = 256):
    return make_tfs(config_seed(i), n_fields, n_cp, n_tf)
