"""Seeded synthetic AMR volumes shaped like the paper's astrophysics inputs.

The paper evaluates on a 4-level FLASH molecular-cloud AMR data set with four
correlated fields (density, temperature, pressure, velocity magnitude; see its
Evaluation section).  That data is not available, so these generators build
stand-ins with the same structure: leaf cells snapped to a logical grid (lower
corner + level, finest level 0, width 2^L; the logical-grid representation of
the Background section), refinement driven by thresholds of a seeded fBm noise
field, and log-normal density with correlated temperature/pressure.

Output cell order is generation order (coarsest level first); the method's
ordering step re-sorts it, and the result does not depend on it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field

import torch

from .noise import blobs, fbm, hash3, substream, uniform_from_hash, zscore

SEED = 230611612

# sub-stream identifiers
S_REFINE, S_FIELDS, S_TF, S_REQ, S_SIZES = 1, 2, 3, 4, 5

# optional progress callback (long generations report each stage)
PROGRESS = None


def _progress(msg: str):
    if PROGRESS is not None:
        PROGRESS(msg)


@dataclass
class Volume:
    """Leaf cells of one AMR volume in original (generation) order."""
    x: torch.Tensor          # int32 [n], lower corner on the logical grid
    y: torch.Tensor
    z: torch.Tensor
    level: torch.Tensor      # uint8 [n], 0 = finest, width 2^level
    fields: list             # M float32 tensors [n]
    names: list = dc_field(default_factory=list)
    base: int = 0            # base grid side (cells at the coarsest level)
    n_levels: int = 1
    level_counts: list = dc_field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def m(self) -> int:
        return len(self.fields)

    def to(self, device) -> "Volume":
        return Volume(self.x.to(device), self.y.to(device), self.z.to(device),
                      self.level.to(device), [f.to(device) for f in self.fields],
                      list(self.names), self.base, self.n_levels, list(self.level_counts))


def _grid_corners(side: int, width: int, device) -> torch.Tensor:
    """Lower corners [side^3, 3] (int64) of a regular grid of cells of
    ``width`` logical units, x fastest."""
    r = torch.arange(side, dtype=torch.int64, device=device) * width
    zz, yy, xx = torch.meshgrid(r, r, r, indexing="ij")
    return torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], dim=1)


def _centres(corners: torch.Tensor, width: int, extent: int) -> torch.Tensor:
    """Cell centres in [0,1)^3 (float64)."""
    return (corners.to(torch.float64) + 0.5 * width) / float(extent)


_CHILD = torch.tensor([[dx, dy, dz] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)],
                      dtype=torch.int64)


def refine_amr(base: int, refine_fracs, seed: int, device="cpu", octaves: int = 6):
    """Build AMR leaf cells by repeated refinement.

    Starts from ``base``^3 cells at the coarsest level L = len(refine_fracs);
    at each level the cells whose fBm noise value lies in the top
    ``refine_fracs[k]`` fraction (threshold = that quantile among the current
    cells of that level) are split into 8 children one level finer.
    Returns (corners int64 [n,3], level uint8 [n], per-level leaf counts
    ordered from coarsest to finest).
    """
    n_ref = len(refine_fracs)
    lmax = n_ref
    extent = base << lmax
    cur = _grid_corners(base, 1 << lmax, device)
    leaves_c, leaves_l, counts = [], [], []
    noise_seed = substream(seed, S_REFINE)
    for k, frac in enumerate(refine_fracs):
        lev = lmax - k
        width = 1 << lev
        if cur.shape[0] == 0:
            counts.append(0)
            continue
        v = fbm(_centres(cur, width, extent), noise_seed, octaves=octaves)
        n_cur = v.shape[0]
        n_refine = int(round(frac * n_cur))
        if n_refine <= 0:
            mask = torch.zeros(n_cur, dtype=torch.bool, device=device)
        elif n_refine >= n_cur:
            mask = torch.ones(n_cur, dtype=torch.bool, device=device)
        else:
            # threshold = the (n_cur - n_refine)-th smallest value; refine strictly above it
            thr = torch.kthvalue(v.cpu(), n_cur - n_refine).values.item()
            mask = v > thr
        del v
        _progress(f"level {lev}: {n_cur} cells, refining {int(mask.sum())}")
        keep = cur[~mask]
        leaves_c.append(keep)
        leaves_l.append(torch.full((keep.shape[0],), lev, dtype=torch.uint8, device=device))
        counts.append(int(keep.shape[0]))
        par = cur[mask]
        del cur, mask
        half = width >> 1
        ch = (par[:, None, :] + _CHILD.to(device)[None, :, :] * half).reshape(-1, 3)
        del par
        cur = ch
    leaves_c.append(cur)
    leaves_l.append(torch.zeros(cur.shape[0], dtype=torch.uint8, device=device))
    counts.append(int(cur.shape[0]))
    corners = torch.cat(leaves_c, dim=0)
    level = torch.cat(leaves_l, dim=0)
    return corners, level, counts


def astro_fields(cent: torch.Tensor, seed: int, n_fields: int = 4, octaves: int = 4):
    """Correlated astrophysics-like fields at cell centres (float64 in,
    float32 out): log-normal density, temperature anti-correlated with
    density, pressure = density * temperature, velocity magnitude; extra
    fields beyond four are independent blob + fBm fields."""
    fs = substream(seed, S_FIELDS)
    g = zscore(blobs(cent, substream(fs, 1)) + 0.5 * fbm(cent, substream(fs, 2), octaves=octaves))
    rho = torch.exp(1.2 * g)
    del g
    n = fbm(cent, substream(fs, 3), octaves=max(1, octaves - 1))
    temp = rho.pow(-0.5) * torch.exp(0.2 * n)
    del n
    pres = rho * temp
    ga = zscore(blobs(cent, substream(fs, 4)) + 0.5 * fbm(cent, substream(fs, 5), octaves=max(1, octaves - 1)))
    gb = zscore(blobs(cent, substream(fs, 6)) + 0.5 * fbm(cent, substream(fs, 7), octaves=max(1, octaves - 1)))
    vel = torch.sqrt(ga * ga + gb * gb)
    del ga, gb
    out = [rho.float(), temp.float(), pres.float(), vel.float()]
    names = ["dens", "temp", "pres", "velmag"]
    for e in range(4, n_fields):
        extra = zscore(blobs(cent, substream(fs, 10 + e)) + 0.5 * fbm(cent, substream(fs, 20 + e), octaves=max(1, octaves - 1)))
        out.append(extra.float())
        names.append(f"extra{e - 3}")
    return out[:n_fields], names[:n_fields]


def make_regular(side: int, n_fields: int, seed: int, device="cpu") -> Volume:
    """Single-level regular grid of ``side``^3 finest cells; each field is a
    seeded sum of 8 Gaussian blobs normalised to [0,1] plus 0.05 * U(0,1)
    per-cell noise."""
    corners = _grid_corners(side, 1, device)
    cent = _centres(corners, 1, side)
    fs = substream(seed, S_FIELDS)
    fields = []
    for m in range(n_fields):
        b = blobs(cent, substream(fs, 100 + m))
        b = (b - b.min()) / max(float(b.max() - b.min()), 1e-300)
        h = hash3(corners[:, 0], corners[:, 1], corners[:, 2], substream(fs, 200 + m))
        fields.append((b + 0.05 * uniform_from_hash(h)).float())
    n = corners.shape[0]
    return Volume(corners[:, 0].int(), corners[:, 1].int(), corners[:, 2].int(),
                  torch.zeros(n, dtype=torch.uint8, device=device), fields,
                  [f"blob{m}" for m in range(n_fields)], side, 1, [n])


def make_amr(base: int, refine_fracs, n_fields: int, seed: int, device="cpu",
             octaves: int = 6, field_octaves: int = 4) -> Volume:
    """Multi-level AMR volume (refinement ratio 2) with astrophysics-like fields."""
    corners, level, counts = refine_amr(base, refine_fracs, seed, device, octaves)
    extent = base << len(refine_fracs)
    width = (1 << level.to(torch.int64))
    cent = (corners.to(torch.float64) + 0.5 * width[:, None].to(torch.float64)) / float(extent)
    del width
    _progress(f"{corners.shape[0]} leaf cells; evaluating {n_fields} fields")
    fields, names = astro_fields(cent, seed, n_fields, field_octaves)
    del cent
    return Volume(corners[:, 0].int(), corners[:, 1].int(), corners[:, 2].int(), level,
                  fields, names, base, len(refine_fracs) + 1, counts)


def expected_leaves_per_base_cell(refine_fracs) -> float:
    """Expected leaf cells per base cell when level k refines a fraction r_k."""
    g, mult = 0.0, 1.0
    for r in refine_fracs:
        g += mult * (1.0 - r)
        mult *= 8.0 * r
    return g + mult


def base_side_for(n_target: float, refine_fracs) -> int:
    return max(2, int(round((n_target / expected_leaves_per_base_cell(refine_fracs)) ** (1.0 / 3.0))))


def make_tf(seed: int, n_cp: int = 4, n_tf: int = 256) -> torch.Tensor:
    """Alpha transfer function of ``n_tf`` entries: piecewise-linear through
    ``n_cp`` control points (positions sorted U[0,1], alpha U[0,1]), constant
    outside them, sampled at entry centres (i + 0.5) / n_tf.  float32 [n_tf]."""
    g = torch.Generator().manual_seed(seed)
    pos = torch.sort(torch.rand(n_cp, generator=g, dtype=torch.float64)).values
    alpha = torch.rand(n_cp, generator=g, dtype=torch.float64)
    t = (torch.arange(n_tf, dtype=torch.float64) + 0.5) / n_tf
    out = torch.empty(n_tf, dtype=torch.float64)
    for i in range(n_tf):
        ti = float(t[i])
        if ti <= pos[0]:
            out[i] = alpha[0]
        elif ti >= pos[-1]:
            out[i] = alpha[-1]
        else:
            k = int(torch.searchsorted(pos, torch.tensor(ti, dtype=torch.float64), right=True)) - 1
            w = (ti - float(pos[k])) / max(float(pos[k + 1] - pos[k]), 1e-300)
            out[i] = (1.0 - w) * alpha[k] + w * alpha[k + 1]
    return out.float()


def make_tfs(seed: int, n_fields: int, n_cp_range=(4, 4), n_tf: int = 256):
    """One TF per field from sub-stream S_TF of ``seed``."""
    ts = substream(seed, S_TF)
    g = torch.Generator().manual_seed(substream(ts, 999))
    out = []
    for m in range(n_fields):
        lo, hi = n_cp_range
        n_cp = lo if lo == hi else int(torch.randint(lo, hi + 1, (1,), generator=g))
        out.append(make_tf(substream(ts, m), n_cp, n_tf))
    return out
