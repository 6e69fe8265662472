"""Seeded, device-agnostic noise primitives for the synthetic AMR inputs.

Nothing here is part of the volume-line method: these functions only make
input data (coordinates, field values, transfer functions).  Every random
quantity is either drawn from a seeded ``torch.Generator`` on the CPU (small
parameter arrays) or taken from a counter-based integer hash of
(stream, lattice coordinate), so the values do not depend on the thread count
and differ between CPU and GPU generation only by floating-point rounding.
"""
from __future__ import annotations

import math

import torch

_M32 = 0xFFFFFFFF


def splitmix64(x: int) -> int:
    """SplitMix64 step (Steele, Lea, Flood 2014) on a Python int; used to
    derive independent sub-stream seeds from (seed, stream id)."""
    x = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def substream(seed: int, stream: int) -> int:
    """63-bit seed of sub-stream ``stream`` of base seed ``seed``."""
    return splitmix64(splitmix64(seed) ^ (stream * 0xD1B54A32D192ED03 & 0xFFFFFFFFFFFFFFFF)) >> 1


def hash32(x: torch.Tensor) -> torch.Tensor:
    """32-bit integer finaliser (Wellons' "lowbias32") evaluated in int64
    arithmetic with explicit masking; input and output lie in [0, 2^32)."""
    x = x & _M32
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & _M32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & _M32
    x = x ^ (x >> 16)
    return x


def hash3(i: torch.Tensor, j: torch.Tensor, k: torch.Tensor, seed: int) -> torch.Tensor:
    """Hash of an integer lattice point and a seed, in [0, 2^32)."""
    h = hash32(i + (seed & _M32))
    h = hash32(h ^ (j & _M32))
    h = hash32(h ^ (k & _M32) ^ ((seed >> 32) & _M32))
    return h


def uniform_from_hash(h: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
    """Map a 32-bit hash to U[0, 1)."""
    return h.to(dtype) * (1.0 / 4294967296.0)


# the 12 edge directions of a cube, as in improved gradient noise
_GRADS = torch.tensor(
    [[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0],
     [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
     [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], dtype=torch.float64)


def _fade(t: torch.Tensor) -> torch.Tensor:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(p: torch.Tensor, seed: int) -> torch.Tensor:
    """Gradient noise (Perlin 2002 style: quintic fade, 12 edge gradients,
    lattice gradients chosen by ``hash3``) at points ``p`` [n, 3] (float64).
    Returns values roughly in [-1, 1]."""
    grads = _GRADS.to(p.device)
    fl = torch.floor(p)
    f = p - fl
    ip = fl.to(torch.int64)
    u = _fade(f)
    out = None
    # accumulate the trilinear blend corner by corner to bound memory
    for cx in (0, 1):
        wx = u[:, 0] if cx else (1.0 - u[:, 0])
        for cy in (0, 1):
            wy = u[:, 1] if cy else (1.0 - u[:, 1])
            for cz in (0, 1):
                wz = u[:, 2] if cz else (1.0 - u[:, 2])
                h = hash3(ip[:, 0] + cx, ip[:, 1] + cy, ip[:, 2] + cz, seed)
                g = grads[(h % 12)]
                d = (g[:, 0] * (f[:, 0] - cx) + g[:, 1] * (f[:, 1] - cy)
                     + g[:, 2] * (f[:, 2] - cz))
                term = d * (wx * wy * wz)
                out = term if out is None else out + term
    return out


def _chunk(p: torch.Tensor, chunk: int | None) -> int:
    if chunk is not None:
        return chunk
    return (1 << 25) if p.is_cuda else (1 << 22)


def fbm(p: torch.Tensor, seed: int, octaves: int = 6, base_freq: float = 4.0,
        lacunarity: float = 2.0, gain: float = 0.5, chunk: int | None = None) -> torch.Tensor:
    """Fractional Brownian motion: sum over octaves of gradient noise, each
    octave with its own seed.  ``p`` is [n, 3] in the unit cube (float64).
    Evaluated in chunks of ``chunk`` points to bound temporary memory."""
    n = p.shape[0]
    chunk = _chunk(p, chunk)
    out = torch.empty(n, dtype=torch.float64, device=p.device)
    for s in range(0, n, chunk):
        q = p[s:s + chunk]
        acc = torch.zeros(q.shape[0], dtype=torch.float64, device=p.device)
        freq, amp = base_freq, 1.0
        for o in range(octaves):
            acc += amp * gradient_noise(q * freq, substream(seed, 100 + o))
            freq *= lacunarity
            amp *= gain
        out[s:s + chunk] = acc
    return out


def blob_params(seed: int, n_blobs: int = 8):
    """Centres U[0,1)^3, widths U[0.03,0.15] and amplitudes U[0.5,1] of
    ``n_blobs`` Gaussian blobs, drawn on the CPU from a seeded generator."""
    g = torch.Generator().manual_seed(seed)
    c = torch.rand(n_blobs, 3, generator=g, dtype=torch.float64)
    sig = 0.03 + 0.12 * torch.rand(n_blobs, generator=g, dtype=torch.float64)
    amp = 0.5 + 0.5 * torch.rand(n_blobs, generator=g, dtype=torch.float64)
    return c, sig, amp


def blobs(p: torch.Tensor, seed: int, n_blobs: int = 8, chunk: int | None = None) -> torch.Tensor:
    """Sum of ``n_blobs`` seeded isotropic Gaussian blobs at points ``p``."""
    c, sig, amp = blob_params(seed, n_blobs)
    c, sig, amp = c.to(p.device), sig.to(p.device), amp.to(p.device)
    n = p.shape[0]
    chunk = _chunk(p, chunk)
    out = torch.empty(n, dtype=torch.float64, device=p.device)
    for s in range(0, n, chunk):
        q = p[s:s + chunk]
        acc = torch.zeros(q.shape[0], dtype=torch.float64, device=p.device)
        for b in range(n_blobs):
            d2 = ((q - c[b]) ** 2).sum(dim=1)
            acc += amp[b] * torch.exp(-d2 / (2.0 * sig[b] * sig[b]))
        out[s:s + chunk] = acc
    return out


def zscore(v: torch.Tensor) -> torch.Tensor:
    m = v.mean()
    s = v.std()
    if not math.isfinite(float(s)) or float(s) == 0.0:
        return v - m
    return (v - m) / s
