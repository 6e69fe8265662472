"""Exact-rational brute-force dynamic volume lines for tiny inputs.

An independent formulation used to pin the oracle: every quantity is a
``fractions.Fraction``; the TF entry is the exact floor of the normalised
value (inputs are chosen away from entry edges, where the oracle's fp32
quantiser agrees with it); bin membership is decided by interval overlap
(cell [E, E + f) meets bin [b, b + 1) on the W-pixel axis) instead of the
floor/ceil projection.  Pure Python loops: small cases only.
"""
from __future__ import annotations

from fractions import Fraction as Q


def entry(x, lo, hi, n_tf):
    t = (Q(x) - Q(lo)) * n_tf / (Q(hi) - Q(lo))
    a = t.numerator // t.denominator
    return min(max(a, 0), n_tf - 1)


def dvl_exact(level, fields, alpha, lo, hi, W, p, fmin, vmax_mode="range", clamp="importance",
              scale_base=2):
    """Returns dict with exact f, E, F, vmax and per-bin member lists/stats."""
    M = len(fields)
    n = len(level)
    n_tf = len(alpha[0])
    I = [[Q(alpha[m][entry(fields[m][h], lo[m], hi[m], n_tf)]) for h in range(n)] for m in range(M)]
    V = [max(I[m][h] for m in range(M)) - min(I[m][h] for m in range(M)) for h in range(n)]
    if vmax_mode == "exact":
        vmax = max(V)
    else:
        im = [entry(min(fields[m]), lo[m], hi[m], n_tf) for m in range(M)]
        jm = [entry(max(fields[m]), lo[m], hi[m], n_tf) for m in range(M)]
        i, j = min(im), max(jm)
        vmax = max(max(Q(alpha[m][a]) for m in range(M)) - min(Q(alpha[m][a]) for m in range(M))
                   for a in range(i, j + 1))
        if vmax == 0:
            hi_a = max(Q(alpha[m][a]) for m in range(M) for a in range(im[m], jm[m] + 1))
            lo_a = min(Q(alpha[m][a]) for m in range(M) for a in range(im[m], jm[m] + 1))
            vmax = hi_a - lo_a
    fmin = Q(fmin)
    f = []
    for h in range(n):
        r = V[h] / vmax if vmax > 0 else Q(0)
        s = Q(scale_base) ** int(level[h])
        if clamp == "importance":
            g = (r * s) ** p
            f.append(max(fmin, g))
        else:
            f.append((max(fmin, r) * s) ** p)
    E = [Q(0)]
    for v in f:
        E.append(E[-1] + v)
    F = E[-1]
    if F == 0:
        f = [Q(1)] * n
        E = [Q(h) for h in range(n + 1)]
        F = E[-1]
    # interval overlap on the pixel axis
    members = [[] for _ in range(W)]
    for h in range(n):
        x1, x2 = E[h] * W / F, E[h + 1] * W / F
        hit = False
        for b in range(W):
            if x1 < b + 1 and x2 > b:
                members[b].append(h)
                hit = True
        if not hit:  # zero-width cell: the bin holding its position (last bin at the end)
            b = min(x1.numerator // x1.denominator, W - 1)
            members[b].append(h)
    out = {"f": f, "E": E, "F": F, "vmax": vmax, "members": members, "mean": [], "vmin": [],
           "vmax_bin": [], "y": []}
    for m in range(M):
        mm, mn, mx, yy = [], [], [], []
        for b in range(W):
            vals = [Q(fields[m][h]) for h in members[b]]
            if not vals:
                mm.append(None); mn.append(None); mx.append(None); yy.append(None)
                continue
            mean = sum(vals) / len(vals)
            mm.append(mean); mn.append(min(vals)); mx.append(max(vals))
            yy.append(Q(alpha[m][entry(mean, lo[m], hi[m], n_tf)]))
        out["mean"].append(mm); out["vmin"].append(mn); out["vmax_bin"].append(mx); out["y"].append(yy)
    return out
