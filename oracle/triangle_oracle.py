"""Triangle sample and degree assortativity, by their definitions (test
infrastructure only; it never imports the product package).

Sec. 3 of Kolda et al. (arXiv 1301.5887): a closed wedge of a uniform wedge
sample is a uniformly sampled triangle (with replacement), because each
triangle owns exactly three wedges.  Sec. 5 (triangle statistics): each
sampled triangle is described by the minimum, middle and maximum degree of
its vertices; triangles are grouped by the bin (Eq. binid, tau = omega = 2)
of the minimum degree and the bin of the maximum degree is summarised per
group by a box plot (quartiles and median, whiskers at the most extreme
points that are not outliers, outliers beyond them).

The paper does not fix the percentile rule or the outlier rule; this oracle
takes the nearest-rank percentile (the ceil(p N)-th smallest value) and
Tukey's fences (1.5 interquartile ranges beyond the quartiles).
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def closed(g: O.Graph, a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Whether each wedge's endpoints are adjacent (a binary search of the
    canonical key min<<32|max in the graph's sorted edge keys)."""
    a = np.asarray(a, dtype=np.uint64)
    c = np.asarray(c, dtype=np.uint64)
    key = (np.minimum(a, c) << np.uint64(32)) | np.maximum(a, c)
    if g.m == 0:
        return np.zeros(key.shape, dtype=bool)
    pos = np.searchsorted(g.keys, key)
    pos = np.minimum(pos, g.m - 1)
    return g.keys[pos] == key


def triangles(g: O.Graph, v, a, c):
    """The sampled wedges' triangles: (index of the wedge in the sample,
    sorted degree triple) for every closed wedge, in sample order."""
    deg = g.degrees().astype(np.int64)
    v = np.asarray(v, dtype=np.int64)
    a = np.asarray(a, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    idx = np.nonzero(closed(g, a, c))[0]
    d = np.sort(np.stack([deg[v[idx]], deg[a[idx]], deg[c[idx]]], axis=1), axis=1)
    return idx, d


def histogram(d: np.ndarray, tau: int, omega: int, max_bins: int) -> np.ndarray:
    """[max_bins, max_bins] counts of (BinId(d_min), BinId(d_max)); triangles
    whose max bin is >= max_bins are left out."""
    h = np.zeros((max_bins, max_bins), dtype=np.uint64)
    for lo, hi in zip(d[:, 0], d[:, 2]):
        b0, b1 = O.bin_id(int(lo), tau, omega), O.bin_id(int(hi), tau, omega)
        if b1 < max_bins:
            h[b0, b1] += 1
    return h


def nearest_rank(sorted_vals, p: float):
    """The ceil(p N)-th smallest of N sorted values (N >= 1)."""
    n = len(sorted_vals)
    r = max(1, math.ceil(p * n))
    return sorted_vals[r - 1]


def box(values) -> dict:
    """Box-plot statistics of a list of values (the max-degree bins of one
    min-degree group)."""
    s = sorted(int(x) for x in values)
    q1, med, q3 = nearest_rank(s, 0.25), nearest_rank(s, 0.5), nearest_rank(s, 0.75)
    iqr = q3 - q1
    lo, hi = q1 - 1.5 * iqr, q3 + 1.5 * iqr
    inside = [x for x in s if lo <= x <= hi]
    return {"count": len(s), "q1": q1, "median": med, "q3": q3,
            "whisker_lo": min(inside + [q1]), "whisker_hi": max(inside + [q3]),
            "outliers": len(s) - len(inside)}


def assortativity(d: np.ndarray, tau: int, omega: int, max_bins: int) -> list:
    """Box statistics of BinId(d_max) for every BinId(d_min) group, in
    increasing min bin."""
    groups = {}
    for lo, hi in zip(d[:, 0], d[:, 2]):
        b1 = O.bin_id(int(hi), tau, omega)
        if b1 < max_bins:
            groups.setdefault(O.bin_id(int(lo), tau, omega), []).append(b1)
    out = []
    for b in sorted(groups):
        row = box(groups[b])
        row["min_bin"] = b
        out.append(row)
    return out
