"""Pins of the triangle-sample oracle (CPU): the sampled triangles are
uniform over the brute-force triangle list (Sec. 3 theorem), their number
matches k times the closed fraction, closed forms (complete graph, windmill)
give a single histogram cell, and the box statistics agree with numpy's
nearest-rank percentile and an explicit Tukey fence."""
import math
from itertools import combinations

import numpy as np
import pytest

from oracle import bruteforce as BF
from oracle import oracle as O
from oracle import triangle_oracle as T


def global_sample(src, dst, n, k, seed, B=16):
    og = O.build_graph(np.asarray(src, np.uint32), np.asarray(dst, np.uint32), n)
    s = O.sample(og, 2, 2, B, np.zeros(B, np.uint64), k, seed, dump_per_bin=k)
    return og, s.v[B], s.a[B], s.c[B], s


def test_sampled_triangles_are_uniform():
    rng = np.random.default_rng(5)
    n = 30
    e = [(u, w) for u, w in combinations(range(n), 2) if rng.random() < 0.2]
    src, dst = zip(*e)
    adj = BF.simple_graph(e, n)
    tris = [t for t in combinations(range(n), 3)
            if t[1] in adj[t[0]] and t[2] in adj[t[0]] and t[2] in adj[t[1]]]
    assert len(tris) > 20
    k = 200_000
    og, v, a, c, _ = global_sample(src, dst, n, k, seed=9)
    idx, d = T.triangles(og, v, a, c)
    got = {}
    for i in idx:
        key = tuple(sorted((int(v[i]), int(a[i]), int(c[i]))))
        got[key] = got.get(key, 0) + 1
    assert set(got) == set(tris)              # only triangles, and every one
    # uniform: chi-square with len(tris) - 1 degrees of freedom, far tail
    cnt = np.array([got[t] for t in tris], dtype=np.float64)
    exp = cnt.sum() / len(tris)
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    df = len(tris) - 1
    assert chi2 < df + 6 * math.sqrt(2 * df), (chi2, df)
    # the number of closed samples is binomial(k, 3T / p)
    p = sum(len(nb) * (len(nb) - 1) // 2 for nb in adj.values())
    q = 3 * len(tris) / p
    assert abs(len(idx) - k * q) <= 5 * math.sqrt(k * q * (1 - q))
    # degree triples are the sorted degrees of the sampled vertices
    deg = og.degrees()
    for j, i in enumerate(idx[:500]):
        assert list(d[j]) == sorted([deg[v[i]], deg[a[i]], deg[c[i]]])


def test_complete_graph_and_windmill():
    n = 9
    e = np.array(list(combinations(range(n), 2)), dtype=np.uint32)
    og, v, a, c, _ = global_sample(e[:, 0], e[:, 1], n, 5000, seed=1)
    idx, d = T.triangles(og, v, a, c)
    assert len(idx) == 5000 and (d == n - 1).all()
    h = T.histogram(d, 2, 2, 16)
    b = O.bin_id(n - 1, 2, 2)
    assert h[b, b] == 5000 and h.sum() == 5000
    # windmill: k triangles sharing a hub, degrees (2, 2, 2k); its leaves'
    # wedges are the closed ones
    kk = 7
    src, dst = [], []
    for t in range(kk):
        x, y = 1 + 2 * t, 2 + 2 * t
        src += [0, 0, x]
        dst += [x, y, y]
    og, v, a, c, _ = global_sample(src, dst, 2 * kk + 1, 20000, seed=2)
    idx, d = T.triangles(og, v, a, c)
    assert (d == [2, 2, 2 * kk]).all()
    h = T.histogram(d, 2, 2, 16)
    assert h[O.bin_id(2, 2, 2), O.bin_id(2 * kk, 2, 2)] == len(idx) == h.sum()
    # every wedge at a leaf is closed, the hub's wedges are closed only within
    # a blade: closed fraction 3k / (C(2k, 2) + 2k)
    q = 3 * kk / (kk * (2 * kk - 1) + 2 * kk)
    assert abs(len(idx) / 20000 - q) < 5 * math.sqrt(q * (1 - q) / 20000)


@pytest.mark.parametrize("seed", range(6))
def test_box_matches_numpy_and_tukey(seed):
    rng = np.random.default_rng(seed)
    vals = list(rng.integers(0, 20, int(rng.integers(1, 300))))
    if seed == 0:
        vals = [7]
    if seed == 1:
        vals = [1] * 50 + [19]                  # one far outlier
    r = T.box(vals)
    for p, key in ((25, "q1"), (50, "median"), (75, "q3")):
        assert r[key] == int(np.percentile(vals, p, method="inverted_cdf"))
    iqr = r["q3"] - r["q1"]
    out = [x for x in vals if x < r["q1"] - 1.5 * iqr or x > r["q3"] + 1.5 * iqr]
    assert r["outliers"] == len(out)
    inside = [x for x in vals if x not in out]
    assert r["whisker_lo"] == min(inside) and r["whisker_hi"] == max(inside)
    if seed == 1:
        assert r["outliers"] == 1 and r["whisker_hi"] == 1
