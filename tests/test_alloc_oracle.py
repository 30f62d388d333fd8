"""Pins of the Phase 2a allocation sampler of the oracle (CPU): per-vertex
counts are the two roundings of q* = C(d,2) k / p_b with E[q_v] = q*, the
totals follow, pairs at a vertex are uniform, and the closed count is
unbiased for k c_b against exact enumeration."""
import math
from fractions import Fraction
from itertools import combinations

import numpy as np

from oracle import oracle as O
from paper_1301_5887_amd.synth import gen


def per_vertex_counts(s, row, total):
    v = s.v[row, :total]
    return {int(x): int(c) for x, c in zip(*np.unique(v, return_counts=True))}


def qstar(og, row_vertices, k, p):
    deg = og.degrees()
    return {v: Fraction(int(deg[v]) * (int(deg[v]) - 1) // 2 * k, p) for v in row_vertices}


def test_counts_are_roundings_and_unbiased():
    n = 300
    src, dst, _ = gen.chung_lu(n, 2.2, 2, 60, 3000, 4)
    og = O.build_graph(src, dst, n)
    B = 16
    nb, pb = O.bins(og, 2, 2, B)
    k = 777
    kk = O.k_for_bins(pb, k)
    deg = og.degrees()
    rows = [b for b in range(B) if pb[b] > 0]
    sums = {b: {} for b in rows}
    R = 200
    for seed in range(R):
        s, tot = O.sample_alloc(og, 2, 2, B, kk, 0, seed, dump_per_bin=4 * k)
        for b in rows:
            verts = [v for v in range(n) if deg[v] >= 2 and O.bin_id(int(deg[v]), 2, 2) == b]
            qs = qstar(og, verts, k, int(pb[b]))
            cnt = per_vertex_counts(s, b, int(tot[b]))
            assert sum(cnt.values()) == int(tot[b]) == int(s.q[b].sum())
            for v in verts:
                c = cnt.get(v, 0)
                assert c in (math.floor(qs[v]), math.ceil(qs[v])), (b, v, c, qs[v])
                sums[b][v] = sums[b].get(v, 0) + c
    # E[q_v] = q*: each vertex's mean over R seeds within 5 binomial sd
    for b in rows:
        verts = list(sums[b])
        qs = qstar(og, verts, k, int(pb[b]))
        for v in verts:
            f = float(qs[v] - math.floor(qs[v]))
            mean = sums[b][v] / R
            assert abs(mean - float(qs[v])) <= 5 * math.sqrt(f * (1 - f) / R) + 1e-12, (b, v)


def test_regular_graph_allocates_exactly():
    # a cycle: every vertex has degree 2 and q* = k / n exactly
    n = 50
    src = np.arange(n, dtype=np.uint32)
    dst = (src + 1) % n
    og = O.build_graph(src, dst.astype(np.uint32), n)
    B = 8
    nb, pb = O.bins(og, 2, 2, B)
    kk = O.k_for_bins(pb, 3 * n)
    s, tot = O.sample_alloc(og, 2, 2, B, kk, 2 * n, 3, dump_per_bin=4 * n)
    b = O.bin_id(2, 2, 2)
    assert int(tot[b]) == 3 * n and int(tot[B]) == 2 * n
    assert all(c == 3 for c in per_vertex_counts(s, b, 3 * n).values())
    assert int(s.q[b, 1:].sum()) == 0          # a cycle has no triangles


def test_pairs_uniform_and_closed_count_unbiased():
    # a bin holding one vertex gets every sample of the bin: its pairs are
    # uniform over its C(d,2) neighbour pairs
    rng = np.random.default_rng(2)
    n, hub = 200, 0
    e = [(hub, w) for w in range(1, 41)]
    e += [(u, w) for u, w in combinations(range(1, 41), 2) if rng.random() < 0.1]
    e += [(int(u), int(w)) for u, w in rng.integers(41, n, (300, 2)) if u != w]
    src, dst = map(lambda a: np.array(a, dtype=np.uint32), zip(*e))
    og = O.build_graph(src, dst, n)
    B = 16
    nb, pb = O.bins(og, 2, 2, B)
    deg = og.degrees()
    bh = O.bin_id(int(deg[hub]), 2, 2)
    assert nb[bh] == 1
    k = 60_000
    kk = O.k_for_bins(pb, k)
    s, tot = O.sample_alloc(og, 2, 2, B, kk, 0, 11, dump_per_bin=k)
    assert int(tot[bh]) == k and (s.v[bh, :k] == hub).all()
    pairs = {}
    for a, c in zip(s.a[bh, :k], s.c[bh, :k]):
        key = (min(a, c), max(a, c))
        pairs[key] = pairs.get(key, 0) + 1
    d = int(deg[hub])
    assert len(pairs) == d * (d - 1) // 2
    cnt = np.array(list(pairs.values()), dtype=np.float64)
    exp = k / len(pairs)
    df = len(pairs) - 1
    assert float(((cnt - exp) ** 2 / exp).sum()) < df + 6 * math.sqrt(2 * df)
    # closed count over seeds: mean of closed / k equals the exact c_b
    P = O.exact(og, 2, 2, B)
    rows = [b for b in range(B) if pb[b] > 0]
    k2 = 2000
    kk2 = O.k_for_bins(pb, k2)
    acc = {b: [] for b in rows}
    for seed in range(60):
        s2, tot2 = O.sample_alloc(og, 2, 2, B, kk2, 0, 100 + seed)
        for b in rows:
            acc[b].append(float(s2.q[b, 1:].sum()) / k2)
    for b in rows:
        c_true = float(P[b, 1:].sum()) / float(pb[b])
        a = np.array(acc[b])
        se = max(a.std(ddof=1), 1e-9) / math.sqrt(len(a))
        assert abs(a.mean() - c_true) <= 5 * se + 1e-12, (b, a.mean(), c_true)
