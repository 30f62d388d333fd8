"""Pure-Python brute force for tiny graphs (test infrastructure only).

Enumerates every wedge and every vertex triple by the definitions of
Sec. 2.1 and 2.2 of Kolda et al. (arXiv 1301.5887), with Python sets.  Used to
pin the C++ oracle's exact mode, its triangle count and its sampler's
support on graphs small enough to enumerate.
"""
from __future__ import annotations

from itertools import combinations


def simple_graph(edges, n):
    """Undirected simple graph: adjacency sets, self-loops and repeats dropped."""
    adj = {v: set() for v in range(n)}
    for u, w in edges:
        if u != w:
            adj[u].add(w)
            adj[w].add(u)
    return adj


def triangles(adj):
    """Number of vertex triples that are pairwise adjacent."""
    t = 0
    for a, b, c in combinations(sorted(adj), 3):
        if b in adj[a] and c in adj[a] and c in adj[b]:
            t += 1
    return t


def wedge_table(adj, bin_of):
    """P[b][q] = |W_{b,q}| (q = 0 open, 1..3 closed with q vertices in bin b),
    keyed by bin id; `bin_of(d)` maps a degree to its bin."""
    P = {}
    for v, nb in adj.items():
        d = len(nb)
        if d < 2:
            continue
        b = bin_of(d)
        row = P.setdefault(b, [0, 0, 0, 0])
        for a, c in combinations(sorted(nb), 2):
            if c in adj[a]:
                q = 1 + (bin_of(len(adj[a])) == b) + (bin_of(len(adj[c])) == b)
                row[q] += 1
            else:
                row[0] += 1
    return P


def all_wedges(adj):
    """Every wedge as (centre, smaller endpoint, larger endpoint)."""
    out = []
    for v, nb in adj.items():
        for a, c in combinations(sorted(nb), 2):
            out.append((v, a, c))
    return out
