"""wedge_validate_csr: the device check of the adjacency form (sorted,
simple, undirected; Sec. 4.1) finds nothing in what wedge_build_csr makes,
and counts each planted fault in copies of it; with WEDGE_VALIDATE set,
wedge_sample_close refuses a faulty adjacency with WEDGE_EGRAPH."""
import numpy as np
import pytest
import torch

from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


def counts(rowptr, col, n, m):
    out = torch.empty(4, dtype=torch.int64, device="cuda")
    W._check(W.lib().wedge_validate_csr(W._ptr(rowptr), W._ptr(col), n, m, W._ptr(out),
                                        W._stream()))
    torch.cuda.synchronize()
    return [int(x) for x in W.to_host_u64(out)]


@pytest.fixture(scope="module")
def graph():
    n, src, dst = gen.rmat_graph500(12, 8, seed=3)
    d = lambda a: torch.from_numpy(a.view(np.int32)).cuda()  # noqa: E731
    g = W.build_csr(d(src), d(dst), n)
    torch.cuda.synchronize()
    return g


def test_built_adjacency_is_valid(graph):
    g = graph
    print(f"[validate] n={g.n} m={g.m}", flush=True)
    assert counts(g.rowptr, g.col, g.n, g.m) == [0, 0, 0, 0]


def test_planted_faults_are_counted(graph):
    g = graph
    rp = W.to_host_u64(g.rowptr).astype(np.int64)
    col = g.col[: 2 * g.m].cpu().numpy().view(np.uint32).copy()
    deg = np.diff(rp)
    v = int(np.argmax(deg))                       # a long row
    a, b = int(rp[v]), int(rp[v + 1])
    # swap two entries of row v: out of order (the reverse searches into an
    # unsorted row may then miss, so one-way entries can be counted as well)
    c1 = col.copy()
    c1[a + 3], c1[a + 4] = c1[a + 4], c1[a + 3]
    r = counts(g.rowptr, torch.from_numpy(c1.view(np.int32)).cuda(), g.n, g.m)
    assert r[0] >= 1 and r[1] == 0 and r[3] == 0
    # a row of one vertex's neighbours with one entry repeated: a repeat
    c1 = col.copy()
    c1[a + 1] = c1[a]
    r = counts(g.rowptr, torch.from_numpy(c1.view(np.int32)).cuda(), g.n, g.m)
    assert r[0] >= 1 and r[1] == 0 and r[3] == 0
    # replace the last entry of row v by v itself: a self-loop, and entries
    # without a reverse (the old neighbour's entry for v now has none)
    c2 = col.copy()
    old = int(c2[b - 1])
    c2[b - 1] = v
    r = counts(g.rowptr, torch.from_numpy(c2.view(np.int32)).cuda(), g.n, g.m)
    assert r[1] == 1 and r[2] >= 1 and r[3] == 0 and old != v
    # an id beyond n
    c3 = col.copy()
    c3[a] = g.n + 5
    r = counts(g.rowptr, torch.from_numpy(c3.view(np.int32)).cuda(), g.n, g.m)
    assert r[3] >= 1
    # rowptr[n] != 2m
    rp2 = g.rowptr.clone()
    rp2[-1] = rp2[-1] + 1
    r = counts(rp2, g.col, g.n, g.m)
    assert r[3] >= 1


def test_env_validation_in_sample_close(graph, monkeypatch):
    g = graph
    bi = W.bin_counts(g, 2, 2, 30)
    hk = W.k_for_bins(bi.h_p_b, 1000)
    monkeypatch.setenv("WEDGE_VALIDATE", "1")
    W.sample_close(g, bi, hk, 1000, 5)            # valid: samples as usual
    torch.cuda.synchronize()
    rp = W.to_host_u64(g.rowptr).astype(np.int64)
    v = int(np.argmax(np.diff(rp)))
    bad = g.col.clone()
    bad[int(rp[v])] = v
    gb = W.Csr(n=g.n, m=g.m, rowptr=g.rowptr, col=bad)
    with pytest.raises(W.WedgeError) as ei:
        W.sample_close(gb, bi, hk, 1000, 5)
    assert ei.value.status == -6 and "WEDGE_VALIDATE" in str(ei.value)
