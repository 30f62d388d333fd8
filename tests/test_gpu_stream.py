"""GPU parity of the streamed path (wedge_sample_stream): a simple edge list in
host memory and no adjacency on the device, against the adjacency path
(wedge_build_csr + wedge_bin_counts + wedge_sample_close) on the same list,
whose parity with the oracle the other GPU tests pin, and against the oracle
directly on a small graph.  Bins, class counts and every record must be
bit-identical.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def host(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).pin_memory()


def simple_edges(src, dst, n, seed):
    """The simple graph of an edge list: one entry per edge, in random order
    and random orientation (ids >= n and self-loops dropped)."""
    ok = (src < n) & (dst < n) & (src != dst)
    s, d = src[ok].astype(np.uint64), dst[ok].astype(np.uint64)
    keys = np.unique(np.minimum(s, d) << np.uint64(32) | np.maximum(s, d))
    rng = np.random.default_rng(seed)
    keys = keys[rng.permutation(keys.size)]
    a = (keys >> np.uint64(32)).astype(np.uint32)
    b = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    flip = rng.random(keys.size) < 0.5
    return np.where(flip, b, a), np.where(flip, a, b)


def adjacency_path(src, dst, n, B, k, kg, seed, tau=2, omega=2, dpb=None):
    ws = W.Workspace()
    g = W.build_csr(dev(src), dev(dst), n, ws=ws)
    bi = W.bin_counts(g, tau, omega, B, ws=ws)
    hk = W.k_for_bins(bi.h_p_b, k)
    kg = kg if int(bi.h_p_b.sum()) else 0
    dpb = dpb or max(int(hk.max()) if hk.size else 0, kg, 1)
    so = W.sample_close(g, bi, hk, kg, seed, dump_per_bin=dpb)
    torch.cuda.synchronize()
    deg = (g.rowptr[1:] - g.rowptr[:-1]).max().item() if n else 0
    return dict(m=g.m, n_b=bi.h_n_b, p_b=bi.h_p_b, hk=hk, kg=kg, dpb=dpb, maxdeg=int(deg),
                q=W.to_host_u64(so.q).reshape(B + 1, 4),
                dump=so.dump.cpu().numpy().view(np.uint32).reshape(B + 1, dpb, 4))


def stream_path(src, dst, n, B, k, kg, seed, dpb, tau=2, omega=2, gather_cap=None, chunk=0,
                pinned=True):
    print(f"[stream] n={n} m_in={len(src)} B={B} k={k} kg={kg} seed={seed} cap={gather_cap} "
          f"chunk={chunk} pinned={pinned}", flush=True)
    if pinned:
        hs, hd = host(src), host(dst)
    else:
        hs, hd = (torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32))
                  for x in (src, dst))
    out = W.sample_stream(hs, hd, n, np.full(B, k, dtype=np.uint64), kg, seed,
                          tau, omega, B, gather_cap=gather_cap, chunk_edges=chunk,
                          dump_per_bin=dpb)
    torch.cuda.synchronize()
    out.q_host = W.to_host_u64(out.q).reshape(B + 1, 4)
    out.dump_host = out.dump.cpu().numpy().view(np.uint32).reshape(B + 1, dpb, 4)
    return out


def assert_same(ref, st, B):
    assert st.m == ref["m"]
    assert (st.bins.h_n_b == ref["n_b"]).all() and (st.bins.h_p_b == ref["p_b"]).all()
    assert (st.h_k == ref["hk"]).all() and st.k_global == ref["kg"]
    assert (st.q_host == ref["q"]).all(), (st.q_host, ref["q"])
    for r in range(B + 1):
        k = ref["kg"] if r == B else int(ref["hk"][r])
        k = min(k, ref["dpb"])
        assert (st.dump_host[r, :k] == ref["dump"][r, :k]).all(), f"row {r}"


@pytest.mark.parametrize("case", ["rmat14", "rmat16_rounds", "bter", "ids25"])
def test_stream_equals_adjacency_path(case):
    B, k, kg, seed, cap, chunk = 40, 3000, 3000, 11, None, 0
    if case == "rmat14":
        n, src, dst = gen.rmat_graph500(14, 16, seed=7)
    elif case == "rmat16_rounds":
        n, src, dst = gen.rmat_graph500(16, 16, seed=7)
        chunk = 100_003          # many chunks and a ragged last one
    elif case == "bter":
        n = 30_000
        src, dst = gen.bter(n, 2.1, 10, 3_000, 11)
    else:
        n = 1 << 25
        src, dst = gen.rmat(25, 400_000, 56)
    a, b = simple_edges(src, dst, n, seed=3)
    ref = adjacency_path(a, b, n, B, k, kg, seed)
    if case == "rmat16_rounds":
        cap = max(ref["maxdeg"], 2 * ref["m"] // 7)
    st = stream_path(a, b, n, B, k, kg, seed, ref["dpb"], gather_cap=cap, chunk=chunk)
    assert_same(ref, st, B)
    assert st.rejected == 0
    if case == "rmat16_rounds":
        assert st.rounds >= 3


@pytest.mark.parametrize("pinned", [True, False])
def test_stream_equals_oracle_small(pinned):
    """Against the oracle, from pinned host memory (read by the copy kernel)
    and from pageable memory (copied by hipMemcpyAsync)."""
    n, src, dst = gen.rmat_graph500(11, 8, seed=4)
    a, b = simple_edges(src, dst, n, seed=5)
    B, k, kg, seed = 24, 5000, 5000, 9
    st = stream_path(a, b, n, B, k, kg, seed, dpb=5000, pinned=pinned)
    og = O.build_graph(a, b, n)
    n_b, p_b = O.bins(og, 2, 2, B)
    assert (st.bins.h_n_b == n_b).all() and (st.bins.h_p_b == p_b).all()
    s = O.sample(og, 2, 2, B, st.h_k, st.k_global, seed, dump_per_bin=5000)
    assert (st.q_host == s.q).all()
    for r in range(B + 1):
        kk = min(st.k_global if r == B else int(st.h_k[r]), 5000)
        d = st.dump_host[r, :kk]
        assert (d[:, 0] == s.v[r, :kk]).all() and (d[:, 1] == s.a[r, :kk]).all(), f"row {r}"
        assert (d[:, 2] == s.c[r, :kk]).all() and (d[:, 3] == s.cls[r, :kk]).all(), f"row {r}"


def test_stream_skips_loops_and_bad_ids():
    n, src, dst = gen.rmat_graph500(12, 8, seed=6)
    a, b = simple_edges(src, dst, n, seed=7)
    a = np.concatenate([a, np.array([5, n, 3, n + 7], dtype=np.uint32)])
    b = np.concatenate([b, np.array([5, 1, n + 1, 2], dtype=np.uint32)])
    B = 30
    ref = adjacency_path(a, b, n, B, 2000, 2000, 5)
    st = stream_path(a, b, n, B, 2000, 2000, 5, ref["dpb"])
    assert_same(ref, st, B)
    assert st.rejected == 3


def test_stream_repeated_edge_is_reported():
    # a 4-clique plus one repeated edge: every vertex is drawn as a centre
    a = np.array([0, 0, 0, 1, 1, 2, 2], dtype=np.uint32)
    b = np.array([1, 2, 3, 2, 3, 3, 3], dtype=np.uint32)
    with pytest.raises(W.WedgeError) as e:
        W.sample_stream(host(a), host(b), 4, np.full(8, 100, dtype=np.uint64), 100, 1, 2, 2, 8)
    assert e.value.status == -6


def test_stream_gather_cap_below_a_centre_degree():
    n = 64
    a = np.zeros(40, dtype=np.uint32)
    b = np.arange(1, 41, dtype=np.uint32)
    with pytest.raises(W.WedgeError) as e:
        W.sample_stream(host(a), host(b), n, np.full(8, 100, dtype=np.uint64), 100, 1, 2, 2, 8,
                        gather_cap=39)
    assert e.value.status == -3


def test_stream_without_edges():
    a = np.zeros(0, dtype=np.uint32)
    st = W.sample_stream(host(a), host(a), 10, np.full(8, 100, dtype=np.uint64), 100, 1,
                         2, 2, 8, dump_per_bin=4)
    torch.cuda.synchronize()
    assert st.m == 0 and st.rounds == 0 and int(st.h_k.sum()) == 0 and st.k_global == 0
    assert (W.to_host_u64(st.q) == 0).all()


def simple_edges_on_device(src, dst, n, seed):
    """simple_edges for large lists: the adjacency built on the device gives
    each edge once (u < w); random order and orientation; host arrays out."""
    g = W.build_csr(dev(src), dev(dst), n, ws=W.Workspace())
    m = g.m
    rows = torch.repeat_interleave(torch.arange(n, dtype=torch.int32, device="cuda"),
                                   g.rowptr[1:] - g.rowptr[:-1])
    col = g.col[: 2 * m]
    keep = col > rows
    u, w = rows[keep], col[keep]
    gen_ = torch.Generator(device="cuda")
    gen_.manual_seed(seed)
    perm = torch.randperm(m, device="cuda", generator=gen_)
    u, w = u[perm], w[perm]
    flip = torch.rand(m, device="cuda", generator=gen_) < 0.5
    a = torch.where(flip, w, u).cpu().numpy().view(np.uint32)
    b = torch.where(flip, u, w).cpu().numpy().view(np.uint32)
    return a, b


def test_stream_rmat_scale24_equals_search():
    """The full scale-24 R-MAT graph (Graph500 shape, edge factor 16): its
    simple edge list in pinned host memory, sampled with no adjacency on the
    device (gather rounds of at most a quarter of the edge ends), against the
    search on the adjacency built afterwards."""
    n, src, dst = gen.rmat_graph500(24, 16, seed=7)
    print(f"[stream] scale 24: simple edge list from {len(src)} draws", flush=True)
    a, b = simple_edges_on_device(src, dst, n, 13)
    m = len(a)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    held = torch.cuda.memory_allocated()
    print(f"[stream] device memory held before the streamed run: {held} B", flush=True)
    assert held < 4 * 2 * m    # less than the adjacency's column array alone
    B, k, kg, seed, dpb = 32, 200_000, 200_000, 21, 2048
    st = stream_path(a, b, n, B, k, kg, seed, dpb, gather_cap=m // 2)
    print(f"[stream] m={m} rounds={st.rounds} gathered={st.gathered}", flush=True)
    # a round holds at most m/2 of the 2m edge ends; the drawn centres' rows
    # cover most of the adjacency, so several rounds were needed
    assert st.rounds >= 2 and st.m == m
    ref = adjacency_path(a, b, n, B, k, kg, seed, dpb=dpb)
    assert_same(ref, st, B)
