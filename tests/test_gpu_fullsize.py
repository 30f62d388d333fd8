"""The plain path at its full benchmark size (R-MAT scale 24, edge factor 16,
seed 7; the launch configuration bench.py times) against the oracle: the whole
CSR and bin table, every sample of the first 2,048 of each bin and of the global
stream one by one, and the class counts of the first 65,536 samples."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


B = 64


@pytest.fixture(scope="module")
def s24():
    t0 = time.time()
    n, src, dst = gen.rmat_graph500(24, 16, 7)
    print(f"[full] generated n={n} m_in={len(src)} in {time.time() - t0:.1f}s", flush=True)
    d_src = torch.from_numpy(src.view(np.int32)).cuda()
    d_dst = torch.from_numpy(dst.view(np.int32)).cuda()
    g = W.build_csr(d_src, d_dst, n)
    bi = W.bin_counts(g, 2, 2, B)
    torch.cuda.synchronize()
    og = O.build_graph(src, dst, n)
    print(f"[full] oracle graph at {time.time() - t0:.1f}s", flush=True)
    return n, src, dst, g, bi, og


def test_rmat_scale24_full_size_sampled_parity(s24):
    t0 = time.time()
    n, src, dst, g, bi, og = s24
    k = W.hoeffding_k(1e-3, 1e-3)
    hk = W.k_for_bins(bi.h_p_b, k)
    so = W.sample_close(g, bi, hk, k, 7, dump_per_bin=2048)   # every sample: counts over all k
    torch.cuda.synchronize()
    print(f"[full] GPU path done at {time.time() - t0:.1f}s", flush=True)
    assert g.m == og.m
    assert (W.to_host_u64(g.rowptr) == og.rowptr).all()
    assert (g.col[: 2 * g.m].cpu().numpy().view(np.uint32) == og.col).all()
    n_b, p_b = O.bins(og, 2, 2, B)
    assert (bi.h_n_b == n_b).all() and (bi.h_p_b == p_b).all()
    # samples one by one: the first 2,048 of each row
    ks = np.minimum(hk, np.uint64(2048)).astype(np.uint64)
    s = O.sample(og, 2, 2, B, ks, 2048, 7, dump_per_bin=2048)
    dump = so.dump.cpu().numpy().view(np.uint32).reshape(B + 1, 2048, 4)
    for row in range(B + 1):
        kk = 2048 if row == B else int(ks[row])
        if kk == 0:
            continue
        assert (dump[row, :kk, 0] == s.v[row, :kk]).all(), row
        assert (dump[row, :kk, 1] == s.a[row, :kk]).all(), row
        assert (dump[row, :kk, 2] == s.c[row, :kk]).all(), row
        assert (dump[row, :kk, 3] == s.cls[row, :kk]).all(), row
    # class counts over the first 65,536 samples of every row
    k2 = np.minimum(hk, np.uint64(1 << 16)).astype(np.uint64)
    s2 = O.sample(og, 2, 2, B, k2, 1 << 16, 7)
    so2 = W.sample_close(g, bi, k2, 1 << 16, 7)
    assert (W.to_host_u64(so2.q).reshape(B + 1, 4) == s2.q).all()
    print(f"[full] compared at {time.time() - t0:.1f}s", flush=True)


def test_rmat_scale24_widened_rows(s24):
    """The rows beyond the plain path on the same graph: the Phase 2a
    allocation (every sample of 20,000 per row), the triangle sample of
    300,000 global-stream wedges, and the closure join of the first 2,048
    wedges of every row against the whole streamed edge list."""
    from oracle import triangle_oracle as TO
    from paper_1301_5887_amd import triangles as TR
    n, src, dst, g, bi, og = s24
    t0 = time.time()
    k = 20_000
    hk = W.k_for_bins(bi.h_p_b, k)
    dpb = k + 4096
    sa, tot = W.sample_alloc(g, bi, hk, k, 11, dump_per_bin=dpb)
    s, otot = O.sample_alloc(og, 2, 2, B, hk, k, 11, dump_per_bin=dpb)
    assert (tot == otot).all()
    assert (W.to_host_u64(sa.q).reshape(B + 1, 4) == s.q).all()
    dump = sa.dump.cpu().numpy().view(np.uint32).reshape(B + 1, dpb, 4)
    for row in range(B + 1):
        t = int(tot[row])
        if t == 0:
            continue
        assert (dump[row, :t, 0] == s.v[row, :t]).all(), row
        assert (dump[row, :t, 1] == s.a[row, :t]).all(), row
        assert (dump[row, :t, 2] == s.c[row, :t]).all(), row
        assert (dump[row, :t, 3] == s.cls[row, :t]).all(), row
    print(f"[full] allocation compared at {time.time() - t0:.1f}s", flush=True)
    kt = 300_000
    ts = TR.sample(g, bi, kt, 13, max_bins=B)
    st = O.sample(og, 2, 2, B, np.zeros(B, dtype=np.uint64), kt, 13, dump_per_bin=kt)
    idx, d = TO.triangles(og, st.v[B], st.a[B], st.c[B])
    assert ts.count == len(idx) and (ts.triangles["sample"] == idx).all()
    assert (ts.triangles["d_max"] == d[:, 2]).all() and (ts.triangles["d_min"] == d[:, 0]).all()
    assert (ts.hist == TO.histogram(d, 2, 2, B)).all()
    print(f"[full] triangles compared at {time.time() - t0:.1f}s", flush=True)
    kj = W.hoeffding_k(1e-3, 1e-3)
    hkj = W.k_for_bins(bi.h_p_b, kj)
    so = W.sample_close(g, bi, hkj, kj, 7, dump_per_bin=2048)
    dmp = so.dump.cpu().numpy().view(np.uint32).reshape(B + 1, 2048, 4)
    rows = [r for r in range(B) if hkj[r] > 0] + [B]
    recs = np.concatenate([dmp[r] for r in rows])
    a = torch.from_numpy(recs[:, 1].view(np.int32).copy()).cuda()
    c = torch.from_numpy(recs[:, 2].view(np.int32).copy()).cuda()
    hs = torch.from_numpy(src.view(np.int32)).pin_memory()
    hd = torch.from_numpy(dst.view(np.int32)).pin_memory()
    closed = W.closure_join(a, c, hs, hd).cpu().numpy()
    assert (closed == (recs[:, 3] > 0)).all()
    print(f"[full] join compared at {time.time() - t0:.1f}s", flush=True)
