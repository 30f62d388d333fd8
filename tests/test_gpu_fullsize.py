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


def test_rmat_scale24_full_size_sampled_parity():
    t0 = time.time()
    n, src, dst = gen.rmat_graph500(24, 16, 7)
    print(f"[full] generated n={n} m_in={len(src)} in {time.time() - t0:.1f}s", flush=True)
    d_src = torch.from_numpy(src.view(np.int32)).cuda()
    d_dst = torch.from_numpy(dst.view(np.int32)).cuda()
    g = W.build_csr(d_src, d_dst, n)
    B = 64
    bi = W.bin_counts(g, 2, 2, B)
    k = W.hoeffding_k(1e-3, 1e-3)
    hk = W.k_for_bins(bi.h_p_b, k)
    so = W.sample_close(g, bi, hk, k, 7, dump_per_bin=2048)   # every sample: counts over all k
    torch.cuda.synchronize()
    print(f"[full] GPU path done at {time.time() - t0:.1f}s", flush=True)
    og = O.build_graph(src, dst, n)
    print(f"[full] oracle graph at {time.time() - t0:.1f}s", flush=True)
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
