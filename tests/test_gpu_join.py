"""Closure by a join against the unsorted edge list streamed from host
memory: the flags equal the sampler's own closure classes and the oracle's
edge-set membership, for one chunk, many ragged chunks, pinned and pageable
host memory."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import triangle_oracle as TO
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


@pytest.mark.parametrize("case,chunk,pinned", [("chung_lu", 0, True), ("chung_lu", 1_000, False),
                                               ("rmat14", 77_777, True)])
def test_join_matches_sampler_and_oracle(case, chunk, pinned):
    if case == "chung_lu":
        n, src, dst = gen.chung_lu_c1(1)
        k = 30_000
    else:
        n, src, dst = gen.rmat_graph500(14, 16, seed=7)
        k = 20_000
    print(f"[join] {case} m_in={len(src)} chunk={chunk} pinned={pinned}", flush=True)
    B = 40
    g = W.build_csr(dev(src), dev(dst), n)
    bi = W.bin_counts(g, 2, 2, B)
    hk = W.k_for_bins(bi.h_p_b, k)
    so = W.sample_close(g, bi, hk, k, 5, dump_per_bin=k)
    torch.cuda.synchronize()
    dump = so.dump.cpu().numpy().view(np.uint32).reshape(B + 1, k, 4)
    rows = [r for r in range(B) if hk[r] > 0] + [B]
    recs = np.concatenate([dump[r] for r in rows])
    a = torch.from_numpy(recs[:, 1].view(np.int32).copy()).cuda()
    c = torch.from_numpy(recs[:, 2].view(np.int32).copy()).cuda()
    hs = torch.from_numpy(src.view(np.int32).copy())
    hd = torch.from_numpy(dst.view(np.int32).copy())
    if pinned:
        hs, hd = hs.pin_memory(), hd.pin_memory()
    closed = W.closure_join(a, c, hs, hd, chunk_edges=chunk).cpu().numpy()
    assert (closed == (recs[:, 3] > 0)).all()
    og = O.build_graph(src, dst, n)
    assert (closed.astype(bool) == TO.closed(og, recs[:, 1], recs[:, 2])).all()
    assert 0 < closed.sum() < len(closed)
