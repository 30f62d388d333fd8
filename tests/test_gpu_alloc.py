"""The Phase 2a allocation sampler on the GPU against the oracle: realised
totals per row, class counts and every dumped sample (centre, endpoints,
class) bit-exact, and the FP64 estimates with the totals as denominators."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def hub_graph():
    rng = np.random.default_rng(4)
    n = 3000
    s = [rng.integers(0, n, 9000)]
    d = [rng.integers(0, n, 9000)]
    for h, k in [(0, 2500), (1, 1200), (2, 700)]:
        s.append(np.full(k, h))
        d.append(rng.choice(n, k, replace=False))
    return n, np.concatenate(s).astype(np.uint32), np.concatenate(d).astype(np.uint32)


CASES = {
    "worked": lambda: (7, *map(lambda c: np.array(c, np.uint32),
                              zip(*[(1, 2), (1, 3), (2, 4), (3, 4), (3, 5), (4, 5), (4, 6)]))),
    "chung_lu": lambda: gen.chung_lu_c1(1),
    "rmat14": lambda: gen.rmat_graph500(14, 16, seed=7),
    "bter": lambda: (30_000, *gen.bter(30_000, 2.1, 10, 3_000, 11)),
    "hubs": hub_graph,
}


@pytest.mark.parametrize("case,k,kg,seed", [("worked", 500, 700, 1), ("chung_lu", 20_000, 20_001, 3),
                                            ("rmat14", 5_000, 4_321, 5), ("bter", 3_000, 3_000, 9),
                                            ("hubs", 40_000, 10_000, 2)])
def test_alloc_matches_oracle(case, k, kg, seed):
    n, src, dst = CASES[case]()
    B = 40
    print(f"[alloc] {case} n={n} k={k} kg={kg} seed={seed}", flush=True)
    g = W.build_csr(dev(src), dev(dst), n)
    bi = W.bin_counts(g, 2, 2, B)
    hk = W.k_for_bins(bi.h_p_b, k)
    dpb = 2 * max(k, kg) + 64
    so, tot = W.sample_alloc(g, bi, hk, kg, seed, dump_per_bin=dpb)
    torch.cuda.synchronize()
    og = O.build_graph(src, dst, n)
    s, otot = O.sample_alloc(og, 2, 2, B, hk, kg, seed, dump_per_bin=dpb)
    assert (tot == otot).all(), (tot, otot)
    q = W.to_host_u64(so.q).reshape(B + 1, 4)
    assert (q == s.q).all()
    dump = so.dump.cpu().numpy().view(np.uint32).reshape(B + 1, dpb, 4)
    for row in range(B + 1):
        t = int(tot[row])
        assert t <= dpb
        if t == 0:
            continue
        assert (dump[row, :t, 0] == s.v[row, :t]).all(), row
        assert (dump[row, :t, 1] == s.a[row, :t]).all(), row
        assert (dump[row, :t, 2] == s.c[row, :t]).all(), row
        assert (dump[row, :t, 3] == s.cls[row, :t]).all(), row
    est = W.estimate(bi, q, tot[:B], int(tot[B]), 1e-3)
    per_bin, glob = O.estimate(bi.h_p_b, s.q, otot[:B], int(otot[B]), 1e-3)
    for b in range(B):
        for key, j in (("c", 0), ("t", 1)):
            assert abs(est.bins[b][key] - per_bin[b, j]) <= 1e-12 * max(1.0, abs(per_bin[b, j]))
    assert abs(est.glob["c_global"] - glob[2]) <= 1e-12 * max(1.0, abs(glob[2]))
