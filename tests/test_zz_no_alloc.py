"""wedge_build_csr_noalloc (the build with its workspace in a static device
array) against wedge_build_csr, through the C ABI: two calls in a row on the
same GPU, the second on a smaller graph (the array keeps the first call's
contents), and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu

MAX_EDGES = 1 << 20


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def build_noalloc(src, dst, n):
    d_src, d_dst = dev(src), dev(dst)
    m_in = len(src)
    rowptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(max(2 * m_in, 1), dtype=torch.int32, device="cuda")
    info = torch.empty(2, dtype=torch.int64, device="cuda")
    rc = W.lib().wedge_build_csr_noalloc(W._ptr(d_src), W._ptr(d_dst), m_in, n, W._ptr(rowptr),
                                         W._ptr(col), W._ptr(info), W._stream())
    assert rc == 0, W.lib().wedge_last_error()
    torch.cuda.synchronize()
    h_info = W.to_host_u64(info)
    m = int(h_info[0])
    return (W.to_host_u64(rowptr), col[: 2 * m].cpu().numpy().view(np.uint32), m,
            int(h_info[1]))


def check_same(src, dst, n):
    print(f"[noalloc] n={n} m_in={len(src)}", flush=True)
    rp, col, m, rej = build_noalloc(src, dst, n)
    g = W.build_csr(dev(src), dev(dst), n)
    torch.cuda.synchronize()
    assert m == g.m and rej == g.rejected
    assert (rp == W.to_host_u64(g.rowptr)).all()
    assert (col == g.col[: 2 * g.m].cpu().numpy().view(np.uint32)).all()


def test_noalloc_matches_build_csr_twice():
    # the largest edge list the static array holds, with repeats, loops and
    # ids out of range
    src, dst = gen.rmat(17, MAX_EDGES, 41)
    n = 1 << 17
    src[:50] = dst[:50]
    src[50:60] = n + 3
    check_same(src, dst, n)
    # a smaller graph second: the array still holds the first call's keys
    src2, dst2 = gen.rmat(11, 5000, 42)
    check_same(src2, dst2, 1 << 11)
    # ids above 2^24 (64-bit keys) on a small edge list
    src3, dst3 = gen.rmat(26, 20000, 43)
    check_same(src3, dst3, 1 << 26)
    # no edges at all: every row empty
    rp, col, m, rej = build_noalloc(np.zeros(0, np.uint32), np.zeros(0, np.uint32), 9)
    assert m == 0 and (rp == 0).all()


def test_noalloc_rejects_sizes_beyond_the_array():
    L = W.lib()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: the size check fails first
    rc = L.wedge_build_csr_noalloc(fake, fake, MAX_EDGES + 1, 10, fake, fake, fake, None)
    assert rc == -3 and b"static scratch" in L.wedge_last_error()
    rc = L.wedge_build_csr_noalloc(fake, fake, 100, 0, fake, fake, fake, None)
    assert rc == -2
