"""Python face of the CPU oracle (test infrastructure only).

Only tests, the smoke check and the CPU-baseline leg of the benchmark import
this module.  It wraps ``wedge_oracle.cpp`` (built into ``liboracle.so`` with
g++, no HIP headers) with numpy arrays.  It never imports the product
package, and the product package never imports it.

Paper: Kolda et al., "Counting Triangles in Massive Graphs with MapReduce"
(arXiv 1301.5887).  Section references are given per function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wedge_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u16p = ctypes.POINTER(ctypes.c_uint16)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.orc_lemire16.argtypes = [ctypes.c_uint32, _u16p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.orc_lemire16.restype = ctypes.c_uint32
        L.orc_lemire64_seq.argtypes = [ctypes.c_uint64, _u64p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.orc_lemire64_seq.restype = ctypes.c_uint64
        L.orc_draw_below.argtypes = [ctypes.c_uint64] * 4 + [ctypes.c_int, ctypes.c_uint64]
        L.orc_draw_below.restype = ctypes.c_uint64
        L.orc_bin_lo_deg.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
        L.orc_bin_lo_deg.restype = ctypes.c_uint64
        L.orc_bin_id.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
        L.orc_bin_id.restype = ctypes.c_uint32
        L.orc_hoeffding_k.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_hoeffding_k.restype = ctypes.c_uint64
        L.orc_canon.argtypes = [_u32p, _u32p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u64p]
        L.orc_canon.restype = ctypes.c_uint64
        L.orc_csr.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u32p]
        L.orc_bins.argtypes = [_u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_uint32, _u64p, _u64p]
        L.orc_bins.restype = ctypes.c_int
        L.orc_center_order.argtypes = [_u64p, ctypes.c_uint32, _u32p]
        L.orc_center_order.restype = ctypes.c_uint64
        L.orc_sample.argtypes = [_u64p, _u32p, ctypes.c_uint32, _u64p, ctypes.c_uint64,
                                 ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, _u64p,
                                 ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_uint64, _u64p,
                                 _u32p, _u32p, _u32p, _u8p, ctypes.c_uint64, ctypes.c_int]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample_alloc.argtypes = [_u64p, _u32p, ctypes.c_uint32, _u64p, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, _u64p,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint64, _u64p, _u64p, _u32p, _u32p, _u32p, _u8p,
                                       ctypes.c_uint64]
        L.orc_sample_alloc.restype = ctypes.c_int
        L.orc_exact.argtypes = [_u64p, _u32p, ctypes.c_uint32, _u64p, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, _u64p]
        L.orc_exact.restype = ctypes.c_int
        L.orc_triangles_forward.argtypes = [_u64p, _u32p, ctypes.c_uint32]
        L.orc_triangles_forward.restype = ctypes.c_uint64
        L.orc_estimate.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_double, _f64p, _f64p]
        L.orc_bucket.argtypes = [ctypes.c_uint64]
        L.orc_bucket.restype = ctypes.c_uint32
        L.orc_pair_census.argtypes = [_u64p, _u32p, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_uint32, _u64p]
        L.orc_pair_census.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def num_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Thread count of the oracle's later parallel loops (process-wide)."""
    lib().orc_set_num_threads(int(t))


# ---------------------------------------------------------------- primitives
def philox4x64_10(ctr, key) -> np.ndarray:
    """Philox4x64-10 block for counter ``ctr`` (4 words) and ``key`` (2 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def lemire16(N: int, xs) -> tuple[int, int]:
    a = np.ascontiguousarray(xs, dtype=np.uint16)
    used = ctypes.c_int(0)
    r = lib().orc_lemire16(N, _p(a, _u16p), len(a), ctypes.byref(used))
    return int(r), used.value


def lemire64_seq(N: int, xs) -> tuple[int, int]:
    a = np.ascontiguousarray(xs, dtype=np.uint64)
    used = ctypes.c_int(0)
    r = lib().orc_lemire64_seq(N, _p(a, _u64p), len(a), ctypes.byref(used))
    return int(r), used.value


def draw_below(seed: int, s: int, bin_word: int, graph: int, t: int, N: int) -> int:
    return int(lib().orc_draw_below(seed, s, bin_word, graph, t, N))


def bin_lo_deg(b: int, tau: int, omega: int) -> int:
    """Eq. binlodeg, integer form."""
    return int(lib().orc_bin_lo_deg(b, tau, omega))


def bin_id(d: int, tau: int, omega: int) -> int:
    """Eq. binid, integer form: max{b : BinLoDeg(b) <= d}."""
    return int(lib().orc_bin_id(d, tau, omega))


def hoeffding_k(eps: float, delta: float) -> int:
    """Thm. Hoeffding: k = ceil(0.5 eps^-2 ln(2/delta))."""
    return int(lib().orc_hoeffding_k(eps, delta))


# -------------------------------------------------------------------- graphs
@dataclass
class Graph:
    n: int
    keys: np.ndarray      # sorted canonical keys min<<32|max, uint64[m]
    rowptr: np.ndarray    # uint64[n+1]
    col: np.ndarray       # uint32[2m], rows ascending
    rejected: int = 0

    @property
    def m(self) -> int:
        return int(self.keys.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)


def build_graph(src, dst, n: int, progress=None) -> Graph:
    """Canonical undirected simple graph and its adjacency (Sec. 4.1, 5.1).
    `progress` (a print function) gets a line after the canonical keys."""
    s = np.ascontiguousarray(src, dtype=np.uint32)
    d = np.ascontiguousarray(dst, dtype=np.uint32)
    keys = np.empty(max(len(s), 1), dtype=np.uint64)
    rej = np.zeros(1, dtype=np.uint64)
    m = int(lib().orc_canon(_p(s, _u32p), _p(d, _u32p), len(s), n, _p(keys, _u64p), _p(rej, _u64p)))
    keys = keys[:m]       # a view: no second copy of a multi-GB key array
    if progress:
        progress(f"[oracle] {m} canonical edge keys sorted")
    rowptr = np.zeros(n + 1, dtype=np.uint64)
    col = np.zeros(max(2 * m, 1), dtype=np.uint32)
    lib().orc_csr(_p(keys, _u64p), m, n, _p(rowptr, _u64p), _p(col, _u32p))
    return Graph(n=n, keys=keys, rowptr=rowptr, col=col[: 2 * m], rejected=int(rej[0]))


def sparse_rows(src, dst, n: int):
    """The adjacency of Sec. 4.1 / 5.1 (undirected, self-loops and repeats
    dropped, ids >= n rejected) for graphs whose n is too large for dense
    rows: returns (the vertices that have edges, ascending; their degrees;
    the concatenation of their rows, each ascending; the number of rejected
    input edges).  Plain numpy, for any n < 2^32."""
    s = np.asarray(src, dtype=np.uint64)
    d = np.asarray(dst, dtype=np.uint64)
    bad = (s >= n) | (d >= n)
    keep = ~bad & (s != d)
    lo = np.minimum(s[keep], d[keep])
    hi = np.maximum(s[keep], d[keep])
    edges = np.unique((lo << np.uint64(32)) | hi)
    a = edges >> np.uint64(32)
    b = edges & np.uint64(0xFFFFFFFF)
    u = np.concatenate([a, b])
    w = np.concatenate([b, a])
    order = np.lexsort((w, u))
    u, w = u[order], w[order]
    verts, deg = np.unique(u, return_counts=True)
    return verts, deg.astype(np.uint64), w.astype(np.uint32), int(bad.sum())


def bins(g: Graph, tau: int, omega: int, max_bins: int):
    """Alg. phase1b: (n_b, p_b) per bin.  Raises if a degree's bin >= max_bins."""
    n_b = np.zeros(max_bins, dtype=np.uint64)
    p_b = np.zeros(max_bins, dtype=np.uint64)
    rc = lib().orc_bins(_p(g.rowptr, _u64p), g.n, tau, omega, max_bins, _p(n_b, _u64p), _p(p_b, _u64p))
    if rc != 0:
        raise ValueError("degree beyond max_bins")
    return n_b, p_b


def center_order(g: Graph) -> np.ndarray:
    """Vertices with d >= 2 sorted by (degree, id): the centre order."""
    out = np.zeros(max(g.n, 1), dtype=np.uint32)
    c = int(lib().orc_center_order(_p(g.rowptr, _u64p), g.n, _p(out, _u32p)))
    return out[:c].copy()


@dataclass
class Samples:
    q: np.ndarray          # uint64[(max_bins+1), 4]; last row = global stream
    v: np.ndarray | None   # uint32[(max_bins+1), dump_per_bin]
    a: np.ndarray | None
    c: np.ndarray | None
    cls: np.ndarray | None


DOMAIN_SAMPLE, DOMAIN_TRAIN, DOMAIN_AUX, DOMAIN_EVAL = 1, 2, 3, 4


def sample(g: Graph, tau: int, omega: int, max_bins: int, k_per_bin, k_global: int,
           seed: int, graph_id: int = 0, dump_per_bin: int = 0, nthreads: int = 0,
           domain: int = DOMAIN_SAMPLE, s_begin: int = 0) -> Samples:
    """Sampling mode: Thms cd-est/td-est over the fixed Philox stream
    (key (seed, domain)); samples s_begin .. s_begin + k - 1 of each row."""
    k = np.ascontiguousarray(k_per_bin, dtype=np.uint64)
    assert k.shape[0] == max_bins
    q = np.zeros((max_bins + 1) * 4, dtype=np.uint64)
    rows = max_bins + 1
    if dump_per_bin > 0:
        dv = np.zeros(rows * dump_per_bin, dtype=np.uint32)
        da = np.zeros_like(dv)
        dc = np.zeros_like(dv)
        dcls = np.zeros(rows * dump_per_bin, dtype=np.uint8)
        ptrs = (_p(dv, _u32p), _p(da, _u32p), _p(dc, _u32p), _p(dcls, _u8p))
    else:
        dv = da = dc = dcls = None
        ptrs = (None, None, None, None)
    keys = g.keys if g.m > 0 else np.zeros(1, dtype=np.uint64)
    col = g.col if g.col.size > 0 else np.zeros(1, dtype=np.uint32)
    rc = lib().orc_sample(_p(g.rowptr, _u64p), _p(col, _u32p), g.n, _p(keys, _u64p), g.m,
                          tau, omega, max_bins, _p(k, _u64p), k_global, seed, graph_id,
                          domain, s_begin, _p(q, _u64p), *ptrs, dump_per_bin, nthreads)
    if rc != 0:
        raise ValueError("oracle sample: bad input (bin out of range or samples in an empty bin)")
    shp = (rows, dump_per_bin)
    return Samples(q=q.reshape(rows, 4),
                   v=None if dv is None else dv.reshape(shp),
                   a=None if da is None else da.reshape(shp),
                   c=None if dc is None else dc.reshape(shp),
                   cls=None if dcls is None else dcls.reshape(shp))


DOMAIN_ALLOC = 7


def sample_alloc(g: Graph, tau: int, omega: int, max_bins: int, k_per_bin, k_global: int,
                 seed: int, graph_id: int = 0, dump_per_bin: int = 0,
                 domain: int = DOMAIN_ALLOC):
    """Phase 2a allocation (Alg. phase2a) and per-vertex sampling: returns
    (Samples with q and dumps, totals[max_bins + 1] = samples drawn per row)."""
    k = np.ascontiguousarray(k_per_bin, dtype=np.uint64)
    assert k.shape[0] == max_bins
    rows = max_bins + 1
    q = np.zeros(rows * 4, dtype=np.uint64)
    tot = np.zeros(rows, dtype=np.uint64)
    if dump_per_bin > 0:
        dv = np.zeros(rows * dump_per_bin, dtype=np.uint32)
        da = np.zeros_like(dv)
        dc = np.zeros_like(dv)
        dcls = np.zeros(rows * dump_per_bin, dtype=np.uint8)
        ptrs = (_p(dv, _u32p), _p(da, _u32p), _p(dc, _u32p), _p(dcls, _u8p))
    else:
        dv = da = dc = dcls = None
        ptrs = (None, None, None, None)
    keys = g.keys if g.m > 0 else np.zeros(1, dtype=np.uint64)
    col = g.col if g.col.size > 0 else np.zeros(1, dtype=np.uint32)
    rc = lib().orc_sample_alloc(_p(g.rowptr, _u64p), _p(col, _u32p), g.n, _p(keys, _u64p), g.m,
                                tau, omega, max_bins, _p(k, _u64p), k_global, seed, graph_id,
                                domain, _p(q, _u64p), _p(tot, _u64p), *ptrs, dump_per_bin)
    if rc != 0:
        raise ValueError("oracle sample_alloc: bad input")
    shp = (rows, dump_per_bin)
    s = Samples(q=q.reshape(rows, 4),
                v=None if dv is None else dv.reshape(shp),
                a=None if da is None else da.reshape(shp),
                c=None if dc is None else dc.reshape(shp),
                cls=None if dcls is None else dcls.reshape(shp))
    return s, tot


def exact(g: Graph, tau: int, omega: int, max_bins: int) -> np.ndarray:
    """Exact mode: |W_{b,q}| by enumeration of every wedge (Sec. 2.1, 2.2)."""
    P = np.zeros((max_bins + 1) * 4, dtype=np.uint64)
    keys = g.keys if g.m > 0 else np.zeros(1, dtype=np.uint64)
    col = g.col if g.col.size > 0 else np.zeros(1, dtype=np.uint32)
    rc = lib().orc_exact(_p(g.rowptr, _u64p), _p(col, _u32p), g.n, _p(keys, _u64p), g.m,
                         tau, omega, max_bins, _p(P, _u64p))
    if rc != 0:
        raise ValueError("degree beyond max_bins")
    return P.reshape(max_bins + 1, 4)


def triangles_forward(g: Graph) -> int:
    col = g.col if g.col.size > 0 else np.zeros(1, dtype=np.uint32)
    return int(lib().orc_triangles_forward(_p(g.rowptr, _u64p), _p(col, _u32p), g.n))


def estimate(p_b, q, k_per_bin, k_global: int, delta: float):
    """Alg. phase4c summary + Eq. global_est in double.

    Returns (per_bin[max_bins, 4] = c_b, t_b, eps_b, valid;
             glob[6] = c, t, c_G, t_G, eps_G, sum_b t_b)."""
    pb = np.ascontiguousarray(p_b, dtype=np.uint64)
    qq = np.ascontiguousarray(q, dtype=np.uint64).reshape(-1)
    kk = np.ascontiguousarray(k_per_bin, dtype=np.uint64)
    B = pb.shape[0]
    assert qq.shape[0] == (B + 1) * 4 and kk.shape[0] == B
    ob = np.zeros(B * 4, dtype=np.float64)
    og = np.zeros(6, dtype=np.float64)
    lib().orc_estimate(_p(pb, _u64p), _p(qq, _u64p), _p(kk, _u64p), B, k_global, delta,
                       _p(ob, _f64p), _p(og, _f64p))
    return ob.reshape(B, 4), og


def k_for_bins(p_b, k: int) -> np.ndarray:
    """k samples for every bin with wedges, 0 for the others (Thm cd-est)."""
    pb = np.asarray(p_b, dtype=np.uint64)
    return np.where(pb > 0, np.uint64(k), np.uint64(0)).astype(np.uint64)


def bucket(d: int) -> int:
    """floor(8 L(d)) with L Mitchell's log2 (control-variate feature bucket)."""
    return int(lib().orc_bucket(d))


def pair_census(g: Graph, tau: int, omega: int, max_bins: int) -> dict:
    """{(bin, centre bucket, lo bucket, hi bucket): wedges} by enumeration."""
    out = np.zeros(max_bins * 256 ** 3, dtype=np.uint64)
    col = g.col if g.col.size > 0 else np.zeros(1, dtype=np.uint32)
    rc = lib().orc_pair_census(_p(g.rowptr, _u64p), _p(col, _u32p), g.n, tau, omega, max_bins,
                               _p(out, _u64p))
    if rc != 0:
        raise ValueError("degree beyond max_bins")
    nz = np.nonzero(out)[0]
    res = {}
    for f in nz:
        f = int(f)
        res[(f >> 24, (f >> 16) & 255, (f >> 8) & 255, f & 255)] = int(out[f])
    return res
