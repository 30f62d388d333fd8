"""ctypes wrapper over ``synth.c`` (built with gcc + OpenMP into libsynth.so)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)

# Graph500 Kronecker generator matrix [a b; c d] (Sec. 5.1).
GRAPH500_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.synth_rmat.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_int, _u32p, _u32p]
        L.synth_chung_lu.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _u32p,
                                     _u32p, _u32p]
        L.synth_bter.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                 ctypes.c_uint64, _u32p, _u32p, ctypes.c_uint64, _u64p]
        L.synth_bter.restype = ctypes.c_uint64
        L.synth_batch_shape.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        _u32p, _u32p]
        _lib = L
    return _lib


def rmat(scale: int, n_edges: int, seed: int, abc=GRAPH500_ABC, permute: bool = True):
    """R-MAT edge list on 2^scale vertices: (src, dst) uint32 arrays."""
    src = np.empty(n_edges, dtype=np.uint32)
    dst = np.empty(n_edges, dtype=np.uint32)
    a, b, c = abc
    _L().synth_rmat(scale, n_edges, a, b, c, seed, int(permute),
                    src.ctypes.data_as(_u32p), dst.ctypes.data_as(_u32p))
    return src, dst


def rmat_graph500(scale: int, edgefactor: int, seed: int, permute: bool = True):
    """Graph500 shape: 2^scale vertices, edgefactor * 2^scale edge draws."""
    n = 1 << scale
    src, dst = rmat(scale, edgefactor * n, seed, GRAPH500_ABC, permute)
    return n, src, dst


def chung_lu(n: int, gamma: float, wmin: int, wmax: int, n_draws: int, seed: int):
    """Chung-Lu edge draws with power-law expected degrees; returns (src, dst, w)."""
    src = np.empty(n_draws, dtype=np.uint32)
    dst = np.empty(n_draws, dtype=np.uint32)
    w = np.empty(n, dtype=np.uint32)
    _L().synth_chung_lu(n, gamma, wmin, wmax, n_draws, seed, src.ctypes.data_as(_u32p),
                        dst.ctypes.data_as(_u32p), w.ctypes.data_as(_u32p))
    return src, dst, w


def chung_lu_c1(seed: int = 1):
    """The small heavy-tailed workload: n = 10,000, exponent 2.3 on [2, 500],
    100,000 endpoint-pair draws (about 1e5 edges after clean-up)."""
    n = 10_000
    src, dst, _ = chung_lu(n, 2.3, 2, 500, 100_000, seed)
    return n, src, dst


def bter(n: int, gamma: float, dmin: int, dmax: int, seed: int, progress=None):
    """BTER-like community graph; returns (src, dst).  `progress` (a print
    function) gets a line after the counting pass."""
    need = np.zeros(1, dtype=np.uint64)
    t0 = time.time()
    _L().synth_bter(n, gamma, dmin, dmax, seed, None, None, 0, need.ctypes.data_as(_u64p))
    cap = int(need[0])
    if progress:
        progress(f"[gen] BTER n={n}: {cap} edges counted in {time.time() - t0:.1f}s")
    src = np.empty(max(cap, 1), dtype=np.uint32)
    dst = np.empty(max(cap, 1), dtype=np.uint32)
    got = _L().synth_bter(n, gamma, dmin, dmax, seed, src.ctypes.data_as(_u32p),
                          dst.ctypes.data_as(_u32p), cap, need.ctypes.data_as(_u64p))
    return src[:got], dst[:got]


def batch_shapes(count: int, seed: int, smin=10, smax=20, emin=8, emax=32):
    """(scale, edgefactor) of each graph of a batch."""
    out = []
    s = np.zeros(1, dtype=np.uint32)
    e = np.zeros(1, dtype=np.uint32)
    for g in range(count):
        _L().synth_batch_shape(seed, g, smin, smax, emin, emax, s.ctypes.data_as(_u32p),
                               e.ctypes.data_as(_u32p))
        out.append((int(s[0]), int(e[0])))
    return out
