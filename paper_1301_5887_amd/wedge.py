"""Thin Python binding of libwedge (ctypes).

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of ``include/wedge.h``.  PyTorch supplies device memory and the stream.
There is no CPU fallback: if ``libwedge.so`` is missing or no GPU is
present, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# WEDGE_LIB selects another build of the same library (the host-sanitizer
# build of the checks); by default the in-tree libwedge.so.
LIB_PATH = os.environ.get("WEDGE_LIB") or os.path.join(_HERE, "libwedge.so")

_c_u64 = ctypes.c_uint64
_c_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p


class WedgeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libwedge status {status}: {message}")
        self.status = status


class WedgeSampleRec(ctypes.Structure):
    _fields_ = [("v", ctypes.c_uint32), ("a", ctypes.c_uint32), ("c", ctypes.c_uint32),
                ("cls", ctypes.c_uint32)]


class WedgeTriangleBoxRow(ctypes.Structure):
    _fields_ = [("count", _c_u64), ("outliers", _c_u64), ("q1", _c_u32), ("median", _c_u32),
                ("q3", _c_u32), ("whisker_lo", _c_u32), ("whisker_hi", _c_u32),
                ("pad", _c_u32)]


class WedgeBinEstimate(ctypes.Structure):
    _fields_ = [("bin", ctypes.c_uint32), ("valid", ctypes.c_uint32), ("lo_deg", _c_u64),
                ("n_b", _c_u64), ("p_b", _c_u64), ("k_b", _c_u64), ("q", _c_u64 * 4),
                ("c", ctypes.c_double), ("t", ctypes.c_double), ("eps", ctypes.c_double)]


class WedgeGlobalEstimate(ctypes.Structure):
    _fields_ = [("p", _c_u64), ("k_global", _c_u64), ("q_global", _c_u64 * 4),
                ("c", ctypes.c_double), ("t", ctypes.c_double), ("c_global", ctypes.c_double),
                ("t_global", ctypes.c_double), ("eps_global", ctypes.c_double),
                ("t_bins_sum", ctypes.c_double)]


class CvFitRow(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("rho2", ctypes.c_double), ("var_x", ctypes.c_double),
                ("var_z", ctypes.c_double), ("plan_plain", _c_u64), ("plan_cv", _c_u64)]


class CvRow(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("sx", ctypes.c_int64), ("sg", ctypes.c_int64),
                ("sg2", ctypes.c_int64), ("sxg", ctypes.c_int64), ("an", ctypes.c_int64),
                ("ag", ctypes.c_int64), ("ag2", ctypes.c_int64), ("beta", ctypes.c_double),
                ("exact_mean", ctypes.c_double), ("mode", _c_u32), ("pad", _c_u32),
                ("done", _c_u64)]


class CvResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("halfwidth", ctypes.c_double),
                ("more", ctypes.c_int32), ("pad", ctypes.c_int32)]


CV_PLAIN, CV_EXACT, CV_AUX, CV_CENTRE = 0, 1, 2, 3


class BatchDesc(ctypes.Structure):
    _fields_ = [("num_graphs", _c_u32), ("max_bins", _c_u32), ("tau", _c_u32), ("max_n", _c_u32),
                ("omega", _c_u64), ("k_per_bin", _c_u64), ("k_global", _c_u64), ("seed", _c_u64),
                ("total_edges", _c_u64), ("total_vertices", _c_u64)]


class LaunchShape(ctypes.Structure):
    _fields_ = [("lanes_in_flight", ctypes.c_int), ("samples_per_tile", _c_u32),
                ("workgroups", _c_u32)]


_dp = ctypes.POINTER(BatchDesc)
_sp = ctypes.POINTER(LaunchShape)

# name -> (restype, argtypes); the C-ABI surface declared in include/wedge.h
SIGNATURES = {
    "wedge_last_error": (ctypes.c_char_p, []),
    "wedge_abi_version": (ctypes.c_int, []),
    "wedge_bin_lo_deg": (_c_u64, [_c_u32, _c_u32, _c_u64]),
    "wedge_bin_id": (_c_u32, [_c_u64, _c_u32, _c_u64]),
    "wedge_hoeffding_k": (_c_u64, [ctypes.c_double, ctypes.c_double]),
    "wedge_build_csr_workspace": (ctypes.c_size_t, [_c_u64, _c_u32]),
    "wedge_build_csr": (ctypes.c_int, [_vp, _vp, _c_u64, _c_u32, _vp, _vp, _vp, _vp,
                                       ctypes.c_size_t, _vp]),
    "wedge_build_csr_noalloc": (ctypes.c_int, [_vp, _vp, _c_u64, _c_u32, _vp, _vp, _vp, _vp]),
    "wedge_validate_csr": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _vp]),
    "wedge_index_bytes": (ctypes.c_size_t, [_c_u32, _c_u64, _c_u32]),
    "wedge_bin_counts_workspace": (ctypes.c_size_t, [_c_u32]),
    "wedge_bin_counts": (ctypes.c_int, [_vp, _c_u32, _c_u64, _c_u32, _c_u64, _c_u32, _vp, _vp,
                                        _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp]),
    "wedge_index_status": (ctypes.c_int, [_vp, ctypes.POINTER(_c_u32), ctypes.POINTER(_c_u64),
                                          ctypes.POINTER(_c_u64), ctypes.POINTER(_c_u64), _vp]),
    "wedge_sample_close": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp, _c_u64,
                                          _c_u64, _c_u32, _vp, _vp, _vp, _c_u64, _vp]),
    "wedge_sample_close_tuned": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp,
                                                _c_u64, _c_u64, _c_u32, _vp, _vp, _vp, _c_u64,
                                                ctypes.c_int, _c_u64, _vp]),
    "wedge_edge_hash_bits": (_c_u32, [_c_u64]),
    "wedge_edge_hash_build": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp, _vp]),
    "wedge_sample_close_hashed": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp,
                                                 _c_u64, _c_u64, _c_u32, _vp, _vp, _vp, _c_u64,
                                                 _vp, _c_u32, _vp]),
    "wedge_estimate": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_u32, _c_u32, _c_u64, _c_u64,
                                      ctypes.c_double, _vp, _vp]),
    "wedge_batch_workspace_bytes": (ctypes.c_size_t, [_dp]),
    "wedge_batch_prepare": (ctypes.c_int, [_dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp]),
    "wedge_batch_sample": (ctypes.c_int, [_dp, _sp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    "wedge_batch_run": (ctypes.c_int, [_dp, _vp, _vp, _vp, _vp, _sp, ctypes.c_double, _vp, _vp,
                                       _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_batch_graph_create": (ctypes.c_int, [_dp, _vp, _vp, _vp, _vp, _sp, ctypes.c_double,
                                                _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_void_p)]),
    "wedge_batch_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "wedge_batch_graph_destroy": (ctypes.c_int, [_vp]),
    "wedge_batch_autotune": (ctypes.c_int, [_dp, _sp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp,
                                            ctypes.c_size_t, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_int), _vp]),
    "wedge_sample_close_autotune": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp,
                                                   _c_u64, _c_u64, _sp, ctypes.c_int, ctypes.c_int,
                                                   _vp, _vp, ctypes.POINTER(ctypes.c_float),
                                                   ctypes.POINTER(ctypes.c_int), _vp]),
    "wedge_sample_close_shape": (ctypes.c_int, [_c_u32, _c_u64, _c_u32, _sp]),
    "wedge_sample_features": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _c_u32,
                                             _c_u64, _vp, _vp, _c_u64, _c_u32, _c_u32,
                                             ctypes.c_int, _vp, _c_u64, _vp, _vp]),
    "wedge_mlp_state_bytes": (ctypes.c_size_t, []),
    "wedge_mlp_set": (ctypes.c_int, [_vp, _vp, _vp]),
    "wedge_mlp_get": (ctypes.c_int, [_vp, _vp, _vp]),
    "wedge_mlp_init": (ctypes.c_int, [_vp, _c_u64, _vp]),
    "wedge_mlp_forward": (ctypes.c_int, [_vp, _vp, _c_u64, _vp, _vp]),
    "wedge_mlp_grad_workspace": (ctypes.c_size_t, [_c_u64]),
    "wedge_mlp_grad": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _c_u64, _c_u64, _vp, _vp, _vp,
                                      ctypes.c_size_t, _vp]),
    "wedge_mlp_adam": (ctypes.c_int, [_vp, _vp, _c_u32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, _vp]),
    "wedge_mlp_train_workspace": (ctypes.c_size_t, [_c_u32, _c_u64]),
    "wedge_mlp_train": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _c_u64, _c_u64, _c_u32, _c_u32,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_cv_moments": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _c_u64, _vp, _vp, _vp]),
    "wedge_cv_keys": (ctypes.c_int, [_vp, _c_u32, _c_u32, _c_u64, _vp]),
    "wedge_cv_gtable_workspace": (ctypes.c_size_t, [_c_u32]),
    "wedge_cv_gtable": (ctypes.c_int, [_vp, _vp, _c_u32, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_cv_centre_means_workspace": (ctypes.c_size_t, [_c_u64]),
    "wedge_cv_centre_means": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _c_u32,
                                             _c_u64, _vp, _vp, _c_u64, _c_u32, _c_u32, _vp,
                                             _vp, _vp, _c_u64, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_sample_alloc_workspace": (ctypes.c_size_t, [_c_u32, _c_u32]),
    "wedge_sample_alloc": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _vp, _c_u64,
                                          _c_u64, _vp, _vp, _vp, _c_u64, _vp, ctypes.c_size_t,
                                          _vp]),
    "wedge_sample_stream_workspace": (ctypes.c_size_t, [_c_u32, _c_u64, _c_u32, _vp, _c_u64,
                                                        _c_u64, _c_u64]),
    "wedge_sample_stream": (ctypes.c_int, [_vp, _vp, _c_u64, _c_u32, _c_u32, _c_u64, _c_u32, _vp,
                                           _c_u64, _c_u64, _c_u64, _c_u64, _vp, _vp, _vp, _vp,
                                           _c_u64, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_closure_join_workspace": (ctypes.c_size_t, [_c_u64, _c_u64]),
    "wedge_closure_join": (ctypes.c_int, [_vp, _vp, _c_u64, _vp, _vp, _c_u64, _c_u64, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    "wedge_triangle_stats_workspace": (ctypes.c_size_t, [_c_u64]),
    "wedge_triangle_stats": (ctypes.c_int, [_vp, _c_u64, _c_u32, _c_u64, _c_u32, _vp, _vp, _vp,
                                            _vp, ctypes.c_size_t, _vp]),
    "wedge_triangle_box": (ctypes.c_int, [_vp, _c_u32, _vp]),
    "wedge_eb_halfwidth": (ctypes.c_double, [_c_u64, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double]),
    "wedge_eb_samples": (_c_u64, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double]),
    "wedge_cv_round_size": (_c_u64, [_c_u64, ctypes.c_double, _c_u32, _c_u64]),
    "wedge_cv_fit": (ctypes.c_int, [_vp, _c_u32, ctypes.c_double, ctypes.c_double, _vp]),
    "wedge_cv_estimate": (ctypes.c_int, [_vp, _c_u32, _c_u32, ctypes.c_double, ctypes.c_double,
                                         _c_u64, _vp]),
    "wedge_cv_bin_means": (ctypes.c_int, [_vp, _vp, _vp, _c_u32, _c_u32, _vp, _vp]),
    "wedge_cv_mean_var": (ctypes.c_int, [_vp, _c_u32, _vp, _vp]),
    "wedge_cv_centre_cost": (ctypes.c_double, [_vp, _vp, _c_u32, _c_u32, ctypes.c_double,
                                               ctypes.c_double]),
    "wedge_cv_plan_centre": (ctypes.c_int, [_vp, _vp, _vp, _c_u32, ctypes.c_double,
                                            ctypes.c_double, _vp, _vp, _vp]),
    "wedge_cv_train_workspace": (ctypes.c_size_t, [_c_u32, _c_u64, _c_u64, _c_u64]),
    "wedge_cv_train": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _c_u32, _c_u64, _vp,
                                      _c_u32, _c_u64, _c_u64, _c_u64, _c_u32, ctypes.c_float,
                                      _c_u64, _c_u64, _vp, ctypes.c_double, ctypes.c_double,
                                      _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "wedge_cv_census_bytes": (ctypes.c_size_t, [_c_u32, _c_u64, _c_u32]),
    "wedge_cv_census": (ctypes.c_int, [_vp, _vp, _c_u32, _c_u64, _vp, _c_u32, _c_u32, _c_u64,
                                       _vp, ctypes.c_size_t, _vp]),
    "wedge_cv_census_keys": (ctypes.c_int, [_vp, _c_u32, ctypes.POINTER(_c_u32), _vp, _vp,
                                            _vp]),
    "wedge_cv_exact_mean_workspace": (ctypes.c_size_t, [_c_u32]),
    "wedge_cv_exact_mean": (ctypes.c_int, [_vp, _vp, _c_u32, _vp, _vp, _vp, ctypes.c_size_t,
                                           _vp]),
}

_lib = None


def lib():
    """The loaded libwedge.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise WedgeError(rc, lib().wedge_last_error().decode())


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_gpu(*tensors):
    if not torch.cuda.is_available():
        raise RuntimeError("libwedge needs a GPU (no CPU fallback)")
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("tensor arguments must live on the GPU")


def _u64_tensor(x: torch.Tensor):
    # torch has no uint64 arithmetic on ROCm for every op; keep int64 storage
    # (same bits) and reinterpret on the host.
    return x


def _empty_bytes(nbytes: int, device) -> torch.Tensor:
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def to_host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64).copy()


# --------------------------------------------------------------- host helpers
def hoeffding_k(eps: float, delta: float) -> int:
    return int(lib().wedge_hoeffding_k(eps, delta))


def bin_lo_deg(b: int, tau: int, omega: int) -> int:
    return int(lib().wedge_bin_lo_deg(b, tau, omega))


def bin_id(d: int, tau: int, omega: int) -> int:
    return int(lib().wedge_bin_id(d, tau, omega))


# ---------------------------------------------------------------- the path
@dataclass
class Csr:
    n: int
    m: int
    rowptr: torch.Tensor   # int64 storage of uint64 [n+1]
    col: torch.Tensor      # int32 storage of uint32 [>= 2m]
    rejected: int = 0


class Workspace:
    """Grow-only device scratch reused across calls."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = _empty_bytes(nbytes, self.device)
        return self.buf


# m (wedge_build_csr) or the index's overflow counter (wedge_bin_counts) when
# a sort's bounded wait between tiles gave up
STALLED = (1 << 64) - 1


def build_csr(src: torch.Tensor, dst: torch.Tensor, n: int, ws: Workspace | None = None,
              stream=None, sync: bool = True, out: tuple | None = None):
    """wedge_build_csr.  Returns a Csr (syncs to read m unless sync=False,
    in which case m is None and info is returned in .rejected as a tensor)."""
    _require_gpu(src, dst)
    assert src.dtype == torch.int32 and dst.dtype == torch.int32 and src.numel() == dst.numel()
    m_in = src.numel()
    dev = src.device
    need = int(lib().wedge_build_csr_workspace(m_in, n))
    wbuf = (ws or Workspace(dev)).get(need)
    if out is None:
        rowptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(2 * m_in, 1), dtype=torch.int32, device=dev)
        info = torch.empty(2, dtype=torch.int64, device=dev)
    else:
        rowptr, col, info = out
    _check(lib().wedge_build_csr(_ptr(src), _ptr(dst), m_in, n, _ptr(rowptr), _ptr(col),
                                 _ptr(info), _ptr(wbuf), wbuf.numel(), _stream(stream)))
    if not sync:
        return rowptr, col, info
    h = to_host_u64(info)
    if int(h[0]) == STALLED:
        raise WedgeError(-4, "wedge_build_csr: the sort gave up waiting between tiles")
    return Csr(n=n, m=int(h[0]), rowptr=rowptr, col=col, rejected=int(h[1]))


@dataclass
class BinIndex:
    n: int
    m: int
    tau: int
    omega: int
    max_bins: int
    n_b: torch.Tensor
    p_b: torch.Tensor
    index: torch.Tensor
    h_n_b: np.ndarray | None = None
    h_p_b: np.ndarray | None = None


def bin_counts(g: Csr, tau: int = 2, omega: int = 2, max_bins: int = 64,
               ws: Workspace | None = None, stream=None, read: bool = True) -> BinIndex:
    """wedge_bin_counts; with read=True also copies n_b, p_b to the host and
    checks the overflow counter."""
    _require_gpu(g.rowptr)
    dev = g.rowptr.device
    n_b = torch.empty(max_bins, dtype=torch.int64, device=dev)
    p_b = torch.empty(max_bins, dtype=torch.int64, device=dev)
    ib = int(lib().wedge_index_bytes(g.n, g.m, max_bins))
    index = _empty_bytes(ib, dev)
    need = int(lib().wedge_bin_counts_workspace(g.n))
    wbuf = (ws or Workspace(dev)).get(need)
    _check(lib().wedge_bin_counts(_ptr(g.rowptr), g.n, g.m, tau, omega, max_bins, _ptr(n_b),
                                  _ptr(p_b), _ptr(index), index.numel(), _ptr(wbuf),
                                  wbuf.numel(), _stream(stream)))
    bi = BinIndex(n=g.n, m=g.m, tau=tau, omega=omega, max_bins=max_bins, n_b=n_b, p_b=p_b,
                  index=index)
    if read:
        st = index_status(bi, stream)
        if st["overflow"] == STALLED:
            raise WedgeError(-4, "wedge_bin_counts: the sort gave up waiting between tiles")
        if st["overflow"]:
            raise WedgeError(-2, f"{st['overflow']} vertices have a bin >= max_bins={max_bins}")
        bi.h_n_b = to_host_u64(n_b)
        bi.h_p_b = to_host_u64(p_b)
    return bi


def index_status(bi: BinIndex, stream=None) -> dict:
    nc = _c_u32(0)
    ov, eb, mm = _c_u64(0), _c_u64(0), _c_u64(0)
    _check(lib().wedge_index_status(_ptr(bi.index), ctypes.byref(nc), ctypes.byref(ov),
                                    ctypes.byref(eb), ctypes.byref(mm), _stream(stream)))
    return {"num_classes": nc.value, "overflow": ov.value, "empty_bin_samples": eb.value,
            "mismatch": mm.value}


def k_for_bins(h_p_b: np.ndarray, k: int) -> np.ndarray:
    """k samples for every bin with wedges (Thm. cd-est), 0 for the rest."""
    return np.where(np.asarray(h_p_b, dtype=np.uint64) > 0, np.uint64(k),
                    np.uint64(0)).astype(np.uint64)


@dataclass
class SampleOut:
    q: torch.Tensor                  # int64 storage [(max_bins+1)*4]
    probe_loads: torch.Tensor
    dump: torch.Tensor | None        # int32 [(max_bins+1)*dump_per_bin, 4]
    h_k: np.ndarray
    k_global: int


def sample_close(g: Csr, bi: BinIndex, h_k: np.ndarray, k_global: int, seed: int,
                 graph_id: int = 0, dump_per_bin: int = 0, stream=None,
                 lanes_in_flight: int | None = None, samples_per_tile: int | None = None,
                 out: SampleOut | None = None) -> SampleOut:
    """wedge_sample_close (asynchronous)."""
    _require_gpu(g.rowptr, g.col, bi.index)
    dev = g.rowptr.device
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    assert hk.shape[0] == bi.max_bins
    rows = bi.max_bins + 1
    if out is None:
        q = torch.empty(rows * 4, dtype=torch.int64, device=dev)
        probe = torch.empty(1, dtype=torch.int64, device=dev)
        dump = (torch.zeros((rows * dump_per_bin, 4), dtype=torch.int32, device=dev)
                if dump_per_bin > 0 else None)
        out = SampleOut(q=q, probe_loads=probe, dump=dump, h_k=hk, k_global=k_global)
    else:
        out.h_k, out.k_global = hk, k_global
    hk_p = hk.ctypes.data_as(ctypes.c_void_p)
    if lanes_in_flight is None and samples_per_tile is None:
        rc = lib().wedge_sample_close(_ptr(g.rowptr), _ptr(g.col), g.n, g.m, _ptr(bi.index),
                                      bi.max_bins, hk_p, k_global, seed, graph_id, _ptr(out.q),
                                      _ptr(out.probe_loads), _ptr(out.dump), dump_per_bin,
                                      _stream(stream))
    else:
        rc = lib().wedge_sample_close_tuned(_ptr(g.rowptr), _ptr(g.col), g.n, g.m,
                                            _ptr(bi.index), bi.max_bins, hk_p, k_global, seed,
                                            graph_id, _ptr(out.q), _ptr(out.probe_loads),
                                            _ptr(out.dump), dump_per_bin,
                                            int(lanes_in_flight or 4),
                                            int(samples_per_tile or 4096), _stream(stream))
    _check(rc)
    return out


@dataclass
class EdgeHash:
    table: torch.Tensor   # int64[2^bits]
    bits: int
    full: torch.Tensor    # int64[1]: keys without an empty slot (expected 0)


def edge_hash(g: Csr, stream=None, table: torch.Tensor | None = None) -> EdgeHash:
    """wedge_edge_hash_build (asynchronous): the graph's edge table."""
    _require_gpu(g.rowptr, g.col)
    bits = int(lib().wedge_edge_hash_bits(g.m))
    if table is None or table.numel() < (1 << bits):
        table = torch.empty(1 << bits, dtype=torch.int64, device=g.rowptr.device)
    full = torch.empty(1, dtype=torch.int64, device=g.rowptr.device)
    _check(lib().wedge_edge_hash_build(_ptr(g.rowptr), _ptr(g.col), g.n, g.m, _ptr(table), bits,
                                       _ptr(full), _stream(stream)))
    return EdgeHash(table=table, bits=bits, full=full)


def sample_close_hashed(g: Csr, bi: BinIndex, h: EdgeHash, h_k: np.ndarray, k_global: int,
                        seed: int, graph_id: int = 0, dump_per_bin: int = 0, stream=None,
                        out: SampleOut | None = None) -> SampleOut:
    """wedge_sample_close_hashed (asynchronous)."""
    _require_gpu(g.rowptr, g.col, bi.index, h.table)
    dev = g.rowptr.device
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    assert hk.shape[0] == bi.max_bins
    rows = bi.max_bins + 1
    if out is None:
        q = torch.empty(rows * 4, dtype=torch.int64, device=dev)
        probe = torch.empty(1, dtype=torch.int64, device=dev)
        dump = (torch.zeros((rows * dump_per_bin, 4), dtype=torch.int32, device=dev)
                if dump_per_bin > 0 else None)
        out = SampleOut(q=q, probe_loads=probe, dump=dump, h_k=hk, k_global=k_global)
    _check(lib().wedge_sample_close_hashed(_ptr(g.rowptr), _ptr(g.col), g.n, g.m, _ptr(bi.index),
                                           bi.max_bins, hk.ctypes.data_as(ctypes.c_void_p),
                                           k_global, seed, graph_id, _ptr(out.q),
                                           _ptr(out.probe_loads), _ptr(out.dump), dump_per_bin,
                                           _ptr(h.table), h.bits, _stream(stream)))
    return out


def sample_close_autotune(g: Csr, bi: BinIndex, h_k: np.ndarray, k_global: int, seed: int,
                          cands: list, reps: int = 3, stream=None):
    """wedge_sample_close_autotune: (best shape, median ms per candidate); the
    pick is then used by wedge_sample_close for graphs of this size."""
    dev = g.rowptr.device
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    rows = bi.max_bins + 1
    q0 = torch.empty(rows * 4, dtype=torch.int64, device=dev)
    q1 = torch.empty(rows * 4, dtype=torch.int64, device=dev)
    arr = (LaunchShape * len(cands))(*cands)
    ms = (ctypes.c_float * len(cands))()
    best = ctypes.c_int(-1)
    _check(lib().wedge_sample_close_autotune(_ptr(g.rowptr), _ptr(g.col), g.n, g.m,
                                             _ptr(bi.index), bi.max_bins,
                                             hk.ctypes.data_as(ctypes.c_void_p), k_global, seed,
                                             arr, len(cands), reps, _ptr(q0), _ptr(q1), ms,
                                             ctypes.byref(best), _stream(stream)))
    return cands[best.value], list(ms)


def sample_close_shape(n: int, m: int, max_bins: int) -> LaunchShape:
    out = LaunchShape()
    _check(lib().wedge_sample_close_shape(n, m, max_bins, ctypes.byref(out)))
    return out


def sample_alloc(g: Csr, bi: BinIndex, h_k: np.ndarray, k_global: int, seed: int,
                 dump_per_bin: int = 0, ws: Workspace | None = None, stream=None):
    """wedge_sample_alloc (Alg. phase2a allocation, then per-vertex pairs).
    Synchronises; returns (SampleOut, totals[max_bins + 1]) with totals the
    realised samples per row."""
    _require_gpu(g.rowptr, g.col, bi.index)
    dev = g.rowptr.device
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    assert hk.shape[0] == bi.max_bins
    rows = bi.max_bins + 1
    q = torch.empty(rows * 4, dtype=torch.int64, device=dev)
    dump = (torch.zeros((rows * dump_per_bin, 4), dtype=torch.int32, device=dev)
            if dump_per_bin > 0 else None)
    tot = np.zeros(rows, dtype=np.uint64)
    need = int(lib().wedge_sample_alloc_workspace(g.n, bi.max_bins))
    wbuf = (ws or Workspace(dev)).get(need)
    _check(lib().wedge_sample_alloc(_ptr(g.rowptr), _ptr(g.col), g.n, g.m, _ptr(bi.index),
                                    bi.max_bins, hk.ctypes.data_as(_vp), k_global, seed,
                                    _ptr(q), tot.ctypes.data_as(_vp), _ptr(dump), dump_per_bin,
                                    _ptr(wbuf), wbuf.numel(), _stream(stream)))
    out = SampleOut(q=q, probe_loads=None, dump=dump, h_k=tot[:bi.max_bins].copy(),
                    k_global=int(tot[bi.max_bins]))
    return out, tot


def closure_join(a: torch.Tensor, c: torch.Tensor, h_src: torch.Tensor, h_dst: torch.Tensor,
                 chunk_edges: int = 0, ws: Workspace | None = None, stream=None) -> torch.Tensor:
    """wedge_closure_join: closure flags (uint8 device tensor) of the wedges
    (a, c) against the host edge list (h_src, h_dst: int32 CPU tensors,
    preferably pinned)."""
    _require_gpu(a, c)
    assert a.numel() == c.numel() and h_src.numel() == h_dst.numel()
    assert not h_src.is_cuda and not h_dst.is_cuda
    k = a.numel()
    closed = torch.empty(max(k, 1), dtype=torch.uint8, device=a.device)
    need = int(lib().wedge_closure_join_workspace(k, chunk_edges))
    wbuf = (ws or Workspace(a.device)).get(need)
    _check(lib().wedge_closure_join(_ptr(a), _ptr(c), k, _vp(h_src.data_ptr()),
                                    _vp(h_dst.data_ptr()), h_src.numel(), chunk_edges,
                                    _ptr(closed), _ptr(wbuf), wbuf.numel(), _stream(stream)))
    return closed[:k]


@dataclass
class StreamOut:
    bins: BinIndex        # n_b, p_b (device and host); index is None (kept inside)
    q: torch.Tensor       # int64[(max_bins + 1) * 4]
    dump: torch.Tensor | None
    h_k: np.ndarray       # samples per bin actually drawn (0 where p_b = 0)
    k_global: int
    m: int                # edges counted
    rejected: int         # edges with an id >= n
    rounds: int           # gather rounds
    gathered: int         # edge ends gathered


def sample_stream(h_src: torch.Tensor, h_dst: torch.Tensor, n: int, h_k: np.ndarray,
                  k_global: int, seed: int, tau: int = 2, omega: int = 2, max_bins: int = 64,
                  gather_cap: int | None = None, chunk_edges: int = 0, dump_per_bin: int = 0,
                  device=None, ws: Workspace | None = None, stream=None) -> StreamOut:
    """wedge_sample_stream: bins, samples and closure tests of a simple edge
    list held in host memory (h_src, h_dst: int32 CPU tensors, preferably
    pinned); no adjacency is built on the device.  Synchronises the stream.
    gather_cap defaults to every edge end (one gather round)."""
    _require_gpu()
    assert not h_src.is_cuda and not h_dst.is_cuda and h_src.numel() == h_dst.numel()
    dev = torch.device(device if device is not None else "cuda")
    m_in = h_src.numel()
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    assert hk.shape[0] == max_bins
    cap = int(gather_cap) if gather_cap else max(2 * m_in, 1)
    rows = max_bins + 1
    n_b = torch.empty(max_bins, dtype=torch.int64, device=dev)
    p_b = torch.empty(max_bins, dtype=torch.int64, device=dev)
    q = torch.empty(rows * 4, dtype=torch.int64, device=dev)
    dump = (torch.zeros((rows * dump_per_bin, 4), dtype=torch.int32, device=dev)
            if dump_per_bin > 0 else None)
    hk_p = hk.ctypes.data_as(ctypes.c_void_p)
    need = int(lib().wedge_sample_stream_workspace(n, m_in, max_bins, hk_p, k_global, cap,
                                                  chunk_edges))
    wbuf = (ws or Workspace(dev)).get(need)
    info = np.zeros(4, dtype=np.uint64)
    _check(lib().wedge_sample_stream(_vp(h_src.data_ptr()), _vp(h_dst.data_ptr()), m_in, n, tau,
                                     omega, max_bins, hk_p, k_global, seed, cap, chunk_edges,
                                     _ptr(n_b), _ptr(p_b), _ptr(q), _ptr(dump), dump_per_bin,
                                     info.ctypes.data_as(ctypes.c_void_p), _ptr(wbuf),
                                     wbuf.numel(), _stream(stream)))
    h_p_b = p_b.cpu().numpy().astype(np.uint64)
    bi = BinIndex(n=n, m=int(info[0]), tau=tau, omega=omega, max_bins=max_bins, n_b=n_b, p_b=p_b,
                  index=None, h_n_b=n_b.cpu().numpy().astype(np.uint64), h_p_b=h_p_b)
    drawn = np.where(h_p_b > 0, hk, 0).astype(np.uint64)
    kg = int(k_global) if int(h_p_b.sum()) > 0 else 0
    return StreamOut(bins=bi, q=q, dump=dump, h_k=drawn, k_global=kg, m=int(info[0]),
                     rejected=int(info[1]), rounds=int(info[2]), gathered=int(info[3]))


@dataclass
class Estimates:
    bins: list = field(default_factory=list)     # per bin: dict
    glob: dict = field(default_factory=dict)
    q: np.ndarray | None = None


def estimate(bi: BinIndex, q: np.ndarray, h_k: np.ndarray, k_global: int,
             delta: float) -> Estimates:
    """wedge_estimate (host FP64 inside the library)."""
    B = bi.max_bins
    qq = np.ascontiguousarray(q, dtype=np.uint64).reshape(-1)
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    nb = np.ascontiguousarray(bi.h_n_b, dtype=np.uint64)
    pb = np.ascontiguousarray(bi.h_p_b, dtype=np.uint64)
    eb = (WedgeBinEstimate * B)()
    eg = WedgeGlobalEstimate()
    _check(lib().wedge_estimate(nb.ctypes.data_as(_vp), pb.ctypes.data_as(_vp),
                                qq.ctypes.data_as(_vp), hk.ctypes.data_as(_vp), B, bi.tau,
                                bi.omega, k_global, delta, ctypes.cast(eb, _vp),
                                ctypes.byref(eg)))
    out = Estimates(q=qq.reshape(B + 1, 4))
    for e in eb:
        out.bins.append({"bin": e.bin, "valid": e.valid, "lo_deg": e.lo_deg, "n_b": e.n_b,
                         "p_b": e.p_b, "k_b": e.k_b, "q": list(e.q), "c": e.c, "t": e.t,
                         "eps": e.eps})
    out.glob = {"p": eg.p, "k_global": eg.k_global, "q_global": list(eg.q_global), "c": eg.c,
                "t": eg.t, "c_global": eg.c_global, "t_global": eg.t_global,
                "eps_global": eg.eps_global, "t_bins_sum": eg.t_bins_sum}
    return out


@dataclass
class PlainResult:
    csr: Csr
    bins: BinIndex
    samples: SampleOut
    est: Estimates


def run_plain(src: torch.Tensor, dst: torch.Tensor, n: int, *, tau: int = 2, omega: int = 2,
              max_bins: int = 64, k: int | None = None, k_global: int | None = None,
              eps: float = 1e-3, delta: float = 1e-3, seed: int = 1, graph_id: int = 0,
              dump_per_bin: int = 0, ws: Workspace | None = None, stream=None) -> PlainResult:
    """The whole plain path: build_csr -> bin_counts -> sample_close -> estimate.
    k (per bin) and k_global default to the Hoeffding size for (eps, delta)."""
    ws = ws or Workspace(src.device)
    kk = hoeffding_k(eps, delta) if k is None else int(k)
    kg = kk if k_global is None else int(k_global)
    g = build_csr(src, dst, n, ws=ws, stream=stream)
    bi = bin_counts(g, tau, omega, max_bins, ws=ws, stream=stream)
    hk = k_for_bins(bi.h_p_b, kk)
    if int(bi.h_p_b.sum()) == 0:
        kg = 0   # no wedges at all: nothing for the global stream to draw
    so = sample_close(g, bi, hk, kg, seed, graph_id=graph_id, dump_per_bin=dump_per_bin,
                      stream=stream)
    q = to_host_u64(so.q)
    est = estimate(bi, q, hk, kg, delta)
    return PlainResult(csr=g, bins=bi, samples=so, est=est)


# ------------------------------------------------------------------ batches
def make_shape(lanes: int = 4, spt: int = 4096, workgroups: int = 0) -> LaunchShape:
    return LaunchShape(int(lanes), int(spt), int(workgroups))


class Batch:
    """A batch of graphs on the device (wedge_batch_*).

    graphs: list of (n_g, src, dst) with local uint32 ids.  Results of graph
    g equal the single-graph path on graph g with graph_id = g."""

    def __init__(self, graphs, *, tau: int = 2, omega: int = 2, max_bins: int = 40,
                 k_per_bin: int = 20_000, k_global: int | None = None, seed: int = 1,
                 device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("libwedge needs a GPU (no CPU fallback)")
        dev = torch.device(device)
        self.G = len(graphs)
        ns = [int(g[0]) for g in graphs]
        ms = [len(g[1]) for g in graphs]
        self.n_g = np.array(ns, dtype=np.uint64)
        self.voff = np.concatenate([[0], np.cumsum(ns)]).astype(np.uint64)
        self.eoff = np.concatenate([[0], np.cumsum(ms)]).astype(np.uint64)
        src = np.concatenate([np.asarray(g[1], dtype=np.uint32) for g in graphs]) if sum(ms) else \
            np.zeros(1, np.uint32)
        dst = np.concatenate([np.asarray(g[2], dtype=np.uint32) for g in graphs]) if sum(ms) else \
            np.zeros(1, np.uint32)
        self.desc = BatchDesc(self.G, max_bins, tau, max(ns), omega, k_per_bin,
                              k_per_bin if k_global is None else k_global, seed, int(sum(ms)),
                              int(sum(ns)))
        self.B = max_bins
        self.tau, self.omega = tau, omega
        self.d_src = torch.from_numpy(src.view(np.int32)).to(dev)
        self.d_dst = torch.from_numpy(dst.view(np.int32)).to(dev)
        self.d_eoff = torch.from_numpy(self.eoff.view(np.int64)).to(dev)
        self.d_voff = torch.from_numpy(self.voff.astype(np.uint32).view(np.int32)).to(dev)
        nbytes = int(lib().wedge_batch_workspace_bytes(ctypes.byref(self.desc)))
        if nbytes == 0:
            _check(-2)
        self.ws = _empty_bytes(nbytes, dev)
        rows = self.G * (max_bins + 1)
        self.n_b = torch.zeros(self.G * max_bins, dtype=torch.int64, device=dev)
        self.p_b = torch.zeros(self.G * max_bins, dtype=torch.int64, device=dev)
        self.q = torch.zeros(rows * 4, dtype=torch.int64, device=dev)
        self.q_try = torch.zeros(rows * 4, dtype=torch.int64, device=dev)
        self.probe = torch.zeros(1, dtype=torch.int64, device=dev)
        self.est_glob = torch.zeros(self.G * 6, dtype=torch.float64, device=dev)
        self.est_bins = torch.zeros(self.G * max_bins * 3, dtype=torch.float64, device=dev)
        self.graph = None

    def _shape(self, shape):
        return None if shape is None else ctypes.byref(shape)

    def prepare(self, stream=None):
        _check(lib().wedge_batch_prepare(ctypes.byref(self.desc), _ptr(self.d_src),
                                         _ptr(self.d_dst), _ptr(self.d_eoff), _ptr(self.d_voff),
                                         _ptr(self.n_b), _ptr(self.p_b), _ptr(self.ws),
                                         self.ws.numel(), _stream(stream)))

    def sample(self, shape: LaunchShape | None = None, delta: float = 1e-3, stream=None,
               probe: bool = False):
        _check(lib().wedge_batch_sample(ctypes.byref(self.desc), self._shape(shape), delta,
                                        _ptr(self.q), _ptr(self.probe) if probe else None,
                                        _ptr(self.est_glob), _ptr(self.est_bins), _ptr(self.ws),
                                        self.ws.numel(), _stream(stream)))

    def run(self, shape: LaunchShape | None = None, delta: float = 1e-3, stream=None):
        _check(lib().wedge_batch_run(ctypes.byref(self.desc), _ptr(self.d_src), _ptr(self.d_dst),
                                     _ptr(self.d_eoff), _ptr(self.d_voff), self._shape(shape),
                                     delta, _ptr(self.n_b), _ptr(self.p_b), _ptr(self.q),
                                     _ptr(self.est_glob), _ptr(self.est_bins), _ptr(self.ws),
                                     self.ws.numel(), _stream(stream)))

    def capture(self, shape: LaunchShape | None = None, delta: float = 1e-3):
        """Capture the whole batch pipeline into a HIP graph."""
        self.destroy_graph()
        h = ctypes.c_void_p()
        _check(lib().wedge_batch_graph_create(ctypes.byref(self.desc), _ptr(self.d_src),
                                              _ptr(self.d_dst), _ptr(self.d_eoff),
                                              _ptr(self.d_voff), self._shape(shape), delta,
                                              _ptr(self.n_b), _ptr(self.p_b), _ptr(self.q),
                                              _ptr(self.est_glob), _ptr(self.est_bins),
                                              _ptr(self.ws), self.ws.numel(), ctypes.byref(h)))
        self.graph = h

    def replay(self, stream=None):
        _check(lib().wedge_batch_graph_launch(self.graph, _stream(stream)))

    def destroy_graph(self):
        if self.graph is not None:
            lib().wedge_batch_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.destroy_graph()
        except Exception:
            pass

    def autotune(self, cands: list[LaunchShape], reps: int = 3, stream=None):
        """Time each candidate shape on the prepared batch; returns
        (best shape, median ms per candidate).  Raises if any candidate's
        counts differ from the first's."""
        arr = (LaunchShape * len(cands))(*cands)
        ms = (ctypes.c_float * len(cands))()
        best = ctypes.c_int(-1)
        _check(lib().wedge_batch_autotune(ctypes.byref(self.desc), arr, len(cands), reps,
                                          _ptr(self.q), _ptr(self.q_try), _ptr(self.ws),
                                          self.ws.numel(), ms, ctypes.byref(best),
                                          _stream(stream)))
        return cands[best.value], list(ms)

    def host(self):
        """Host copies: n_b, p_b [G, B]; q [G, B+1, 4]; est_glob [G, 6];
        est_bins [G, B, 3]."""
        G, B = self.G, self.B
        return dict(n_b=to_host_u64(self.n_b).reshape(G, B),
                    p_b=to_host_u64(self.p_b).reshape(G, B),
                    q=to_host_u64(self.q).reshape(G, B + 1, 4),
                    est_glob=self.est_glob.cpu().numpy().reshape(G, 6),
                    est_bins=self.est_bins.cpu().numpy().reshape(G, B, 3))

    def csr_of(self, g: int):
        """Row offsets and adjacency of graph g in local ids (from the
        workspace: rowptr is its first region, col the second)."""
        n_tot = int(self.voff[-1])
        rp_all = self.ws[: 8 * (n_tot + 1)].view(torch.int64)
        off = (8 * (n_tot + 1) + 255) // 256 * 256
        col_all = self.ws[off: off + 4 * 2 * max(int(self.eoff[-1]), 1)].view(torch.int32)
        v0, v1 = int(self.voff[g]), int(self.voff[g + 1])
        rp = rp_all[v0: v1 + 1].cpu().numpy().view(np.uint64).copy()
        col = col_all[int(rp[0]): int(rp[-1])].cpu().numpy().view(np.uint32).copy() - v0
        return rp - rp[0], col
