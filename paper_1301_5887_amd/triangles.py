"""Triangle sample and degree assortativity (wedge_triangle_stats,
wedge_triangle_box): the closed wedges of the global stream's uniform wedge
sample are uniform triangles; their sorted degrees are grouped by the bin of
the smallest degree, and the bin of the largest degree is summarised per
group as in the paper's box plots (Sec. 5)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import cv as C
from . import wedge as W

TRIANGLE_DTYPE = np.dtype([("d_min", "<u4"), ("d_mid", "<u4"), ("d_max", "<u4"),
                           ("sample", "<u4")])


@dataclass
class TriangleSample:
    k: int                  # wedges drawn
    count: int              # closed ones = sampled triangles
    triangles: np.ndarray | None   # TRIANGLE_DTYPE[count]
    hist: np.ndarray        # [max_bins, max_bins] by (BinId(d_min), BinId(d_max))
    box: list               # per min bin: dict of the box statistics (count 0 omitted)


def stats(rec: torch.Tensor, k: int, tau: int = 2, omega: int = 2, max_bins: int = 64,
          keep_triangles: bool = True, stream=None):
    """wedge_triangle_stats on k feature records; returns device tensors
    (triangles or None, count[1], hist[max_bins * max_bins])."""
    dev = rec.device
    tri = (torch.empty(max(k, 1) * 4, dtype=torch.int32, device=dev) if keep_triangles
           else None)
    count = torch.empty(1, dtype=torch.int64, device=dev)
    hist = torch.empty(max_bins * max_bins, dtype=torch.int64, device=dev)
    ws = W._empty_bytes(int(W.lib().wedge_triangle_stats_workspace(k)), dev)
    W._check(W.lib().wedge_triangle_stats(W._ptr(rec), k, tau, omega, max_bins, W._ptr(tri),
                                          W._ptr(count), W._ptr(hist), W._ptr(ws), ws.numel(),
                                          W._stream(stream)))
    return tri, count, hist


def box(hist: np.ndarray) -> list:
    """wedge_triangle_box on a host histogram [max_bins, max_bins]."""
    B = hist.shape[0]
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    rows = (W.WedgeTriangleBoxRow * B)()
    W._check(W.lib().wedge_triangle_box(h.ctypes.data_as(W._vp), B, rows))
    out = []
    for b in range(B):
        r = rows[b]
        if r.count:
            out.append({"min_bin": b, "count": int(r.count), "q1": r.q1, "median": r.median,
                        "q3": r.q3, "whisker_lo": r.whisker_lo, "whisker_hi": r.whisker_hi,
                        "outliers": int(r.outliers)})
    return out


def sample(g: W.Csr, bi: W.BinIndex, k: int, seed: int, tau: int = 2, omega: int = 2,
           max_bins: int = 64, keep_triangles: bool = True, stream=None) -> TriangleSample:
    """k wedges of the global stream (the samples wedge_sample_close draws
    for it with this seed), their triangles and the assortativity summary."""
    B = bi.max_bins
    hk = np.zeros(B + 1, dtype=np.uint64)
    hk[B] = k
    rec = C.new_records(1, k, g.rowptr.device)
    C.sample_features(g, bi, hk, 0, seed, C.DOMAIN_SAMPLE, True, rec, k, stream=stream)
    tri, count, hist = stats(rec, k, tau, omega, max_bins, keep_triangles, stream)
    n = int(W.to_host_u64(count)[0])
    h = W.to_host_u64(hist).reshape(max_bins, max_bins)
    t = None
    if tri is not None:
        t = tri[: 4 * n].cpu().numpy().view(np.uint8).view(TRIANGLE_DTYPE).copy()
    return TriangleSample(k=k, count=n, triangles=t, hist=h, box=box(h))
