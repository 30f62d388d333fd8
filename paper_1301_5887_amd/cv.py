"""Learned control variate for wedge sampling (binding + driver).

For every bin b (and the global stream) the closed fraction c_b of Thm.
cd-est is estimated by
    c_CV = mean_EVAL(X - beta_b g) + beta_b mu_g
where X is the exact closure label of a uniform wedge of the bin, g in (0,1)
is the network's closure probability from the wedge's degrees, beta_b is fixed
from held-out TRAIN draws before any EVAL draw, and the TRAIN, EVAL, AUX and
centre draws use distinct Philox key domains, so c_CV is unbiased whatever the
network learned.  mu_g, the mean of g over the bin's wedges, comes in one of
three forms:
  exact    from the census of (bin, centre bucket, endpoint bucket pair)
           counts (the network depends on the wedge only through them);
  centre   from centre draws: v with probability p_v / p_b and gbar(v), the
           mean of g over all wedges at v (E[gbar] = mu_g);
  AUX      from uniform wedge draws without a closure test.
Draws come in rounds whose sizes are fixed before any EVAL draw (first round
from the held-out draws, then growing by a constant factor); after round i
the two-sided empirical-Bernstein half-width at delta_i = delta / (i (i+1))
(a union bound over rounds) is checked against eps: EB(n, var(X - beta g),
1 + |beta|) at delta_i for the exact form, plus |beta| EB of the mean of
gbar (or of g) with delta_i split in two for the centre (AUX) form.
beta = 0 is plain wedge sampling with the same rule ("plain-EB").  All work
runs in libwedge: the sampler in feature mode, the network's forward,
gradient and Adam kernels, the census, the centre draws, the integer moment
sums, and the estimator itself (wedge_cv_fit, wedge_cv_estimate,
wedge_cv_bin_means, wedge_cv_plan_centre, wedge_cv_train); this module only
marshals arguments and sequences the calls.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import wedge as W

FEATURE_DTYPE = np.dtype([("dv", "<u4"), ("dlo", "<u4"), ("dhi", "<u4"), ("bin", "<u2"),
                          ("closed", "u1"), ("cls", "u1")])
NPARAM = 4545
DOMAIN_SAMPLE, DOMAIN_TRAIN, DOMAIN_AUX, DOMAIN_EVAL, DOMAIN_CENTRE = 1, 2, 3, 4, 6


def _L():
    return W.lib()


def eb_halfwidth(n: int, var: float, R: float, delta: float) -> float:
    return float(_L().wedge_eb_halfwidth(int(n), float(max(var, 0.0)), float(R), float(delta)))


def records_to_numpy(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint8).reshape(-1).view(FEATURE_DTYPE)


def sample_features(g: W.Csr, bi: W.BinIndex, h_k: np.ndarray, s_begin, seed: int,
                    domain: int, closure: bool, out: torch.Tensor, stride: int,
                    graph_id: int = 0, stream=None):
    """wedge_sample_features into out (int32 tensor viewed as records);
    s_begin is one first sample index for every row or an array of them."""
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    assert hk.shape[0] == bi.max_bins + 1
    sb = np.zeros(bi.max_bins + 1, dtype=np.uint64)
    sb[:] = np.asarray(s_begin, dtype=np.uint64)
    W._check(_L().wedge_sample_features(W._ptr(g.rowptr), W._ptr(g.col), g.n, g.m,
                                        W._ptr(bi.index), bi.max_bins, bi.tau, bi.omega,
                                        hk.ctypes.data_as(W._vp), sb.ctypes.data_as(W._vp),
                                        seed, domain, graph_id,
                                        int(closure), W._ptr(out), stride, None,
                                        W._stream(stream)))


def new_records(rows: int, stride: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(rows * stride, 1) * 4, dtype=torch.int32, device=device)


class _RoundBuffers:
    """Device buffers of the training draws and of the sequential rounds,
    kept between rounds and calls (grown, never shrunk, held until the process
    ends), so that a timed round allocates no device memory once a first call
    has sized them.  Calls that use them must not overlap (one stream)."""

    def __init__(self):
        self._bufs = {}

    def take(self, name: str, n: int, dtype, device) -> torch.Tensor:
        key = (name, str(torch.device(device)), dtype)
        n = max(int(n), 1)
        b = self._bufs.get(key)
        if b is None or b.numel() < n:
            b = torch.empty(n, dtype=dtype, device=device)
            self._bufs[key] = b
        return b[:n]

    def records(self, name: str, rows: int, stride: int, device) -> torch.Tensor:
        return self.take(name, max(rows * stride, 1) * 4, torch.int32, device)


_ROUND_BUFFERS = _RoundBuffers()


class Mlp:
    """Network state on the device (wedge_mlp_*)."""

    def __init__(self, device="cuda"):
        self.state = W._empty_bytes(int(_L().wedge_mlp_state_bytes()), torch.device(device))
        self.grad = torch.zeros(NPARAM, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = W.Workspace(device)
        self.t = 0

    def init(self, seed: int, stream=None):
        W._check(_L().wedge_mlp_init(W._ptr(self.state), seed, W._stream(stream)))
        self.t = 0

    def set(self, params: torch.Tensor, stream=None):
        assert params.dtype == torch.float32 and params.numel() == NPARAM and params.is_cuda
        W._check(_L().wedge_mlp_set(W._ptr(self.state), W._ptr(params), W._stream(stream)))
        self.t = 0

    def get(self, stream=None) -> torch.Tensor:
        out = torch.empty(NPARAM, dtype=torch.float32, device=self.state.device)
        W._check(_L().wedge_mlp_get(W._ptr(self.state), W._ptr(out), W._stream(stream)))
        return out

    def forward(self, rec: torch.Tensor, n: int, out: torch.Tensor, stream=None):
        W._check(_L().wedge_mlp_forward(W._ptr(self.state), W._ptr(rec), n, W._ptr(out),
                                        W._stream(stream)))

    def grad_of(self, rec: torch.Tensor, rows: int, stride: int, j0: int, per_row: int,
                stream=None):
        n = rows * per_row
        ws = self.ws.get(int(_L().wedge_mlp_grad_workspace(n)))
        W._check(_L().wedge_mlp_grad(W._ptr(self.state), W._ptr(rec), rows, stride, j0, per_row,
                                     W._ptr(self.grad), W._ptr(self.loss), W._ptr(ws),
                                     ws.numel(), W._stream(stream)))

    def train(self, rec: torch.Tensor, rows: int, stride: int, n_fit: int, per_row_batch: int,
              epochs: int, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        """wedge_mlp_train: every minibatch step queued by the library."""
        ws = self.ws.get(int(_L().wedge_mlp_train_workspace(rows, per_row_batch)))
        W._check(_L().wedge_mlp_train(W._ptr(self.state), W._ptr(rec), rows, stride, n_fit,
                                      per_row_batch, epochs, self.t, lr, b1, b2, eps,
                                      W._ptr(self.loss), W._ptr(ws), ws.numel(),
                                      W._stream(stream)))
        self.t += epochs * (n_fit // per_row_batch)

    def adam(self, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8, grad: torch.Tensor | None = None,
             stream=None):
        self.t += 1
        g = self.grad if grad is None else grad
        W._check(_L().wedge_mlp_adam(W._ptr(self.state), W._ptr(g), self.t, lr, b1, b2, eps,
                                     W._stream(stream)))


def moments(rec: torch.Tensor, gv: torch.Tensor, rows: int, stride: int, per_row: int,
            out: torch.Tensor | None = None, counts=None, stream=None) -> torch.Tensor:
    """Integer moment sums [rows, 5] (count, sum X, 2^32 sum g, 2^32 sum g^2,
    2^32 sum X g), accumulated into `out`; `counts` (per row) overrides
    per_row.  rec=None takes X = 0 (moments of g alone)."""
    if out is None:
        out = torch.zeros(rows * 5, dtype=torch.int64, device=gv.device)
    cp = None
    if counts is not None:
        ca = np.ascontiguousarray(counts, dtype=np.uint64)
        cp = ca.ctypes.data_as(W._vp)
    W._check(_L().wedge_cv_moments(W._ptr(rec), W._ptr(gv), rows, stride, per_row, cp,
                                   W._ptr(out), W._stream(stream)))
    return out


KPAIRS = 256 * 257 // 2


class Census:
    """wedge_cv_census of a graph and the exact means it yields."""

    def __init__(self, g: W.Csr, bi: W.BinIndex, stream=None):
        dev = g.rowptr.device
        self.bi = bi
        self.buf = W._empty_bytes(int(_L().wedge_cv_census_bytes(g.n, g.m, bi.max_bins)), dev)
        W._check(_L().wedge_cv_census(W._ptr(g.rowptr), W._ptr(g.col), g.n, g.m,
                                      W._ptr(bi.index), bi.max_bins, bi.tau, bi.omega,
                                      W._ptr(self.buf), self.buf.numel(), W._stream(stream)))
        cap = 256 + bi.max_bins + 1
        nk = ctypes.c_uint32(0)
        kb = np.zeros(cap, dtype=np.uint32)
        kk = np.zeros(cap, dtype=np.uint32)
        W._check(_L().wedge_cv_census_keys(W._ptr(self.buf), bi.max_bins, ctypes.byref(nk),
                                           kb.ctypes.data_as(W._vp), kk.ctypes.data_as(W._vp),
                                           W._stream(stream)))
        self.nkeys = nk.value
        self.key_bin = kb[: self.nkeys].copy()
        self.key_bucket = kk[: self.nkeys].copy()

    def table(self) -> np.ndarray:
        """[nkeys, 32896] wedge counts (host copy)."""
        off = _table_offset(self.bi.max_bins)
        t = self.buf[off: off + 8 * self.nkeys * KPAIRS].view(torch.int64)
        return t.cpu().numpy().view(np.uint64).reshape(self.nkeys, KPAIRS)

    def means(self, net: "Mlp", stream=None) -> dict:
        """Exact mean of g over the wedges of every bin (and 'global')."""
        dev = self.buf.device
        cap = 256 + self.bi.max_bins + 1
        ws = W._empty_bytes(int(_L().wedge_cv_exact_mean_workspace(self.bi.max_bins)), dev)
        ksum = torch.zeros(cap, dtype=torch.float64, device=dev)
        kcnt = torch.zeros(cap, dtype=torch.int64, device=dev)
        W._check(_L().wedge_cv_exact_mean(W._ptr(net.state), W._ptr(self.buf), self.bi.max_bins,
                                          W._ptr(ksum), W._ptr(kcnt), W._ptr(ws), ws.numel(),
                                          W._stream(stream)))
        s = np.ascontiguousarray(ksum.cpu().numpy()[: self.nkeys])
        c = np.ascontiguousarray(W.to_host_u64(kcnt)[: self.nkeys])
        B = self.bi.max_bins
        mean = np.zeros(B + 1, dtype=np.float64)
        den = np.zeros(B + 1, dtype=np.uint64)
        kb = np.ascontiguousarray(self.key_bin, dtype=np.uint32)
        W._check(_L().wedge_cv_bin_means(s.ctypes.data_as(W._vp), c.ctypes.data_as(W._vp),
                                         kb.ctypes.data_as(W._vp), self.nkeys, B,
                                         mean.ctypes.data_as(W._vp), den.ctypes.data_as(W._vp)))
        out = {b: float(mean[b]) for b in range(B) if den[b] > 0}
        out[B] = float(mean[B])
        self.counts = den[:B]
        return out


class CentreTable:
    """The network's g for every (bin, centre bucket) key and endpoint bucket
    pair (wedge_cv_keys + wedge_cv_gtable), for the centre draws."""

    def __init__(self, g: W.Csr, bi: W.BinIndex, net: "Mlp", stream=None):
        dev = g.rowptr.device
        self.bi = bi
        self.keys = W._empty_bytes(int(_L().wedge_cv_census_bytes(g.n, g.m, bi.max_bins)), dev)
        W._check(_L().wedge_cv_keys(W._ptr(self.keys), bi.max_bins, bi.tau, bi.omega,
                                    W._stream(stream)))
        cap = 256 + bi.max_bins + 1
        self.gtable = torch.empty(cap * KPAIRS, dtype=torch.float32, device=dev)
        ws = W._empty_bytes(int(_L().wedge_cv_gtable_workspace(bi.max_bins)), dev)
        W._check(_L().wedge_cv_gtable(W._ptr(net.state), W._ptr(self.keys), bi.max_bins,
                                      W._ptr(self.gtable), W._ptr(ws), ws.numel(),
                                      W._stream(stream)))


def centre_means(g: W.Csr, bi: W.BinIndex, table: CentreTable, h_k, s_begin, seed: int,
                 domain: int, out: torch.Tensor, stride: int, vout: torch.Tensor | None = None,
                 stream=None):
    """wedge_cv_centre_means into out (float32 [rows][stride])."""
    hk = np.ascontiguousarray(h_k, dtype=np.uint64)
    sb = np.zeros(bi.max_bins + 1, dtype=np.uint64)
    sb[:] = np.asarray(s_begin, dtype=np.uint64)
    ws = W._empty_bytes(int(_L().wedge_cv_centre_means_workspace(int(hk.sum()))),
                        g.rowptr.device)
    W._check(_L().wedge_cv_centre_means(W._ptr(g.rowptr), W._ptr(g.col), g.n, g.m,
                                        W._ptr(bi.index), bi.max_bins, bi.tau, bi.omega,
                                        hk.ctypes.data_as(W._vp), sb.ctypes.data_as(W._vp),
                                        seed, domain, 0, W._ptr(table.keys),
                                        W._ptr(table.gtable), W._ptr(out), stride,
                                        W._ptr(vout) if vout is not None else None, W._ptr(ws),
                                        ws.numel(), W._stream(stream)))


def _table_offset(max_bins: int) -> int:
    cap = 256 + max_bins + 1
    r = lambda x: (x + 255) // 256 * 256  # noqa: E731
    return r(8) + r(max_bins * 256 * 4) + 3 * r(cap * 4)


def fit_rows(mom: np.ndarray, eps: float, delta: float):
    """wedge_cv_fit over moments [rows, 5]: per row (beta, rho^2, var_x,
    var_z, first-round plan plain, plan control variate)."""
    m = np.ascontiguousarray(mom, dtype=np.int64)
    R = m.shape[0]
    out = (W.CvFitRow * max(R, 1))()
    W._check(_L().wedge_cv_fit(m.ctypes.data_as(W._vp), R, eps, delta, out))
    return [out[i] for i in range(R)]


def estimate_rows(rows: list, round_i: int, delta: float, eps: float, max_per_row: int):
    """wedge_cv_estimate over a list of W.CvRow: [(estimate, half-width, more)]."""
    arr = (W.CvRow * max(len(rows), 1))(*rows)
    out = (W.CvResult * max(len(rows), 1))()
    W._check(_L().wedge_cv_estimate(arr, len(rows), round_i, delta, eps, max_per_row, out))
    return [(out[i].estimate, out[i].halfwidth, bool(out[i].more)) for i in range(len(rows))]


def mean_var_rows(mom: np.ndarray):
    """wedge_cv_mean_var over moments [rows, 5] of values without labels."""
    m = np.ascontiguousarray(mom, dtype=np.int64)
    R = m.shape[0]
    mean = np.zeros(max(R, 1))
    var = np.zeros(max(R, 1))
    W._check(_L().wedge_cv_mean_var(m.ctypes.data_as(W._vp), R, mean.ctypes.data_as(W._vp),
                                    var.ctypes.data_as(W._vp)))
    return mean[:R], var[:R]


@dataclass
class SequentialResult:
    estimates: dict = field(default_factory=dict)     # row -> estimate
    halfwidth: dict = field(default_factory=dict)
    eval_samples: dict = field(default_factory=dict)
    aux_samples: dict = field(default_factory=dict)
    rounds: int = 0
    seconds: float = 0.0

    @property
    def total_eval(self) -> int:
        return int(sum(self.eval_samples.values()))

    @property
    def total_aux(self) -> int:
        return int(sum(self.aux_samples.values()))


def _moments_per_row(recs, gv, counts, stride, dev):
    """Moments of the first counts[j] records of every row j."""
    A = len(counts)
    mom = moments(recs, gv, A, stride, 0, counts=counts)
    return W.to_host_u64(mom).view(np.int64).reshape(A, 5)


def sequential(g: W.Csr, bi: W.BinIndex, rows: list[int], eps: float, delta: float, seed: int,
               net: Mlp | None, beta: dict | None, n0: int = 1 << 14,
               max_per_row: int = 1 << 26, exact_means: dict | None = None,
               first: dict | None = None, growth: float = 2.0,
               centre: CentreTable | None = None, centre_first: dict | None = None,
               stream=None) -> SequentialResult:
    """EVAL (and, with a network and no exact means, AUX) draws in rounds:
    row r's running total after round i is first[r] * growth^(i-1) (n0 for
    every row without a plan), until every row's half-width at
    delta_i = delta / (i (i+1)) is <= eps.  The plan must not depend on the
    EVAL draws (a pilot from TRAIN draws, or a constant).  With a centre
    table, rows with beta != 0 take the control variate's mean from centre
    draws instead, centre_first[r] * growth^(i-1) of them after round i."""
    dev = g.rowptr.device
    B = bi.max_bins
    rows = sorted(rows)
    t0 = time.perf_counter()
    res = SequentialResult()
    mode = W.CV_PLAIN
    if net is not None:
        mode = (W.CV_CENTRE if centre is not None else
                W.CV_EXACT if exact_means is not None else W.CV_AUX)
    stats = {r: W.CvRow(beta=(beta or {}).get(r, 0.0) if net is not None else 0.0,
                        exact_mean=(exact_means or {}).get(r, 0.0), mode=mode) for r in rows}
    done = {r: 0 for r in rows}
    cdone = {r: 0 for r in rows}
    use_centre = centre is not None and net is not None
    active = list(rows)
    i = 0
    while active:
        i += 1
        hk = np.zeros(B + 1, dtype=np.uint64)
        sb = np.zeros(B + 1, dtype=np.uint64)
        incs = []
        for r in active:
            base = first.get(r, n0) if first else n0
            target = int(_L().wedge_cv_round_size(int(base), growth, i, max_per_row))
            inc = max(target - done[r], 0)
            hk[r], sb[r] = inc, done[r]
            incs.append(inc)
        if max(incs) == 0:
            break
        A = len(active)   # records are compact: row j is active[j]
        stride = max(incs)
        recs = _ROUND_BUFFERS.records("eval", A, stride, dev)
        sample_features(g, bi, hk, sb, seed, DOMAIN_EVAL, True, recs, stride, stream=stream)
        gv = _ROUND_BUFFERS.take("eval_g", A * stride, torch.float32, dev)
        # g only matters on rows whose beta is not 0 (plain rows use X alone);
        # the forward writes every entry, otherwise g is 0
        if net is not None and any((beta or {}).get(r, 0.0) != 0.0 for r in active):
            net.forward(recs, A * stride, gv, stream=stream)
        else:
            gv.zero_()
        m = _moments_per_row(recs, gv, incs, stride, dev)
        am = None
        cm, crow = None, []
        if use_centre:
            hc = np.zeros(B + 1, dtype=np.uint64)
            sc = np.zeros(B + 1, dtype=np.uint64)
            for r in active:
                if beta.get(r, 0.0) == 0.0:
                    continue
                target = int(_L().wedge_cv_round_size(int(centre_first[r]), growth, i,
                                                       max_per_row))
                if target > cdone[r]:
                    hc[r], sc[r] = target - cdone[r], cdone[r]
                    crow.append(r)
            if crow:
                cinc = [int(hc[r]) for r in crow]
                cstride = max(cinc)
                cout = _ROUND_BUFFERS.take("centre", len(crow) * cstride, torch.float32, dev)
                centre_means(g, bi, centre, hc, sc, seed, DOMAIN_CENTRE, cout, cstride,
                             stream=stream)
                cm = _moments_per_row(None, cout, cinc, cstride, dev)
        elif net is not None and exact_means is None:
            arecs = _ROUND_BUFFERS.records("aux", A, stride, dev)
            sample_features(g, bi, hk, sb, seed, DOMAIN_AUX, False, arecs, stride, stream=stream)
            agv = _ROUND_BUFFERS.take("aux_g", A * stride, torch.float32, dev)
            net.forward(arecs, A * stride, agv, stream=stream)
            am = _moments_per_row(arecs, agv, incs, stride, dev)
        for j, r in enumerate(crow):
            st = stats[r]
            st.an += int(cm[j, 0]); st.ag += int(cm[j, 2]); st.ag2 += int(cm[j, 3])
            cdone[r] += int(cm[j, 0])
        for j, r in enumerate(active):
            st = stats[r]
            st.n += int(m[j, 0]); st.sx += int(m[j, 1]); st.sg += int(m[j, 2])
            st.sg2 += int(m[j, 3]); st.sxg += int(m[j, 4])
            if am is not None:
                st.an += int(am[j, 0]); st.ag += int(am[j, 2]); st.ag2 += int(am[j, 3])
            done[r] += incs[j]
            st.done = done[r]
        results = estimate_rows([stats[r] for r in active], i, delta, eps, max_per_row)
        still = []
        for r, (est, hw, more) in zip(active, results):
            st = stats[r]
            res.estimates[r], res.halfwidth[r] = est, hw
            res.eval_samples[r] = st.n
            res.aux_samples[r] = st.an
            if more:
                still.append(r)
        active = still
        res.rounds = i
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    return res


@dataclass
class TrainResult:
    net: Mlp
    beta: dict
    losses: list
    train_samples: int
    seconds: float
    rho2: dict = field(default_factory=dict)
    holdout: dict = field(default_factory=dict)   # row -> moments of the held-out draws
    fit: dict = field(default_factory=dict)       # row -> W.CvFitRow


def train(g: W.Csr, bi: W.BinIndex, rows: list[int], n_train: int, seed: int,
          epochs: int = 1, per_row_batch: int = 4096, lr: float = 2e-2, holdout: float = 0.2,
          init_seed: int = 7, eps: float = 1e-3, delta: float = 1e-3,
          stream=None) -> TrainResult:
    """wedge_cv_train: TRAIN draws (exact labels) spread evenly over `rows`;
    the first columns of every row fit the network (Adam on minibatches that
    hold every row), the rest are held out for beta, the fitted correlation
    and the round plans (at eps, delta)."""
    dev = g.rowptr.device
    rows = sorted(rows)
    R = len(rows)
    t0 = time.perf_counter()
    per_row = max(n_train // R, 2 * per_row_batch)
    n_fit = int(per_row * (1 - holdout)) // per_row_batch * per_row_batch
    n_hold = per_row - n_fit
    net = Mlp(dev)
    ws = _ROUND_BUFFERS.take("train_ws", int(_L().wedge_cv_train_workspace(R, n_fit, n_hold,
                                                                          per_row_batch)),
                             torch.uint8, dev)
    hr = np.ascontiguousarray(rows, dtype=np.uint32)
    fit = (W.CvFitRow * R)()
    mom = np.zeros((R, 5), dtype=np.int64)
    loss = ctypes.c_float(0.0)
    W._check(_L().wedge_cv_train(W._ptr(g.rowptr), W._ptr(g.col), g.n, g.m, W._ptr(bi.index),
                                 bi.max_bins, bi.tau, bi.omega, hr.ctypes.data_as(W._vp), R,
                                 n_fit, n_hold, per_row_batch, epochs, lr, seed, init_seed,
                                 W._ptr(net.state), eps, delta, fit,
                                 mom.ctypes.data_as(W._vp), ctypes.byref(loss), W._ptr(ws),
                                 ws.numel(), W._stream(stream)))
    net.t = epochs * (n_fit // per_row_batch)
    return TrainResult(net=net, beta={r: fit[i].beta for i, r in enumerate(rows)},
                       losses=[loss.value], train_samples=per_row * R,
                       seconds=time.perf_counter() - t0,
                       rho2={r: fit[i].rho2 for i, r in enumerate(rows)},
                       holdout={r: mom[i].copy() for i, r in enumerate(rows)},
                       fit={r: fit[i] for i, r in enumerate(rows)})


def plans(tr: TrainResult):
    """First-round sample counts per row from the held-out TRAIN draws (the
    fit's empirical-Bernstein n at delta / 2) for plain sampling and for the
    control variate.  They use no EVAL draw."""
    return ({r: int(f.plan_plain) for r, f in tr.fit.items()},
            {r: int(f.plan_cv) for r, f in tr.fit.items()})


# Centre draws of the pilot start at this sample index, far past any draw an
# estimate uses, so the plan is independent of the draws it schedules.
PILOT_BEGIN = 1 << 40
# Cost of one centre draw in EVAL draws, 1 + a d^b for a centre of degree d
# (fitted to launch times of both kinds of draw on R-MAT graphs: the lane
# path's pair loop and the wave path's gathers grow slower than d).
CENTRE_COST = (0.15, 0.7)


def centre_pilot(g: W.Csr, bi: W.BinIndex, rows: list[int], table: CentreTable, seed: int,
                 n: int = 4096, stream=None) -> dict:
    """(mean, variance) of gbar over n centre draws per row from the pilot
    range of the centre stream."""
    B = bi.max_bins
    rows = sorted(rows)
    hk = np.zeros(B + 1, dtype=np.uint64)
    hk[rows] = n
    out = torch.empty(len(rows) * n, dtype=torch.float32, device=g.rowptr.device)
    centre_means(g, bi, table, hk, PILOT_BEGIN, seed, DOMAIN_CENTRE, out, n, stream=stream)
    m = _moments_per_row(None, out, [n] * len(rows), n, g.rowptr.device)
    mean, var = mean_var_rows(m)
    return {r: (float(mean[j]), float(var[j])) for j, r in enumerate(rows)}


def centre_cost(bi: W.BinIndex, r: int, model=CENTRE_COST) -> float:
    """wedge_cv_centre_cost: modelled cost of a centre draw of row r in EVAL
    draws."""
    nb = np.ascontiguousarray(bi.h_n_b, dtype=np.uint64)
    pb = np.ascontiguousarray(bi.h_p_b, dtype=np.uint64)
    return float(_L().wedge_cv_centre_cost(nb.ctypes.data_as(W._vp), pb.ctypes.data_as(W._vp),
                                           bi.max_bins, r, model[0], model[1]))


def plans_centre(tr: TrainResult, pilot: dict, bi: W.BinIndex, eps: float, delta: float,
                 model=CENTRE_COST):
    """wedge_cv_plan_centre: first-round EVAL and centre draws and the beta
    of every row for the centre form, from the held-out TRAIN draws and the
    centre pilot (a row without a pilot entry is planned at zero gbar
    variance, the cheapest case)."""
    rows = sorted(tr.fit)
    R = len(rows)
    fit = (W.CvFitRow * R)(*[tr.fit[r] for r in rows])
    var = np.ascontiguousarray([pilot[r][1] if r in pilot else 0.0 for r in rows],
                               dtype=np.float64)
    cost = np.ascontiguousarray([centre_cost(bi, r, model) for r in rows], dtype=np.float64)
    ne = np.zeros(R, dtype=np.uint64)
    nc = np.zeros(R, dtype=np.uint64)
    bu = np.zeros(R, dtype=np.float64)
    W._check(_L().wedge_cv_plan_centre(fit, var.ctypes.data_as(W._vp),
                                       cost.ctypes.data_as(W._vp), R, eps, delta,
                                       ne.ctypes.data_as(W._vp), nc.ctypes.data_as(W._vp),
                                       bu.ctypes.data_as(W._vp)))
    return ({r: int(ne[j]) for j, r in enumerate(rows)},
            {r: int(nc[j]) for j, r in enumerate(rows)},
            {r: float(bu[j]) for j, r in enumerate(rows)})


def compare(g: W.Csr, bi: W.BinIndex, eps: float = 1e-3, delta: float = 1e-3, seed: int = 11,
            n_train: int = 10_000_000, epochs: int = 1, per_row_batch: int = 8192,
            lr: float = 4e-2, growth: float = 1.1, aux_form: bool = True,
            exact_form: bool = True, pilot: int = 4096) -> dict:
    """Samples and wall time to reach a half-width <= eps at confidence
    1 - delta on every sampled bin and on the global stream, for plain
    sampling with the empirical-Bernstein stopping rule and for the learned
    control variate with the same rule.  Both follow round plans from the
    held-out TRAIN draws (first round at the predicted n, then growing by
    `growth`).  TRAIN draws count as closure checks of the control-variate
    form; AUX draws (no closure test) are reported separately.  The control
    variate's mean comes from centre draws (learned_cv_centre), from the
    census (learned_cv_exact_mean, exact_form) or from AUX draws (aux_form)."""
    B = bi.max_bins
    rows = [r for r in range(B) if bi.h_p_b[r] > 0] + [B]
    torch.cuda.synchronize()
    tr = train(g, bi, rows, n_train, seed, epochs=epochs, per_row_batch=per_row_batch, lr=lr,
               eps=eps, delta=delta)
    plan_plain, plan_cv = plans(tr)
    # rows where the held-out draws predict fewer samples without the control
    # variate (small rho^2: the wider range 1 + |beta| of the bound costs more
    # than the variance it removes) keep beta = 0, i.e. plain sampling
    beta_used = {r: (tr.beta[r] if plan_cv[r] < plan_plain[r] else 0.0) for r in rows}
    plan_used = {r: min(plan_cv[r], plan_plain[r]) for r in rows}
    pe = sequential(g, bi, rows, eps, delta, seed, None, None, first=plan_plain, growth=growth)
    # rows that could gain from centre draws even at zero gbar variance get a
    # pilot; the others keep the plain form without spending any centre draw
    t0 = time.perf_counter()
    _, _, screen = plans_centre(tr, {}, bi, eps, delta)
    prow = [r for r in rows if screen[r] != 0.0]
    table, pil = None, {}
    if prow:
        table = CentreTable(g, bi, tr.net)
        pil = centre_pilot(g, bi, prow, table, seed, n=pilot)
    torch.cuda.synchronize()
    t_pilot = time.perf_counter() - t0
    ce_eval, ce_centre, ce_beta = plans_centre(tr, pil, bi, eps, delta)
    ce_beta = {r: (ce_beta[r] if r in pil else 0.0) for r in rows}
    if table is not None:
        cvc = sequential(g, bi, rows, eps, delta, seed, tr.net, ce_beta, first=ce_eval,
                         growth=growth, centre=table, centre_first=ce_centre)
    else:   # plain on every row: the same plan and draws as plain-EB
        cvc = pe
    means, cvx, t_census = {}, None, 0.0
    if exact_form:
        t0 = time.perf_counter()
        census = Census(g, bi)
        means = census.means(tr.net)
        torch.cuda.synchronize()
        t_census = time.perf_counter() - t0
        cvx = sequential(g, bi, rows, eps, delta, seed, tr.net, beta_used, first=plan_used,
                         growth=growth, exact_means=means)
    cvr = None
    if aux_form:
        cvr = sequential(g, bi, rows, eps, delta, seed, tr.net, tr.beta, first=plan_cv,
                         growth=growth)
    per_row = {}
    for r in rows:
        name = "global" if r == B else str(r)
        row = {"beta": round(tr.beta[r], 5), "rho2": round(tr.rho2[r], 5),
               "plan_plain": plan_plain[r], "plain_eb_samples": pe.eval_samples[r],
               "plain_eb_estimate": pe.estimates[r], "plain_eb_halfwidth": pe.halfwidth[r],
               "centre_beta": round(ce_beta[r], 5), "centre_plan_eval": ce_eval[r],
               "centre_plan_centre": ce_centre[r],
               "centre_pilot_var": pil[r][1] if r in pil else None,
               "centre_cost": round(centre_cost(bi, r), 3),
               "cv_centre_eval_samples": cvc.eval_samples[r],
               "cv_centre_draws": cvc.aux_samples[r], "cv_centre_estimate": cvc.estimates[r],
               "cv_centre_halfwidth": cvc.halfwidth[r]}
        if cvx is not None:
            row.update({"beta_used": round(beta_used[r], 5), "plan_cv": plan_cv[r],
                        "cv_exact_eval_samples": cvx.eval_samples[r],
                        "exact_mean_g": means.get(r), "cv_exact_estimate": cvx.estimates[r],
                        "cv_exact_halfwidth": cvx.halfwidth[r]})
        if cvr is not None:
            row.update({"cv_aux_eval_samples": cvr.eval_samples[r],
                        "cv_aux_samples": cvr.aux_samples[r], "cv_aux_estimate": cvr.estimates[r],
                        "cv_aux_halfwidth": cvr.halfwidth[r]})
        per_row[name] = row
    out = {
        "eps": eps, "delta": delta, "rows": len(rows), "growth": growth,
        "train": {"closure_checks": tr.train_samples, "seconds": tr.seconds,
                  "final_loss": tr.losses[-1], "epochs": epochs,
                  "minibatch": per_row_batch * len(rows)},
        "plain_eb": {"closure_checks": pe.total_eval, "seconds": pe.seconds, "rounds": pe.rounds},
        "learned_cv_centre": {"closure_checks": cvc.total_eval + tr.train_samples,
                              "eval_checks": cvc.total_eval, "train_checks": tr.train_samples,
                              "centre_draws": cvc.total_aux, "pilot_draws": pilot * len(pil),
                              "seconds": cvc.seconds + tr.seconds + t_pilot,
                              "eval_seconds": cvc.seconds, "table_pilot_seconds": t_pilot,
                              "train_seconds": tr.seconds, "rounds": cvc.rounds,
                              "rows_with_cv": int(sum(1 for r in rows if ce_beta[r] != 0.0))},
        "network_gain_eval_checks": pe.total_eval / max(cvc.total_eval, 1),
        "per_row": per_row,
    }
    if cvx is not None:
        out["network_gain_eval_checks_exact_mean"] = pe.total_eval / max(cvx.total_eval, 1)
    if cvx is not None:
        out["learned_cv_exact_mean"] = {"closure_checks": cvx.total_eval + tr.train_samples,
                                        "eval_checks": cvx.total_eval,
                                        "train_checks": tr.train_samples,
                                        "seconds": cvx.seconds + tr.seconds + t_census,
                                        "eval_seconds": cvx.seconds, "census_seconds": t_census,
                                        "train_seconds": tr.seconds, "rounds": cvx.rounds}
    if cvr is not None:
        out["learned_cv_aux"] = {"closure_checks": cvr.total_eval + tr.train_samples,
                                 "eval_checks": cvr.total_eval, "aux_draws": cvr.total_aux,
                                 "seconds": cvr.seconds + tr.seconds, "rounds": cvr.rounds}
    return out
