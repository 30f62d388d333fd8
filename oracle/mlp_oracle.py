"""MLP oracle for the learned control variate (test infrastructure only).

A 4 -> 64 -> 64 -> 1 perceptron with GELU hidden units and a sigmoid output
predicts the closure probability of a sampled wedge from the log-degrees of
its centre and endpoints and the centre's bin; it enters the wedge-sampling
estimator (Thm. cd-est) only as a control variate, so every closure test
stays exact.  This module is the plain NumPy float64 definition of what the
GPU kernels compute:

  features  x = (K(d_v) / 256, K(min(d_a, d_c)) / 256, K(max(d_a, d_c)) / 256,
            bin / 32) with K(d) = floor(8 L(d)) the log-degree bucket and
            L(d) = e + (d - 2^e) / 2^e, e = floor(log2 d) (Mitchell's
            piecewise-linear log2); every feature is exact in bfloat16, and
            the network is a function of (bin, bucket of the centre, bucket
            pair of the endpoints), which makes its mean over all wedges of
            a bin a finite sum over a census of bucket pairs
  layer 1   h1 = GELU(W1 x + b1),  GELU(a) = a/2 (1 + erf(a / sqrt 2))
  layer 2   h2 = GELU(W2 h1 + b2)
  output    z = W3 h2 + b3,  g = sigmoid(z)
  loss      binary cross-entropy averaged over the batch,
            softplus(z) - y z
  update    Adam (Kingma & Ba, 2015) on float32 master weights.

BF16 rounding points mirror the GPU: weights, features and the hidden
activations that feed the next layer are rounded to bfloat16 (round to
nearest even) before each product; accumulation and biases stay wide.

It never imports the product package.
"""
from __future__ import annotations

import math

import numpy as np

H = 64
NF = 4
# parameter vector layout (float32 master copy on the GPU)
SHAPES = [("W1", (H, NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)),
          ("b3", (1,))]
SIZES = [int(np.prod(s)) for _, s in SHAPES]
NPARAM = sum(SIZES)   # 4545


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for (name, shp), sz in zip(SHAPES, SIZES):
        out[name] = theta[o:o + sz].reshape(shp)
        o += sz
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to float32 as the GPU holds it."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    rounded = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def mitchell_log2(d) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    e = np.floor(np.log2(np.maximum(d, 1.0)))
    p = np.exp2(e)
    return e + (d - p) / p


def bucket(d) -> np.ndarray:
    """K(d) = floor(8 L(d)) for d >= 1 (0 for d = 0), exactly in integers."""
    d = np.asarray(d, dtype=np.int64)
    out = np.zeros(d.shape, dtype=np.int64)
    pos = d > 0
    e = np.floor(np.log2(np.maximum(d, 1))).astype(np.int64)
    e = np.where((np.int64(1) << e) > d, e - 1, e)          # guard float log2
    e = np.where((np.int64(1) << (e + 1)) <= d, e + 1, e)
    p = np.int64(1) << e
    out[pos] = (8 * e + ((d - p) * 8) // p)[pos]
    return out


def features(dv, da, dc, b) -> np.ndarray:
    """Feature rows (n, 4) of wedges with centre degree dv, endpoint degrees
    da, dc (unordered) and centre bin b."""
    lo = np.minimum(da, dc)
    hi = np.maximum(da, dc)
    x = np.stack([bucket(dv) / 256.0, bucket(lo) / 256.0, bucket(hi) / 256.0,
                  np.asarray(b, dtype=np.float64) / 32.0], axis=1)
    return x


def gelu(a):
    return 0.5 * a * (1.0 + np.vectorize(math.erf)(a / math.sqrt(2.0)))


def gelu_grad(a):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(a / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * a * a) / math.sqrt(2.0 * math.pi)
    return cdf + a * pdf


def forward(theta: np.ndarray, x: np.ndarray, rounding: bool = True):
    """Returns (g, cache).  x: (n, 4)."""
    p = unpack(theta)
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    xb = r(x)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    a1 = xb @ W1.T + p["b1"]
    h1 = r(gelu(a1))
    a2 = h1 @ W2.T + p["b2"]
    h2 = gelu(a2)
    z = h2 @ W3 + p["b3"][0]
    g = 1.0 / (1.0 + np.exp(-z))
    return g, dict(xb=xb, W1=W1, W2=W2, W3=W3, a1=a1, h1=h1, a2=a2, h2=h2, z=z)


def loss(theta, x, y, rounding=True) -> float:
    g, c = forward(theta, x, rounding)
    z = c["z"]
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def backward(theta: np.ndarray, x: np.ndarray, y: np.ndarray, rounding: bool = True):
    """Gradient of the mean BCE loss w.r.t. the parameter vector.  The
    rounded weights are treated as the weights (straight-through), as the GPU
    does when it updates the float32 master copy; with rounding, the
    back-propagated pre-activation gradients that enter a matrix product are
    rounded to bfloat16 like the GPU's matrix-core operands."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    g, c = forward(theta, x, rounding)
    n = x.shape[0]
    dz = (g - y) / n
    dW3 = c["h2"].T @ dz
    db3 = np.array([dz.sum()])
    dh2 = np.outer(dz, c["W3"])
    da2 = dh2 * gelu_grad(c["a2"])
    da2r = r(da2)
    dW2 = da2r.T @ c["h1"]
    db2 = da2.sum(axis=0)
    dh1 = da2r @ c["W2"]
    da1 = dh1 * gelu_grad(c["a1"])
    dW1 = r(da1).T @ c["xb"]
    db1 = da1.sum(axis=0)
    return pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step t >= 1), bias-corrected."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


def init_params(seed: int) -> np.ndarray:
    """A reproducible starting point for tests (uniform, fan-in scaled)."""
    rng = np.random.default_rng(seed)
    p = {}
    for (name, shp) in SHAPES:
        fan_in = shp[1] if len(shp) == 2 else (H if name != "b1" else NF)
        bound = 1.0 / math.sqrt(fan_in)
        p[name] = rng.uniform(-bound, bound, size=shp)
    return pack(p).astype(np.float32).astype(np.float64)


# ---------------------------------------------------- control-variate estimator
def cv_estimate(x_eval, g_eval, g_aux, beta):
    """Unbiased control-variate estimate of E[X]:
    mean_EVAL(X - beta g) + beta mean_AUX(g), with beta fixed beforehand and
    the AUX draws independent of the EVAL draws."""
    z = np.asarray(x_eval, np.float64) - beta * np.asarray(g_eval, np.float64)
    return float(z.mean() + beta * np.mean(np.asarray(g_aux, np.float64)))


def eb_halfwidth(n: int, var: float, R: float, delta: float) -> float:
    """Two-sided empirical-Bernstein half-width (Maurer & Pontil 2009,
    Thm. 4, each side at delta/2) for the mean of n i.i.d. values in an
    interval of length R with sample variance var (n-1 denominator)."""
    if n < 2:
        return float("inf")
    L = math.log(4.0 / delta)
    return math.sqrt(2.0 * var * L / n) + 7.0 * R * L / (3.0 * (n - 1))
