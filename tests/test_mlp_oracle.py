"""Pins of the MLP oracle: forward, backward and Adam against torch's
independent float64 implementation, central finite differences, and
closed-form special cases; the control-variate estimator against its
defining identities."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def torch_model(theta):
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in M.unpack(theta.copy()).items()}
    return p


def torch_loss(p, x, y):
    xt = torch.tensor(x, dtype=torch.float64)
    a1 = xt @ p["W1"].T + p["b1"]
    h1 = torch.nn.functional.gelu(a1)            # exact erf form
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = torch.nn.functional.gelu(a2)
    z = h2 @ p["W3"] + p["b3"][0]
    yt = torch.tensor(y, dtype=torch.float64)
    return torch.nn.functional.binary_cross_entropy_with_logits(z, yt), torch.sigmoid(z)


def data(n=200, seed=0):
    rng = np.random.default_rng(seed)
    dv = rng.integers(2, 5000, n)
    da = rng.integers(1, 5000, n)
    dc = rng.integers(1, 5000, n)
    b = rng.integers(2, 14, n)
    x = M.features(dv, da, dc, b)
    y = (rng.random(n) < 0.3).astype(np.float64)
    return x, y


def test_parameter_count():
    assert M.NPARAM == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4545


def test_mitchell_log2_exact_at_powers_and_linear_between():
    assert M.mitchell_log2([1, 2, 4, 1024]).tolist() == [0, 1, 2, 10]
    assert M.mitchell_log2([3]).tolist() == [1.5]
    assert M.mitchell_log2([6, 12]).tolist() == [2.5, 3.5]
    d = np.arange(1, 1 << 16)
    L = M.mitchell_log2(d)
    assert (np.abs(L - np.log2(d)) <= 0.0861).all()   # Mitchell's max error
    assert (L.astype(np.float32).astype(np.float64) == L).all()


def test_bf16_rounding_ties_to_even():
    assert M.bf16([1.0, 0.0, -2.0]).tolist() == [1.0, 0.0, -2.0]
    one_plus_half_ulp = 1.0 + 2.0 ** -8           # halfway between 1 and next bf16
    assert M.bf16([one_plus_half_ulp])[0] == 1.0   # tie -> even mantissa
    assert M.bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6
    x = np.random.default_rng(0).normal(size=1000)
    r = M.bf16(x)
    assert (np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-30).all()


def test_forward_matches_torch_float64():
    theta = M.init_params(1)
    x, y = data()
    g, _ = M.forward(theta, x, rounding=False)
    p = torch_model(theta)
    _, gt = torch_loss(p, x, y)
    assert np.allclose(g, gt.detach().numpy(), rtol=1e-13, atol=1e-15)
    assert M.loss(theta, x, y, rounding=False) == pytest.approx(
        float(torch_loss(p, x, y)[0]), rel=1e-13)


def test_backward_matches_torch_autograd_and_finite_differences():
    theta = M.init_params(2)
    x, y = data(64, seed=3)
    gr = M.backward(theta, x, y, rounding=False)
    p = torch_model(theta)
    L, _ = torch_loss(p, x, y)
    L.backward()
    gt = M.pack({k: v.grad.numpy() for k, v in p.items()})
    assert np.allclose(gr, gt, rtol=1e-10, atol=1e-14)
    # central differences on a sample of coordinates
    rng = np.random.default_rng(4)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss(tp, x, y, rounding=False) - M.loss(tm, x, y, rounding=False)) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(gr[i])) + 1e-9, i


def test_rounded_pass_stays_close_to_exact():
    theta = M.init_params(5)
    x, y = data(256, seed=6)
    g0, _ = M.forward(theta, x, rounding=False)
    g1, _ = M.forward(theta, x, rounding=True)
    assert np.abs(g0 - g1).max() < 2e-2
    d0 = M.backward(theta, x, y, rounding=False)
    d1 = M.backward(theta, x, y, rounding=True)
    cos = float(d0 @ d1 / np.linalg.norm(d0) / np.linalg.norm(d1))
    assert cos > 0.999


def test_adam_matches_torch():
    theta = M.init_params(7)
    x, y = data(128, seed=8)
    p = torch_model(theta)
    opt = torch.optim.Adam(list(p.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = theta.copy(), np.zeros(M.NPARAM), np.zeros(M.NPARAM)
    for t in range(1, 6):
        gr = M.backward(th, x, y, rounding=False)
        th, m, v = M.adam_step(th, gr, m, v, t)
        opt.zero_grad()
        L, _ = torch_loss(p, x, y)
        L.backward()
        opt.step()
        tt = M.pack({k: w.detach().numpy() for k, w in p.items()})
        assert np.allclose(th, tt, rtol=1e-9, atol=1e-12)


def test_special_cases():
    # all weights zero: g = sigmoid(b3), gradient only on b3 and W3 = 0 rows
    theta = np.zeros(M.NPARAM)
    theta[-1] = 0.7
    x, y = data(50, seed=9)
    g, _ = M.forward(theta, x, rounding=True)
    assert np.allclose(g, 1 / (1 + math.exp(-0.7)))
    gr = M.backward(theta, x, y, rounding=True)
    assert gr[-1] == pytest.approx(float(np.mean(g - y)), rel=1e-12)
    assert np.allclose(gr[:-1 - 64], 0.0)          # GELU(0) = 0 kills W3's gradient too
    # GELU closed forms
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert M.gelu(np.array([8.0]))[0] == pytest.approx(8.0, rel=1e-14)
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5


def test_cv_estimator_identities():
    rng = np.random.default_rng(10)
    X = (rng.random(5000) < 0.2).astype(float)
    aux = rng.random(3000)
    # constant g: the control variate cancels exactly
    c = M.cv_estimate(X, np.full(5000, 0.37), np.full(3000, 0.37), beta=0.8)
    assert c == pytest.approx(X.mean(), abs=1e-15)
    # g = the exact label, beta = 1: the EVAL residual is identically zero
    z = X - 1.0 * X
    assert (z == 0).all()
    assert M.cv_estimate(X, X, aux, beta=1.0) == pytest.approx(aux.mean(), abs=1e-15)
    # beta = 0 is the plain estimator
    assert M.cv_estimate(X, rng.random(5000), aux, beta=0.0) == X.mean()


def test_eb_halfwidth_properties():
    # decreasing in n, increasing in the variance, reduces to the range term at var 0
    w = [M.eb_halfwidth(n, 0.1, 1.0, 1e-3) for n in (100, 1000, 10000)]
    assert w[0] > w[1] > w[2]
    assert M.eb_halfwidth(1000, 0.2, 1.0, 1e-3) > M.eb_halfwidth(1000, 0.1, 1.0, 1e-3)
    L = math.log(4e3)
    assert M.eb_halfwidth(1000, 0.0, 1.0, 1e-3) == pytest.approx(7 * L / (3 * 999))
    # valid coverage on Bernoulli(0.1) over many trials
    rng = np.random.default_rng(11)
    miss = 0
    for _ in range(400):
        s = (rng.random(2000) < 0.1).astype(float)
        if abs(s.mean() - 0.1) > M.eb_halfwidth(2000, s.var(ddof=1), 1.0, 0.05):
            miss += 1
    assert miss / 400 <= 0.05
