"""Learned control variate on the GPU: the feature stream against the
oracle's sampler, the network's forward pass, gradient and Adam step against
the MLP oracle (BF16 tolerance), exact integer moments, and the estimator's
defining identities and unbiasedness."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from oracle import oracle as O
from paper_1301_5887_amd import cv as C
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


@pytest.fixture(scope="module")
def c1():
    n, src, dst = gen.chung_lu_c1(1)
    g = W.build_csr(dev(src), dev(dst), n)
    bi = W.bin_counts(g, 2, 2, 24)
    og = O.build_graph(src, dst, n)
    return g, bi, og


def test_feature_stream_matches_oracle(c1):
    g, bi, og = c1
    B = bi.max_bins
    rows = [r for r in range(B) if bi.h_p_b[r] > 0] + [B]
    k, s_begin, seed = 3000, 1000, 77
    hk = np.zeros(B + 1, dtype=np.uint64)
    hk[rows] = k
    print(f"[cv] feature stream rows={len(rows)} k={k} s_begin={s_begin}", flush=True)
    for domain, closure in ((C.DOMAIN_TRAIN, True), (C.DOMAIN_AUX, False)):
        recs = C.new_records(len(rows), k)
        C.sample_features(g, bi, hk, s_begin, seed, domain, closure, recs, k)
        torch.cuda.synchronize()
        r = C.records_to_numpy(recs).reshape(len(rows), k)
        s = O.sample(og, 2, 2, B, hk[:B], int(hk[B]), seed, dump_per_bin=k, domain=domain,
                     s_begin=s_begin)
        deg = og.degrees().astype(np.int64)
        for j, row in enumerate(rows):
            v, a, c, cls = s.v[row], s.a[row], s.c[row], s.cls[row]
            assert (r["dv"][j] == deg[v]).all()
            assert (r["dlo"][j] == np.minimum(deg[a], deg[c])).all()
            assert (r["dhi"][j] == np.maximum(deg[a], deg[c])).all()
            assert all(int(b) == O.bin_id(int(d), 2, 2) for b, d in zip(r["bin"][j][:200], deg[v][:200]))
            if closure:
                assert (r["closed"][j] == (cls > 0)).all()
                assert (r["cls"][j] == cls).all()
            else:
                assert (r["closed"][j] == 0).all()


def test_feature_stream_per_row_starts(c1):
    """Rows drawn from different sample indices and in different numbers in
    one launch: each row matches the oracle's stream at its own start."""
    g, bi, og = c1
    B = bi.max_bins
    rows = [r for r in range(B) if bi.h_p_b[r] > 0] + [B]
    hk = np.zeros(B + 1, dtype=np.uint64)
    sb = np.zeros(B + 1, dtype=np.uint64)
    for j, r in enumerate(rows):
        hk[r] = 500 + 97 * j
        sb[r] = 1000 + 4099 * j
    stride = int(hk.max())
    print(f"[cv] per-row starts rows={len(rows)} stride={stride}", flush=True)
    recs = C.new_records(len(rows), stride)
    C.sample_features(g, bi, hk, sb, 5, C.DOMAIN_EVAL, True, recs, stride)
    torch.cuda.synchronize()
    r = C.records_to_numpy(recs).reshape(len(rows), stride)
    deg = og.degrees().astype(np.int64)
    for j, row in enumerate(rows):
        k1 = np.zeros(B + 1, dtype=np.uint64)
        k1[row] = hk[row]
        s = O.sample(og, 2, 2, B, k1[:B], int(k1[B]), 5, dump_per_bin=int(hk[row]),
                     domain=C.DOMAIN_EVAL, s_begin=int(sb[row]))
        k = int(hk[row])
        assert (r["dv"][j][:k] == deg[s.v[row]]).all()
        assert (r["closed"][j][:k] == (s.cls[row] > 0)).all()
        assert (r["cls"][j][:k] == s.cls[row]).all()


def make_records(n, seed):
    rng = np.random.default_rng(seed)
    rec = np.zeros(n, dtype=C.FEATURE_DTYPE)
    rec["dv"] = rng.integers(2, 3000, n)
    a = rng.integers(1, 3000, n)
    b = rng.integers(1, 3000, n)
    rec["dlo"] = np.minimum(a, b)
    rec["dhi"] = np.maximum(a, b)
    rec["bin"] = [O.bin_id(int(d), 2, 2) for d in rec["dv"]]
    rec["closed"] = (rng.random(n) < 0.3).astype(np.uint8)
    return rec


def upload_records(rec):
    return torch.from_numpy(rec.view(np.uint8).copy()).cuda().view(torch.int32)


def oracle_x(rec):
    return M.features(rec["dv"].astype(np.int64), rec["dlo"].astype(np.int64),
                      rec["dhi"].astype(np.int64), rec["bin"].astype(np.int64))


def net_with(theta):
    net = C.Mlp()
    net.set(torch.tensor(theta, dtype=torch.float32, device="cuda"))
    return net


def test_mlp_forward_matches_oracle():
    rec = make_records(3001, 1)            # ragged: not a multiple of 16
    theta = M.init_params(3)
    net = net_with(theta)
    g = torch.zeros(len(rec), dtype=torch.float32, device="cuda")
    net.forward(upload_records(rec), len(rec), g)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.float64)
    go, _ = M.forward(theta, oracle_x(rec), rounding=True)
    err = np.abs(gg - go)
    assert err.max() < 2e-3 and err.mean() < 2e-4, (err.max(), err.mean())


def test_mlp_gradient_matches_oracle():
    rec = make_records(1040, 2)
    theta = M.init_params(4)
    net = net_with(theta)
    net.grad_of(upload_records(rec), 1, len(rec), 0, len(rec))
    torch.cuda.synchronize()
    gg = net.grad.cpu().numpy().astype(np.float64)
    y = rec["closed"].astype(np.float64)
    go = M.backward(theta, oracle_x(rec), y, rounding=True)
    for (name, _), sz, off in zip(M.SHAPES, M.SIZES, np.cumsum([0] + M.SIZES[:-1])):
        a, b = gg[off:off + sz], go[off:off + sz]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))
        assert rel <= 2e-2 and cos >= 0.999, (name, rel, cos)
    lo = M.loss(theta, oracle_x(rec), y, rounding=True)
    assert abs(float(net.loss.item()) - lo) <= 1e-3 * abs(lo)


def test_minibatch_view_selects_rows():
    """A minibatch of per_row records from each row equals the gradient over
    those records laid out contiguously."""
    rec = make_records(4 * 300, 5)
    theta = M.init_params(6)
    net = net_with(theta)
    d = upload_records(rec)
    net.grad_of(d, 4, 300, 40, 32)            # rows of 300, columns 40..71
    torch.cuda.synchronize()
    g1 = net.grad.cpu().numpy().copy()
    sub = np.concatenate([rec[r * 300 + 40: r * 300 + 72] for r in range(4)])
    net.grad_of(upload_records(sub), 1, len(sub), 0, len(sub))
    torch.cuda.synchronize()
    g2 = net.grad.cpu().numpy()
    assert np.allclose(g1, g2, rtol=1e-5, atol=1e-9)


def test_train_loop_equals_step_by_step_calls():
    """wedge_mlp_train queues exactly the grad + Adam steps a caller would."""
    rows, per_row, batch = 3, 2048, 256
    rec = make_records(rows * per_row, 31)
    x = upload_records(rec)
    theta = M.init_params(5)
    a, b = net_with(theta), net_with(theta)
    a.train(x, rows, per_row, 1536, batch, 2, lr=3e-3)
    for ep in range(2):
        for j0 in range(0, 1536, batch):
            b.grad_of(x, rows, per_row, j0, batch)
            b.adam(lr=3e-3)
    torch.cuda.synchronize()
    assert a.t == b.t == 12
    assert torch.equal(a.get(), b.get())
    assert torch.equal(a.loss, b.loss)


def test_adam_step_matches_oracle():
    theta = M.init_params(8)
    net = net_with(theta)
    rng = np.random.default_rng(9)
    m = np.zeros(M.NPARAM)
    v = np.zeros(M.NPARAM)
    th = theta.copy()
    for t in range(1, 4):
        grad = rng.normal(scale=1e-2, size=M.NPARAM).astype(np.float32)
        net.adam(lr=1e-3, grad=torch.tensor(grad, device="cuda"))
        th, m, v = M.adam_step(th, grad.astype(np.float64), m, v, t, lr=1e-3)
    torch.cuda.synchronize()
    got = net.get().cpu().numpy().astype(np.float64)
    assert np.allclose(got, th, rtol=1e-5, atol=1e-7)


def test_moments_are_exact_integers():
    rec = make_records(5000, 10)
    d = upload_records(rec)
    net = net_with(M.init_params(11))
    g = torch.zeros(len(rec), dtype=torch.float32, device="cuda")
    net.forward(d, len(rec), g)
    mom = C.moments(d, g, 5, 1000, 997)       # 5 rows of 1000, first 997 used
    torch.cuda.synchronize()
    got = W.to_host_u64(mom).view(np.int64).reshape(5, 5)
    gv = g.cpu().numpy().astype(np.float64).reshape(5, 1000)[:, :997]
    X = rec["closed"].reshape(5, 1000)[:, :997].astype(np.int64)
    gq = np.rint(gv * 2.0 ** 32).astype(np.int64)
    g2q = np.rint(gv * gv * 2.0 ** 32).astype(np.int64)
    ref = np.stack([np.full(5, 997), X.sum(1), gq.sum(1), g2q.sum(1), (X * gq).sum(1)], 1)
    assert (got == ref).all()
    # a count per row, as the sequential rounds use
    cnt = [1000, 0, 17, 640, 999]
    mom = C.moments(d, g, 5, 1000, 0, counts=cnt)
    got = W.to_host_u64(mom).view(np.int64).reshape(5, 5)
    gv = g.cpu().numpy().astype(np.float64).reshape(5, 1000)
    X = rec["closed"].reshape(5, 1000).astype(np.int64)
    for r, c in enumerate(cnt):
        gq = np.rint(gv[r, :c] * 2.0 ** 32).astype(np.int64)
        g2q = np.rint(gv[r, :c] * gv[r, :c] * 2.0 ** 32).astype(np.int64)
        ref = [c, X[r, :c].sum(), gq.sum(), g2q.sum(), (X[r, :c] * gq).sum()]
        assert list(got[r]) == ref, r


def test_constant_network_equals_plain(c1):
    """g constant: the control variate cancels, c_CV = plain mean exactly."""
    g, bi, og = c1
    theta = np.zeros(M.NPARAM)
    theta[-1] = -0.4
    net = net_with(theta)
    rows = [r for r in range(bi.max_bins) if bi.h_p_b[r] > 0]
    beta = {r: 0.8 for r in rows}
    cvr = C.sequential(g, bi, rows, 1e-9, 1e-3, 5, net, beta, n0=1 << 13, max_per_row=1 << 13)
    pl = C.sequential(g, bi, rows, 1e-9, 1e-3, 5, None, None, n0=1 << 13, max_per_row=1 << 13)
    for r in rows:
        assert cvr.estimates[r] == pytest.approx(pl.estimates[r], abs=1e-12)


def test_cv_unbiased_and_not_worse_than_plain(c1):
    """Over independent seeds, the CV estimate of every bin is centred on the
    exact closed fraction (3 standard errors) and its spread is no larger
    than plain sampling's beyond noise."""
    g, bi, og = c1
    B = bi.max_bins
    P = O.exact(og, 2, 2, B)
    rows = [r for r in range(B) if bi.h_p_b[r] > 0]
    tr = C.train(g, bi, rows, 200_000, seed=3, epochs=2, per_row_batch=256, lr=5e-3)
    assert tr.losses[-1] < 0.69
    ests_cv = {r: [] for r in rows}
    ests_pl = {r: [] for r in rows}
    R, n = 24, 1 << 12
    for sd in range(R):
        cvr = C.sequential(g, bi, rows, 1e-9, 1e-3, 100 + sd, tr.net, tr.beta, n0=n,
                           max_per_row=n)
        pl = C.sequential(g, bi, rows, 1e-9, 1e-3, 100 + sd, None, None, n0=n, max_per_row=n)
        for r in rows:
            ests_cv[r].append(cvr.estimates[r])
            ests_pl[r].append(pl.estimates[r])
    for r in rows:
        c_true = float(P[r, 1:].sum()) / float(bi.h_p_b[r])
        e = np.array(ests_cv[r])
        se = max(e.std(ddof=1), 1e-6) / math.sqrt(R)
        assert abs(e.mean() - c_true) <= 3.5 * se + 1e-9, (r, e.mean(), c_true, se)
        assert e.std(ddof=1) <= 1.5 * np.std(ests_pl[r], ddof=1) + 1e-6


def small_graphs():
    e = np.array([[1, 2], [1, 3], [2, 4], [3, 4], [3, 5], [4, 5], [4, 6]], dtype=np.uint32)
    yield "worked_example", 7, e[:, 0], e[:, 1]
    rng = np.random.default_rng(12)
    yield "random", 300, rng.integers(0, 300, 3000).astype(np.uint32), \
        rng.integers(0, 300, 3000).astype(np.uint32)
    n, src, dst = gen.chung_lu_c1(1)
    yield "chung_lu", n, src, dst
    # every census mode: hubs above 2048 neighbours, medium centres, and a
    # low-degree background
    rng = np.random.default_rng(13)
    n = 6000
    s = [rng.integers(0, n, 12000)]
    d = [rng.integers(0, n, 12000)]
    for h, k in [(0, 3500), (1, 2600), (2, 2100)]:
        s.append(np.full(k, h))
        d.append(rng.choice(n, k, replace=False))
    for h in range(10, 40):
        k = int(rng.integers(40, 1500))
        s.append(np.full(k, h))
        d.append(rng.choice(n, k, replace=False))
    yield "hubs", n, np.concatenate(s).astype(np.uint32), np.concatenate(d).astype(np.uint32)


@pytest.mark.parametrize("case", ["worked_example", "random", "chung_lu", "hubs"])
def test_census_matches_oracle(case):
    name, n, src, dst = next(c for c in small_graphs() if c[0] == case)
    print(f"[cv] census {name}", flush=True)
    tau, omega, B = 2, 2, 24
    g = W.build_csr(dev(src), dev(dst), n)
    bi = W.bin_counts(g, tau, omega, B)
    cen = C.Census(g, bi)
    tab = cen.table()
    og = O.build_graph(src, dst, n)
    ref = O.pair_census(og, tau, omega, B)
    got = {}
    for key in range(cen.nkeys):
        nz = np.nonzero(tab[key])[0]
        for p in nz:
            j = int((math.isqrt(8 * int(p) + 1) - 1) // 2)
            i = int(p) - j * (j + 1) // 2
            got[(int(cen.key_bin[key]), int(cen.key_bucket[key]), i, j)] = int(tab[key, p])
    assert got == ref
    per_bin = np.zeros(B, dtype=np.uint64)
    for (b, k, i, j), c in ref.items():
        per_bin[b] += c
    assert (per_bin == bi.h_p_b).all()


def test_exact_mean_matches_oracle_and_sampling(c1):
    g, bi, og = c1
    B = bi.max_bins
    theta = M.init_params(21)
    net = net_with(theta)
    cen = C.Census(g, bi)
    means = cen.means(net)
    ref = O.pair_census(og, 2, 2, B)
    num = np.zeros(B)
    den = np.zeros(B)
    keys = list(ref.keys())
    kb = np.array([k[0] for k in keys])
    x = np.stack([np.array([k[1] for k in keys]) / 256.0, np.array([k[2] for k in keys]) / 256.0,
                  np.array([k[3] for k in keys]) / 256.0, kb / 32.0], axis=1)
    go, _ = M.forward(theta, x, rounding=True)
    cnt = np.array([ref[k] for k in keys], dtype=np.float64)
    for b in range(B):
        sel = kb == b
        if sel.any():
            num[b] = (cnt[sel] * go[sel]).sum()
            den[b] = cnt[sel].sum()
    for b in range(B):
        if den[b] > 0:
            assert abs(means[b] - num[b] / den[b]) < 2e-3, b
    # the mean over uniform EVAL draws agrees within sampling error
    rows = [b for b in range(B) if bi.h_p_b[b] > 0]
    k = 1 << 16
    hk = np.zeros(B + 1, dtype=np.uint64)
    hk[rows] = k
    recs = C.new_records(len(rows), k)
    C.sample_features(g, bi, hk, 0, 9, C.DOMAIN_EVAL, False, recs, k)
    gv = torch.zeros(len(rows) * k, dtype=torch.float32, device="cuda")
    net.forward(recs, len(rows) * k, gv)
    emp = gv.cpu().numpy().reshape(len(rows), k).astype(np.float64)
    for j, b in enumerate(rows):
        se = emp[j].std(ddof=1) / math.sqrt(k)
        assert abs(emp[j].mean() - means[b]) <= 5 * se + 1e-7, (b, emp[j].mean(), means[b], se)


def test_exact_mean_cv_unbiased_and_tighter(c1):
    g, bi, og = c1
    B = bi.max_bins
    P = O.exact(og, 2, 2, B)
    rows = [r for r in range(B) if bi.h_p_b[r] > 0]
    tr = C.train(g, bi, rows, 200_000, seed=4, epochs=2, per_row_batch=256, lr=5e-3)
    means = C.Census(g, bi).means(tr.net)
    ests, pl = {r: [] for r in rows}, {r: [] for r in rows}
    R, n = 24, 1 << 12
    for sd in range(R):
        cvx = C.sequential(g, bi, rows, 1e-9, 1e-3, 300 + sd, tr.net, tr.beta, n0=n,
                           max_per_row=n, exact_means=means)
        p = C.sequential(g, bi, rows, 1e-9, 1e-3, 300 + sd, None, None, n0=n, max_per_row=n)
        for r in rows:
            ests[r].append(cvx.estimates[r])
            pl[r].append(p.estimates[r])
    worse = 0
    for r in rows:
        c_true = float(P[r, 1:].sum()) / float(bi.h_p_b[r])
        e = np.array(ests[r])
        se = max(e.std(ddof=1), 1e-6) / math.sqrt(R)
        assert abs(e.mean() - c_true) <= 3.5 * se + 1e-9, (r, e.mean(), c_true, se)
        worse += e.std(ddof=1) > np.std(pl[r], ddof=1)
    assert worse <= len(rows) // 2


def test_compare_reaches_the_interval(c1):
    """The estimator comparison end to end on the small graph: every row of
    plain-EB and of the exact-mean control variate stops with a half-width
    <= eps, and each estimate lies within a few eps of the exact c_b."""
    g, bi, og = c1
    B = bi.max_bins
    P = O.exact(og, 2, 2, B)
    eps = 0.01
    print("[cv] compare on the Chung-Lu graph, eps=0.01", flush=True)
    res = C.compare(g, bi, eps=eps, delta=1e-3, seed=17, n_train=200_000, epochs=2,
                    per_row_batch=512, lr=3e-3, aux_form=False)
    wedges = P.sum(axis=1)
    closed = P[:, 1:].sum(axis=1)
    c_glob = float(closed.sum()) / float(wedges.sum())
    for name, row in res["per_row"].items():
        c_true = c_glob if name == "global" else float(closed[int(name)]) / float(wedges[int(name)])
        assert row["plain_eb_halfwidth"] <= eps and row["cv_exact_halfwidth"] <= eps, name
        assert row["cv_centre_halfwidth"] <= eps, name
        assert abs(row["plain_eb_estimate"] - c_true) <= 3 * eps, name
        assert abs(row["cv_exact_estimate"] - c_true) <= 3 * eps, name
        assert abs(row["cv_centre_estimate"] - c_true) <= 3 * eps, name
        if row["centre_beta"] == 0.0:
            assert row["cv_centre_draws"] == 0, name
    assert res["learned_cv_exact_mean"]["train_checks"] > 0
    assert res["learned_cv_centre"]["train_checks"] > 0


def centre_gbar(og, theta, centres):
    """Mean of the network's g over every neighbour pair of each centre,
    summed by endpoint bucket pair (the network sees the endpoints only
    through their buckets); the grouping is checked against plain pair
    enumeration on the small centres."""
    deg = og.degrees().astype(np.int64)
    parts, combos = {}, {}
    for v in np.unique(centres):
        v = int(v)
        d = int(deg[v])
        b = O.bin_id(d, 2, 2)
        kv = int(M.bucket(np.array([d]))[0])
        nb = og.col[int(og.rowptr[v]): int(og.rowptr[v + 1])]
        h = np.bincount(M.bucket(deg[nb]), minlength=256).astype(np.float64)
        nz = np.nonzero(h)[0]
        pi, pj = np.meshgrid(nz, nz, indexing="ij")
        up = pi <= pj
        pi, pj = pi[up], pj[up]
        w = np.where(pi == pj, h[pi] * (h[pi] - 1) / 2, h[pi] * h[pj])
        idx = [combos.setdefault((kv, b, int(i), int(j)), len(combos)) for i, j in zip(pi, pj)]
        parts[v] = (d, b, nb, np.array(idx), w)
    keys = np.array(list(combos.keys()), dtype=np.float64)
    x = np.stack([keys[:, 0] / 256.0, keys[:, 2] / 256.0, keys[:, 3] / 256.0,
                  keys[:, 1] / 32.0], axis=1)
    gk = M.forward(theta, x, rounding=True)[0]
    out = {}
    for v, (d, b, nb, idx, w) in parts.items():
        out[v] = float((w * gk[idx]).sum()) / (d * (d - 1) / 2)
        if d <= 12:
            pa, pc = np.triu_indices(d, 1)
            xd = M.features(np.full(pa.size, d), deg[nb[pa]], deg[nb[pc]], np.full(pa.size, b))
            direct = M.forward(theta, xd, rounding=True)[0].mean()
            assert abs(direct - out[v]) < 1e-12, (v, direct, out[v])
    return out


@pytest.mark.parametrize("case", ["chung_lu", "hubs"])
def test_centre_draws_match_oracle(case, c1):
    """Centres drawn from the centre stream equal the oracle sampler's centres
    at the same indices (key (seed, 6)); gbar of every draw matches the mean of
    the oracle network over all neighbour pairs of that centre."""
    if case == "chung_lu":
        g, bi, og = c1
    else:
        name, n, src, dst = next(c for c in small_graphs() if c[0] == case)
        g = W.build_csr(dev(src), dev(dst), n)
        bi = W.bin_counts(g, 2, 2, 24)
        og = O.build_graph(src, dst, n)
    B = bi.max_bins
    theta = M.init_params(31)
    net = net_with(theta)
    table = C.CentreTable(g, bi, net)
    rows = [r for r in range(B) if bi.h_p_b[r] > 0] + [B]
    hk = np.zeros(B + 1, dtype=np.uint64)
    sb = np.zeros(B + 1, dtype=np.uint64)
    for j, r in enumerate(rows):
        hk[r] = 300 + 37 * j
        sb[r] = 5000 * j
    stride = int(hk.max())
    print(f"[cv] centre draws {case} rows={len(rows)} stride={stride}", flush=True)
    out = torch.full((len(rows) * stride,), -1.0, dtype=torch.float32, device="cuda")
    vout = torch.zeros(len(rows) * stride, dtype=torch.int32, device="cuda")
    C.centre_means(g, bi, table, hk, sb, 3, C.DOMAIN_CENTRE, out, stride, vout=vout)
    torch.cuda.synchronize()
    gb = out.cpu().numpy().reshape(len(rows), stride).astype(np.float64)
    vv = vout.cpu().numpy().view(np.uint32).reshape(len(rows), stride)
    allv = []
    for j, r in enumerate(rows):
        k = int(hk[r])
        k1 = np.zeros(B + 1, dtype=np.uint64)
        k1[r] = k
        s = O.sample(og, 2, 2, B, k1[:B], int(k1[B]), 3, dump_per_bin=k,
                     domain=C.DOMAIN_CENTRE, s_begin=int(sb[r]))
        assert (vv[j, :k] == s.v[r]).all(), r
        assert (gb[j, k:] == -1.0).all()          # nothing past the row's draws
        allv.append(s.v[r])
    ref = centre_gbar(og, theta, np.concatenate(allv))
    deg = og.degrees()
    assert deg[np.concatenate(allv)].max() > 32 or case == "chung_lu"
    err = max(abs(gb[j, i] - ref[int(vv[j, i])]) for j, r in enumerate(rows)
              for i in range(int(hk[r])))
    assert err < 2e-3, err


def test_centre_mean_is_the_exact_mean(c1):
    """E[gbar(v)] over centres drawn with probability p_v / p_b is the mean of
    g over the bin's wedges: the centre-draw average agrees with the census's
    exact mean within sampling error, per bin."""
    g, bi, og = c1
    B = bi.max_bins
    net = net_with(M.init_params(21))
    means = C.Census(g, bi).means(net)
    table = C.CentreTable(g, bi, net)
    rows = [r for r in range(B) if bi.h_p_b[r] > 0] + [B]
    k = 1 << 15
    hk = np.zeros(B + 1, dtype=np.uint64)
    hk[rows] = k
    out = torch.empty(len(rows) * k, dtype=torch.float32, device="cuda")
    C.centre_means(g, bi, table, hk, 0, 12, C.DOMAIN_CENTRE, out, k)
    gb = out.cpu().numpy().reshape(len(rows), k).astype(np.float64)
    for j, r in enumerate(rows):
        se = gb[j].std(ddof=1) / math.sqrt(k)
        assert abs(gb[j].mean() - means[r]) <= 5 * se + 2e-6, (r, gb[j].mean(), means[r], se)


def test_centre_cv_unbiased(c1):
    """The centre-draw control variate over repeated seeds: its mean matches
    the exact c_b within a few standard errors on every row it is used on."""
    g, bi, og = c1
    B = bi.max_bins
    P = O.exact(og, 2, 2, B)
    rows = [r for r in range(B) if bi.h_p_b[r] > 0]
    tr = C.train(g, bi, rows, 200_000, seed=4, epochs=2, per_row_batch=256, lr=5e-3)
    table = C.CentreTable(g, bi, tr.net)
    ests = {r: [] for r in rows}
    R, n = 24, 1 << 12
    first = {r: n for r in rows}
    for sd in range(R):
        res = C.sequential(g, bi, rows, 1e-9, 1e-3, 500 + sd, tr.net, tr.beta, first=first,
                           max_per_row=n, centre=table, centre_first=first)
        for r in rows:
            assert res.aux_samples[r] == (n if tr.beta[r] != 0.0 else 0)
            ests[r].append(res.estimates[r])
    for r in rows:
        c_true = float(P[r, 1:].sum()) / float(bi.h_p_b[r])
        e = np.array(ests[r])
        se = max(e.std(ddof=1), 1e-6) / math.sqrt(R)
        assert abs(e.mean() - c_true) <= 3.5 * se + 1e-9, (r, e.mean(), c_true, se)
