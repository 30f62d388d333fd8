"""Batched form on the GPU: every graph of a batch against the oracle run on
that graph alone (graph_id = its index), bit-exact counts and bins, device
estimates within 1e-12; HIP-graph replays equal to the eager run; counts
invariant under every launch shape the autotuner tries."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1301_5887_amd import wedge as W
from paper_1301_5887_amd.synth import gen

pytestmark = pytest.mark.gpu

REL = 1e-12


def mixed_graphs(seed=0, count=24):
    rng = np.random.default_rng(seed)
    graphs = []
    for i in range(count - 5):
        s = int(rng.integers(5, 13))
        ef = int(rng.integers(4, 17))
        n, src, dst = gen.rmat_graph500(s, ef, seed=1000 + i)
        graphs.append((n, src, dst))
    graphs.append((3, np.array([0, 1, 2], np.uint32), np.array([0, 1, 2], np.uint32)))  # loops only
    graphs.append((2, np.array([0], np.uint32), np.array([1], np.uint32)))            # no wedges
    graphs.append((41, np.zeros(40, np.uint32), np.arange(1, 41, dtype=np.uint32)))   # star
    e = np.array([(i, j) for i in range(9) for j in range(i + 1, 9)], dtype=np.uint32)
    graphs.append((9, e[:, 0], e[:, 1]))                                               # K_9
    bad_src = np.array([0, 1, 2, 70, 3], np.uint32)                                    # id 70 >= n
    bad_dst = np.array([1, 2, 0, 1, 1], np.uint32)
    graphs.append((5, bad_src, bad_dst))
    return graphs


def oracle_batch(graphs, tau, omega, B, k, kg, seed, delta):
    out = []
    for g, (n, src, dst) in enumerate(graphs):
        og = O.build_graph(src, dst, n)
        n_b, p_b = O.bins(og, tau, omega, B)
        kb = O.k_for_bins(p_b, k)
        kgg = kg if int(p_b.sum()) > 0 else 0
        s = O.sample(og, tau, omega, B, kb, kgg, seed, graph_id=g)
        per_bin, glob = O.estimate(p_b, s.q, kb, kgg, delta)
        out.append(dict(og=og, n_b=n_b, p_b=p_b, q=s.q, per_bin=per_bin, glob=glob))
    return out


def check_batch(h, ref, B):
    for g, r in enumerate(ref):
        assert (h["n_b"][g] == r["n_b"]).all(), g
        assert (h["p_b"][g] == r["p_b"]).all(), g
        assert (h["q"][g] == r["q"]).all(), (g, h["q"][g], r["q"])
        gl = h["est_glob"][g]
        for j in range(6):
            assert abs(gl[j] - r["glob"][j]) <= REL * max(1.0, abs(r["glob"][j])), (g, j)
        eb = h["est_bins"][g]
        for b in range(B):
            for j in range(3):
                x, y = eb[b, j], r["per_bin"][b, j]
                assert abs(x - y) <= REL * max(1.0, abs(y)), (g, b, j)


@pytest.fixture(scope="module")
def mixed():
    graphs = mixed_graphs()
    tau, omega, B, k, kg, seed, delta = 2, 2, 24, 3000, 2500, 17, 1e-3
    print(f"[batch] G={len(graphs)} B={B} k={k} kg={kg} seed={seed}", flush=True)
    ref = oracle_batch(graphs, tau, omega, B, k, kg, seed, delta)
    bt = W.Batch(graphs, tau=tau, omega=omega, max_bins=B, k_per_bin=k, k_global=kg, seed=seed)
    return graphs, ref, bt, B, delta


def test_batch_matches_oracle_per_graph(mixed):
    graphs, ref, bt, B, delta = mixed
    bt.run(delta=delta)
    torch.cuda.synchronize()
    h = bt.host()
    check_batch(h, ref, B)
    # adjacency of a few graphs, in local ids
    for g in (0, 3, len(graphs) - 2):
        rp, col = bt.csr_of(g)
        assert (rp == ref[g]["og"].rowptr).all() and (col == ref[g]["og"].col).all()


@pytest.mark.parametrize("shape", [(1, 256, 256), (2, 1024, 64), (4, 4096, 0), (8, 2048, 1024),
                                   (4, 512, 3)])
def test_batch_launch_shape_invariance(mixed, shape):
    graphs, ref, bt, B, delta = mixed
    bt.prepare()
    bt.sample(W.make_shape(*shape), delta=delta)
    torch.cuda.synchronize()
    check_batch(bt.host(), ref, B)


def test_batch_graph_capture_replays(mixed):
    graphs, ref, bt, B, delta = mixed
    bt.capture(W.make_shape(4, 2048, 512), delta=delta)
    for rep in range(3):
        bt.q.zero_()
        bt.est_glob.zero_()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        x = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        bt.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        check_batch(bt.host(), ref, B)
    bt.destroy_graph()


def test_batch_autotune_picks_a_candidate(mixed):
    graphs, ref, bt, B, delta = mixed
    bt.prepare()
    cands = [W.make_shape(4, 4096, 0), W.make_shape(1, 512, 256), W.make_shape(2, 2048, 1024),
             W.make_shape(8, 8192, 2048)]
    best, ms = bt.autotune(cands, reps=2)
    assert len(ms) == 4 and all(t > 0 for t in ms)
    assert best in cands
    h = bt.host()
    q_ref = h["q"]
    for g, r in enumerate(ref):
        assert (q_ref[g] == r["q"]).all()


def test_batch_graph500_recipe_reduced_scales():
    """The batch recipe (scales and edge factors drawn per graph from the
    batch seed) with scales 6..12 so the oracle covers all 512 graphs."""
    shapes = gen.batch_shapes(512, seed=100, smin=6, smax=12, emin=8, emax=32)
    graphs = []
    for g, (s, ef) in enumerate(shapes):
        n, src, dst = gen.rmat_graph500(s, ef, seed=100 + g)
        graphs.append((n, src, dst))
    tau, omega, B, k, seed, delta = 2, 2, 20, 1500, 5, 1e-3
    print(f"[batch512] G=512 B={B} k={k}", flush=True)
    bt = W.Batch(graphs, tau=tau, omega=omega, max_bins=B, k_per_bin=k, k_global=k, seed=seed)
    bt.capture(None, delta=delta)
    bt.replay()
    torch.cuda.synchronize()
    h = bt.host()
    ref = oracle_batch(graphs, tau, omega, B, k, k, seed, delta)
    check_batch(h, ref, B)
    bt.destroy_graph()


FULL_CHUNKS = 8


@pytest.fixture(scope="module")
def full_recipe():
    """The batched workload at its full size: 512 R-MAT graphs (Graph500
    parameters, scales 10..20 and edge factors 8..32 drawn from the batch
    seed, seeds 100..611), 20,000 samples per bin and per global stream, the
    launch shape picked by the autotuner, the whole pipeline captured into
    one HIP graph and replayed.  Returns the graphs and the replay's
    per-graph results (host copies; the device batch is released)."""
    import time
    shapes = gen.batch_shapes(512, seed=100)
    graphs = []
    for g, (s, ef) in enumerate(shapes):
        n, src, dst = gen.rmat_graph500(s, ef, seed=100 + g)
        graphs.append((n, src, dst))
    m_tot = sum(len(x[1]) for x in graphs)
    tau, omega, B, k, seed, delta = 2, 2, 24, 20_000, 5, 1e-3
    print(f"[batch-full] G=512 edges={m_tot} B={B} k={k}", flush=True)
    bt = W.Batch(graphs, tau=tau, omega=omega, max_bins=B, k_per_bin=k, k_global=k, seed=seed)
    bt.prepare()
    cands = [W.make_shape(4, 4096, 0), W.make_shape(2, 2048, 0), W.make_shape(8, 8192, 0),
             W.make_shape(4, 16384, 2048), W.make_shape(4, 4096, 1024)]
    best, ms = bt.autotune(cands, reps=2)
    print(f"[batch-full] autotune ms={['%.3f' % t for t in ms]} best={best.lanes_in_flight},"
          f"{best.samples_per_tile},{best.workgroups}", flush=True)
    bt.capture(best, delta=delta)
    bt.q.zero_()
    torch.cuda.synchronize()
    bt.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.replay()
    torch.cuda.synchronize()
    print(f"[batch-full] one replay of the whole pipeline: {time.perf_counter() - t0:.4f} s",
          flush=True)
    h = bt.host()
    bt.destroy_graph()
    del bt
    torch.cuda.empty_cache()
    return dict(graphs=graphs, h=h, tau=tau, omega=omega, B=B, k=k, seed=seed, delta=delta)


@pytest.mark.parametrize("chunk", range(FULL_CHUNKS))
def test_batch_full_recipe_oracle(full_recipe, chunk):
    """Every graph of the full-size batch (this chunk's 64 of the 512)
    against the oracle run on that graph alone: n_b, p_b and q bit-exact,
    the device's FP64 estimates within 1e-12."""
    F = full_recipe
    graphs, h, B, k = F["graphs"], F["h"], F["B"], F["k"]
    per = len(graphs) // FULL_CHUNKS
    lo, hi = chunk * per, (chunk + 1) * per if chunk < FULL_CHUNKS - 1 else len(graphs)
    print(f"[batch-full] oracle graphs {lo}..{hi - 1}", flush=True)
    for g in range(lo, hi):
        n, src, dst = graphs[g]
        og = O.build_graph(src, dst, n)
        n_b, p_b = O.bins(og, F["tau"], F["omega"], B)
        kb = O.k_for_bins(p_b, k)
        kgg = k if int(p_b.sum()) > 0 else 0
        s = O.sample(og, F["tau"], F["omega"], B, kb, kgg, F["seed"], graph_id=g)
        per_bin, glob = O.estimate(p_b, s.q, kb, kgg, F["delta"])
        assert (h["n_b"][g] == n_b).all() and (h["p_b"][g] == p_b).all(), g
        assert (h["q"][g] == s.q).all(), g
        for j in range(6):
            assert abs(h["est_glob"][g][j] - glob[j]) <= REL * max(1.0, abs(glob[j])), (g, j)
        eb = h["est_bins"][g]
        for b in range(B):
            for j in range(3):
                x, y = eb[b, j], per_bin[b, j]
                assert abs(x - y) <= REL * max(1.0, abs(y)), (g, b, j)
