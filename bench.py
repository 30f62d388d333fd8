"""Benchmark of the plain wedge-sampling path on one MI355X.

Workload: Graph500 R-MAT, scale 28, edge factor 16 (a, b, c, d = 0.57, 0.19,
0.19, 0.05), seed 7, ids relabelled by a seeded bijection: 2^28 vertices and
2^32 edge draws, the stand-in for the paper's largest Graph500 graph; degree
bins with tau = omega = 2; eps = delta = 1e-3, so k = 3,800,452 Hoeffding
samples per bin and for the global stream.  Synthetic, generated on the host,
uploaded to HBM before timing.  --scale 24 gives the smaller R-MAT workload.

One step = the whole path on that edge list: wedge_build_csr (degrees and
sorted adjacency), wedge_bin_counts (bins and sampling index),
wedge_sample_close (samples and exact closure tests), wedge_estimate
(FP64 summary), including the two small host reads the path needs (m, and
the per-bin wedge counts that decide which bins are sampled).

--graph bter runs the same step on a BTER-like community graph instead
(power-law target degrees with exponent --bter-gamma on [--bter-dmin,
--bter-dmax], dense blocks of d + 1 vertices of density 1/ln d, excess degree by
Chung-Lu; n = --bter-n).

After the timed steps, on the same graph: the estimator comparison (plain
Hoeffding, plain with empirical-Bernstein stopping, learned control variate),
the triangle sample, and the CPU oracle (all host threads, plus a one-thread
leg) whose rowptr/col, bins, class counts over every sample and first 2,048
samples of every row are compared element by element with the GPU's.  Then
the batched workload (512 R-MAT graphs in one captured pipeline) is timed.

Prints one JSON line.  value = closure checks per second of the whole step.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "closure checks/s + s per M edges at fixed CI; learned-CV vs plain samples"
PEAK_HBM_GBS = 8000.0
# bytes the sampler must read per sample besides its search: the centre's
# adjacency start (8), the two neighbour ids (8), the row bounds of the
# endpoint whose row is searched (16); the other endpoint's row bounds (16)
# only for a closed sample of a bin (its class needs both degrees); plus 4
# bytes per adjacency word the search reads (counted by the kernel).
BYTES_PER_SAMPLE = 32
BYTES_PER_CLOSED_BIN_SAMPLE = 16
BYTES_PER_PROBE = 4
# the per-check count of the hot-path table: the centre's vertex id (4), its
# row bounds (16), the two neighbour ids (8), both endpoints' row bounds (32),
# plus 4 bytes per adjacency word the search reads
TABLE_BYTES_PER_SAMPLE = 60
SAMPLER_SRC = os.path.join(ROOT, "paper_1301_5887_amd", "csrc", "sample.hip")
DUMP_PER_ROW = 2048


def pmc_file(scale: int) -> str:
    return os.path.join(ROOT, "profiles", f"sample_close_rmat_s{scale}_counters.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sampler_hash() -> str:
    h = hashlib.sha256()
    for p in (SAMPLER_SRC, os.path.join(ROOT, "paper_1301_5887_amd", "csrc", "rng.hpp")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def csr_hash() -> str:
    """Hash of the adjacency build's sources, kept with its counter summary
    (the counts stand for the build only while these files are unchanged)."""
    h = hashlib.sha256()
    for name in ("csr.hip", "radix.hip", "radix.hpp"):
        with open(os.path.join(ROOT, "paper_1301_5887_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def host_info() -> dict:
    """CPU model, memory and core counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"cpu_model": model, "mem_total_gib": mem, "nproc": affinity,
            "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--graph", choices=["rmat", "bter"], default="rmat")
    ap.add_argument("--bter-n", type=int, default=130_000_000)
    ap.add_argument("--bter-gamma", type=float, default=2.1)
    ap.add_argument("--bter-dmin", type=int, default=10)
    ap.add_argument("--bter-dmax", type=int, default=1_000_000)
    ap.add_argument("--scale", type=int, default=28)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--delta", type=float, default=1e-3)
    ap.add_argument("--max-bins", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-one-thread-per-row", type=int, default=1 << 16,
                    help="samples per row of the oracle's one-thread leg")
    ap.add_argument("--triangles", type=int, default=5_000_000,
                    help="wedges of the global stream for the triangle sample (0: skip)")
    ap.add_argument("--alloc-seeds", type=int, default=0,
                    help="compare the Phase 2a allocation sampler with the i.i.d. one over "
                         "this many seeds (0: skip)")
    ap.add_argument("--stream", action="store_true",
                    help="also run the streamed path (edge list in host memory, no adjacency "
                         "on the device) on the step graph's simple edge list")
    ap.add_argument("--join", action="store_true",
                    help="also test the step's wedges by a join against the edge list "
                         "streamed from host memory")
    ap.add_argument("--no-cv", action="store_true",
                    help="skip the plain-EB / learned-CV comparison")
    ap.add_argument("--cv-train", type=int, default=10_000_000)
    ap.add_argument("--cv-repeats", type=int, default=3,
                    help="timed runs of the estimator comparison after one warm-up run; "
                         "each estimator's time is the median over them")
    ap.add_argument("--no-hash", action="store_true",
                    help="skip the closure-by-edge-table leg")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched workload (512 R-MAT graphs)")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="after timing, run one device copy of this size (counter calibration)")
    ap.add_argument("--calibrate-gather", type=int, default=0,
                    help="after timing, gather one 4-byte word from each of this many "
                         "distinct random 128-byte lines of a 16 GiB array (counter "
                         "calibration for random loads)")
    ap.add_argument("--pmc-summarize", nargs="+", metavar="DIR",
                    help="write the sampler's and the sort's HBM traffic and L2 hit rate from "
                         "rocprofv3 --pmc runs of this bench (each with --calibrate-copy-gib "
                         "and --calibrate-gather), one directory per run")
    ap.add_argument("--pmc-k", type=int, default=0, help="closure checks of the profiled run")
    ap.add_argument("--pmc-copy-gib", type=float, default=1.0)
    ap.add_argument("--pmc-gather", type=int, default=0)
    ap.add_argument("--pmc-out", default=None, help="summary file (default: the workload's)")
    return ap.parse_args()


def main():
    args = parse_args()
    if args.pmc_summarize:
        pmc_summarize(args.pmc_summarize, args.pmc_k, args.pmc_copy_gib, args.pmc_gather,
                      args.pmc_out or pmc_file(args.scale))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: every box here has one "
                                   "GPU, so --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_1301_5887_amd.synth import gen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    if args.graph == "bter":
        n = args.bter_n
        src, dst = gen.bter(n, args.bter_gamma, args.bter_dmin, args.bter_dmax, args.seed,
                            progress=log)
        workload = (f"BTER-like, n {n}, degree power law {args.bter_gamma:g} on "
                    f"[{args.bter_dmin}, {args.bter_dmax}], seed {args.seed}")
    else:
        n, src, dst = gen.rmat_graph500(args.scale, args.edgefactor, args.seed)
        workload = (f"R-MAT scale {args.scale}, edgefactor {args.edgefactor}, "
                    f"Graph500 (0.57,0.19,0.19,0.05), seed {args.seed}")
    log(f"[bench] generated {workload}: n={n} m_in={len(src)} in {time.time() - t0:.1f}s")

    out, cpu = plain_workload(args, torch, n, src, dst, workload)
    out["cpu_baseline"] = cpu
    del src, dst
    gc.collect()
    torch.cuda.empty_cache()
    out["batch"] = None if args.no_batch else batch_block(args, torch)
    print(json.dumps(out))


def plain_workload(args, torch, n, src, dst, workload):
    """The timed steps and everything measured on the same graph; returns
    (the JSON line without the batch block, cpu_baseline)."""
    from paper_1301_5887_amd import wedge as W

    d_src = torch.from_numpy(src.view(np.int32)).cuda()
    d_dst = torch.from_numpy(dst.view(np.int32)).cuda()
    m_in = len(src)
    B = args.max_bins
    k = W.hoeffding_k(args.eps, args.delta)
    dev = d_src.device
    lib = W.lib()
    stream = torch.cuda.current_stream()

    # all buffers allocated once, outside the timed region
    ws = W.Workspace(dev)
    ws.get(max(int(lib.wedge_build_csr_workspace(m_in, n)), int(lib.wedge_bin_counts_workspace(n))))
    rowptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(2 * m_in, dtype=torch.int32, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    n_b = torch.empty(B, dtype=torch.int64, device=dev)
    p_b = torch.empty(B, dtype=torch.int64, device=dev)
    index = W._empty_bytes(int(lib.wedge_index_bytes(n, m_in, B)), dev)
    q = torch.empty((B + 1) * 4, dtype=torch.int64, device=dev)
    probe = torch.empty(1, dtype=torch.int64, device=dev)
    h_info = torch.empty(2, dtype=torch.int64, pin_memory=True)
    h_nb = torch.empty(B, dtype=torch.int64, pin_memory=True)
    h_pb = torch.empty(B, dtype=torch.int64, pin_memory=True)
    h_q = torch.empty((B + 1) * 4, dtype=torch.int64, pin_memory=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]

    def step():
        wbuf = ws.buf
        ev[0].record(stream)
        W._check(lib.wedge_build_csr(W._ptr(d_src), W._ptr(d_dst), m_in, n, W._ptr(rowptr),
                                     W._ptr(col), W._ptr(info), W._ptr(wbuf), wbuf.numel(),
                                     W._stream()))
        ev[1].record(stream)
        h_info.copy_(info)
        m = int(h_info[0])
        if m < 0:
            raise RuntimeError("wedge_build_csr: the sort gave up waiting between tiles")
        W._check(lib.wedge_bin_counts(W._ptr(rowptr), n, m, 2, 2, B, W._ptr(n_b), W._ptr(p_b),
                                      W._ptr(index), index.numel(), W._ptr(wbuf), wbuf.numel(),
                                      W._stream()))
        ev[2].record(stream)
        h_nb.copy_(n_b)
        h_pb.copy_(p_b)
        pb = h_pb.numpy().view(np.uint64)
        hk = W.k_for_bins(pb, k)
        kg = k if int(pb.sum()) > 0 else 0
        ev[3].record(stream)
        W._check(lib.wedge_sample_close(W._ptr(rowptr), W._ptr(col), n, m, W._ptr(index), B,
                                        hk.ctypes.data_as(W._vp), kg, args.seed, 0, W._ptr(q),
                                        W._ptr(probe), None, 0, W._stream()))
        ev[4].record(stream)
        h_q.copy_(q)
        bi = W.BinIndex(n=n, m=m, tau=2, omega=2, max_bins=B, n_b=n_b, p_b=p_b, index=index,
                        h_n_b=h_nb.numpy().view(np.uint64).copy(), h_p_b=pb.copy())
        est = W.estimate(bi, h_q.numpy().view(np.uint64).copy(), hk, kg, args.delta)
        torch.cuda.synchronize()
        times = {"build_csr": ev[0].elapsed_time(ev[1]), "bin_counts": ev[1].elapsed_time(ev[2]),
                 "sample_close": ev[3].elapsed_time(ev[4])}
        return m, hk, kg, est, times

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i} done")
    torch.cuda.synchronize()
    phase = {"build_csr": [], "bin_counts": [], "sample_close": []}
    # no garbage-collection pass inside a timed region (a full pass of this
    # process takes tens of ms)
    gc.collect()
    gc.disable()
    t_start = time.perf_counter()
    for i in range(args.steps):
        m, hk, kg, est, times = step()
        for kx, vx in times.items():
            phase[kx].append(vx)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    gc.enable()
    log(f"[bench] timed {args.steps} steps in {t_total:.3f}s")
    del d_src, d_dst            # the edge list stays on the host for the oracle
    ms_step = 1000.0 * t_total / args.steps
    K = int(hk.sum()) + kg
    st_ix = W.index_status(W.BinIndex(n=n, m=m, tau=2, omega=2, max_bins=B, n_b=n_b, p_b=p_b,
                                      index=index))
    if st_ix["overflow"] or st_ix["mismatch"] or st_ix["empty_bin_samples"]:
        raise RuntimeError(f"index status after the timed steps: {st_ix}")
    probes = int(W.to_host_u64(probe)[0])
    avg = {kx: float(np.mean(vx)) for kx, vx in phase.items()}
    q_step = h_q.numpy().view(np.uint64).reshape(B + 1, 4).copy()

    roofline = sampler_roofline(args, K, q_step, probes, avg["sample_close"])
    roofline_csr = csr_roofline(n, m_in, m, avg["build_csr"])
    csr_traffic(args, roofline_csr, m_in, K, avg["build_csr"])
    roofline_bins = bins_roofline(n, avg["bin_counts"])
    # the streaming ceiling (left out of counter runs, whose calibration copy
    # must be the only large copy)
    stream = stream_copy_rate(torch, dev) if args.calibrate_copy_gib <= 0 else None
    roofline["stream_copy_GBps"] = roofline_csr["stream_copy_GBps"] = stream
    if stream and roofline.get("traffic_GBps_at_this_launch_time"):
        roofline["frac_of_stream_copy"] = round(roofline["traffic_GBps_at_this_launch_time"] /
                                                stream, 4)
    if stream:
        roofline_csr["frac_sort_of_stream_copy"] = round(roofline_csr["achieved_sort"] / stream, 4)
        roofline_bins["frac_pass_of_stream_copy"] = round(roofline_bins["achieved_pass"] / stream,
                                                          4)

    if args.calibrate_copy_gib > 0:
        nbytes = int(args.calibrate_copy_gib * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nbytes} bytes done")
        del a, b
    if args.calibrate_gather > 0:
        lines = 1 << 27                       # 16 GiB of int32 in 128-byte lines
        big = torch.ones(lines * 32, dtype=torch.int32, device=dev)
        idx = torch.randperm(lines, device=dev)[: args.calibrate_gather] * 32
        torch.cuda.synchronize()
        got = torch.index_select(big, 0, idx)
        torch.cuda.synchronize()
        log(f"[bench] calibration gather of {args.calibrate_gather} random lines done "
            f"(sum {int(got.sum().item())})")
        del big, idx, got
        torch.cuda.empty_cache()

    g = W.Csr(n=n, m=int(m), rowptr=rowptr, col=col)
    bi = W.BinIndex(n=n, m=int(m), tau=2, omega=2, max_bins=B, n_b=n_b, p_b=p_b,
                    index=index, h_n_b=h_nb.numpy().view(np.uint64).copy(),
                    h_p_b=h_pb.numpy().view(np.uint64).copy())
    cvcmp = None if args.no_cv else estimator_comparison(args, torch, g, bi, K,
                                                         avg["sample_close"])
    alloc = alloc_comparison(args, torch, W, g, bi, hk, kg, k) if args.alloc_seeds > 0 else None
    join = closure_join(args, torch, W, g, bi, hk, kg, src, dst) if args.join else None
    if args.stream:
        # the timed steps' workspace is not needed any more; the streamed leg
        # builds its edge list on the device and needs the room at scale 28
        ws.buf = None
        gc.collect()
        torch.cuda.empty_cache()
    streamed = stream_leg(args, torch, W, g, bi, k, kg, q_step) if args.stream else None
    tri = triangle_sample(args, torch, g, bi, est) if args.triangles > 0 else None
    hashp = None if args.no_hash else hash_probe(args, torch, W, g, bi, hk, kg, q_step,
                                                  avg["sample_close"], probes)

    cpu = None
    if not args.no_cpu_baseline:
        # the GPU's own samples for the element-wise comparison: the first
        # DUMP_PER_ROW of every row, from the same seed as the timed steps
        so = W.sample_close(g, bi, hk, kg, args.seed, dump_per_bin=DUMP_PER_ROW)
        gpu = {"q": q_step, "q_dump_run": W.to_host_u64(so.q).reshape(B + 1, 4),
               "dump": so.dump.view(B + 1, DUMP_PER_ROW, 4).cpu().numpy().view(np.uint32),
               "n_b": h_nb.numpy().view(np.uint64).copy(),
               "p_b": h_pb.numpy().view(np.uint64).copy(), "rowptr": rowptr, "col": col,
               "m": int(m), "est": [est.glob[x] for x in ("c", "t", "c_global", "t_global")]}
        del so
        cpu = cpu_baseline(args, torch, src, dst, n, B, k, hk, kg, workload, gpu)

    out = {
        "metric": METRIC,
        "value": K / (ms_step / 1000.0),
        "unit": "closure checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{workload}; tau=omega=2; eps=delta={args.eps:g}",
                   "n": n, "m": int(m), "m_in": m_in, "k_per_bin": k,
                   "bins_sampled": int((hk > 0).sum()), "k_global": kg, "closure_checks": K},
        "s_per_M_edges": (ms_step / 1000.0) / (m / 1e6),
        "s_per_M_edges_without_csr": ((ms_step - avg["build_csr"]) / 1000.0) / (m / 1e6),
        "sample_close_checks_per_s": K / (avg["sample_close"] / 1000.0),
        "phase_ms": {kx: round(vx, 4) for kx, vx in avg.items()},
        "roofline": roofline,
        "roofline_csr": roofline_csr,
        "roofline_bins": roofline_bins,
        "estimators": cvcmp,
        "triangle_sample": tri,
        "hash_probe": hashp,
        "closure_join": join,
        "streamed": streamed,
        "allocation_form": alloc,
        "estimates": {"c": est.glob["c"], "c_global": est.glob["c_global"], "t": est.glob["t"],
                      "t_global": est.glob["t_global"], "eps": est.glob["eps_global"]},
        "paper_context": "Hadoop, 32 nodes: 225 s + 0.33 s per million edges",
    }
    return out, cpu


def sampler_roofline(args, K, qh, probes, t_ms):
    """Roofline of the closure-probe kernel (k_sample_close) over the step's
    launch: algorithmic bytes per launch / the launch's HIP-event time."""
    B = qh.shape[0] - 1
    closed_bins = int(qh[:B, 1:].sum())
    alg_bytes = (BYTES_PER_SAMPLE * K + BYTES_PER_CLOSED_BIN_SAMPLE * closed_bins +
                 BYTES_PER_PROBE * probes)
    table_bytes = TABLE_BYTES_PER_SAMPLE * K + BYTES_PER_PROBE * probes
    t = t_ms / 1000.0
    achieved = alg_bytes / t / 1e9
    out = {"kernel": "k_sample_close", "bound": "hbm", "achieved": round(achieved, 2),
           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 5),
           "traffic": None, "algorithmic_bytes_per_launch": alg_bytes,
           "table_bytes_per_launch": table_bytes,
           "frac_table_bytes": round(table_bytes / t / 1e9 / PEAK_HBM_GBS, 5),
           "probe_loads": probes, "closed_bin_samples": closed_bins, "amplification": None,
           "kernel_ms": round(t_ms, 4)}
    pf = pmc_file(args.scale) if args.graph == "rmat" else None
    if pf and os.path.exists(pf):
        with open(pf) as f:
            pmc = json.load(f)
        if pmc.get("sampler_hash") == sampler_hash() and pmc.get("workload_K") == K:
            traffic = pmc.get("hbm_bytes_per_launch")
            out["traffic"] = traffic
            out["amplification"] = round(traffic / alg_bytes, 2) if traffic else None
            out["traffic_GBps_at_this_launch_time"] = round(traffic / t / 1e9, 1) if traffic else None
            # the HBM bytes the counters see over this launch time, against the peak
            out["frac_traffic"] = (round(traffic / t / 1e9 / PEAK_HBM_GBS, 5)
                                   if traffic else None)
            for key in ("l2_hit_rate", "request_mix", "traffic_by_requests"):
                if key in pmc:
                    out[key] = pmc[key]
    return out


def stream_copy_rate(torch, dev, gib: int = 4, reps: int = 5) -> float:
    """Achieved streaming bandwidth of this GPU: a device-to-device copy of
    `gib` GiB (read + write bytes per second, median of `reps` HIP-event timed
    copies on the current stream), the practical ceiling beside the 8 TB/s
    vendor peak."""
    nbytes = gib << 30
    a = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).fill_(1)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    b.copy_(a)
    times = []
    for _ in range(reps):
        ev[0].record(st)
        b.copy_(a)
        ev[1].record(st)
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / (float(np.median(times)) / 1e3) / 1e9, 1)


def bins_roofline(n, t_ms):
    """wedge_bin_counts against the HBM peak: the least bytes of a degree
    pass plus a counting sort of the vertices by degree (read rowptr, read
    the degrees and write the vertex order: 20 B per vertex), and the bytes
    of this build (the degree pass reads rowptr and writes the degree code
    and row word of every vertex; the pass by degree reads rowptr again and
    writes the order and each vertex's row start: 37 B per vertex; the sort
    of the few vertices of degree >= 255 is left out)."""
    t = t_ms / 1000.0
    least, ours = 20 * n, 37 * n
    return {"phase": "wedge_bin_counts", "bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "min_bytes": least, "achieved_min": round(least / t / 1e9, 2),
            "frac_min": round(least / t / 1e9 / PEAK_HBM_GBS, 5),
            "pass_bytes": ours, "achieved_pass": round(ours / t / 1e9, 2),
            "frac_pass": round(ours / t / 1e9 / PEAK_HBM_GBS, 5)}


def csr_traffic(args, rf, m_in, K, t_ms):
    """HBM bytes of one adjacency build from the stored counter summary (the
    first digit pass, the later passes, the dedup; the edge histogram's read
    of the 8 bytes of every input edge is added at its size, as it streams
    the list once), while the build's sources and the workload match it."""
    rf["traffic"] = None
    pf = pmc_file(args.scale) if args.graph == "rmat" else None
    if not (pf and os.path.exists(pf)):
        return
    with open(pf) as f:
        pmc = json.load(f)
    if pmc.get("csr_hash") != csr_hash() or pmc.get("workload_K") != K:
        return
    grp = pmc.get("groups", {})
    parts = [grp.get(x, {}) for x in ("k_os_pass_first", "k_os_pass_later", "k_dedup")]
    if not all("read_bytes" in p and "write_bytes" in p for p in parts):
        return
    first, later, dedup = (p["read_bytes"] + p["write_bytes"] for p in parts)
    traffic = first + (rf["digit_passes"] - 1) * later + dedup + 8 * m_in
    t = t_ms / 1000.0
    rf["traffic"] = traffic
    rf["traffic_GBps"] = round(traffic / t / 1e9, 1)
    rf["frac_traffic"] = round(traffic / t / 1e9 / PEAK_HBM_GBS, 5)
    rf["traffic_over_sort_bytes"] = round(traffic / rf["sort_bytes"], 3)


def csr_roofline(n, m_in, m, t_ms):
    """The CSR build's least bytes (read the edge list, write col and rowptr)
    and the bytes of this sort (histogram read of the edges; first pass reads
    the edges and writes two keys per edge; each later digit pass reads and
    writes every key, 6 or 8 bytes; the dedup reads the keys once and writes
    col and rowptr), against the phase time."""
    nkeys = 2 * m_in
    idbits = max(n - 1, 1).bit_length()
    digits = 2 * ((idbits + 7) // 8) if idbits <= 24 else (2 * idbits + 7) // 8
    kb = 6 if idbits <= 24 else 8
    csr_min = 8 * m_in + 4 * 2 * m + 8 * (n + 1)
    csr_sort = (8 * m_in + (8 * m_in + kb * nkeys) + (digits - 1) * 2 * kb * nkeys
                + kb * nkeys + 4 * 2 * m + 8 * (n + 1))
    t = t_ms / 1000.0
    return {"phase": "wedge_build_csr", "bound": "hbm", "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "digit_passes": digits, "key_bytes": kb,
            "min_bytes": csr_min, "achieved_min": round(csr_min / t / 1e9, 2),
            "frac_min": round(csr_min / t / 1e9 / PEAK_HBM_GBS, 5),
            "sort_bytes": csr_sort, "achieved_sort": round(csr_sort / t / 1e9, 2),
            "frac_sort": round(csr_sort / t / 1e9 / PEAK_HBM_GBS, 5)}


def estimator_comparison(args, torch, g, bi, K, t_sample_ms):
    from paper_1301_5887_amd import cv as CV

    # the first run pays one-time costs (kernel loading, buffer allocation);
    # the identical runs after it are timed, and each estimator reports the
    # run with its median time (its checks are the same in every run)
    runs = []
    for r in range(1 + max(args.cv_repeats, 1)):
        gc.collect()
        gc.disable()
        out = CV.compare(g, bi, eps=args.eps, delta=args.delta, seed=args.seed + 1000,
                         n_train=args.cv_train)
        gc.enable()
        if r > 0:
            runs.append(out)
        log(f"[bench] estimator comparison run {r} done")
    cvcmp = dict(runs[0])
    for name in ("train", "plain_eb", "learned_cv_centre", "learned_cv_exact_mean",
                 "learned_cv_aux"):
        if name in cvcmp:
            times = sorted(runs, key=lambda o: o[name]["seconds"])
            cvcmp[name] = times[len(times) // 2][name]
    cvcmp["timed_runs"] = len(runs)
    cvcmp["seconds_each_run"] = {
        name: [round(o[name]["seconds"], 6) for o in runs]
        for name in ("plain_eb", "learned_cv_centre", "learned_cv_exact_mean") if name in runs[0]}
    cvcmp["plain_hoeffding"] = {"closure_checks": K, "seconds": t_sample_ms / 1000.0}
    # the learned forms against the plain (Hoeffding) form at the same
    # interval; rows_with_cv says whether the network was used at all
    cvcmp["vs_plain_hoeffding"] = {
        name: {"fewer_closure_checks": cvcmp[name]["closure_checks"] < K,
               "less_wall_time": cvcmp[name]["seconds"] < t_sample_ms / 1000.0}
        for name in ("learned_cv_centre", "learned_cv_exact_mean") if name in cvcmp}
    lc = cvcmp["learned_cv_centre"]
    lx = cvcmp.get("learned_cv_exact_mean")
    log(f"[bench] estimator comparison: plain-Hoeffding {K} checks, plain-EB "
        f"{cvcmp['plain_eb']['closure_checks']}, learned-CV with centre draws "
        f"{lc['closure_checks']} (eval {lc['eval_checks']}, centre draws "
        f"{lc['centre_draws']}, {lc['seconds']:.4f} s)"
        + (f", learned-CV with exact mean {lx['closure_checks']} (eval "
           f"{lx['eval_checks']}, {lx['seconds']:.4f} s)" if lx else ""))
    return cvcmp


def alloc_comparison(args, torch, W, g, bi, hk, kg, k):
    """The paper's allocation (Alg. phase2a) against the i.i.d. draws at the
    same k: time of one sampling of every row, and the spread of the per-bin
    and global c estimates over independent seeds."""
    B = bi.max_bins
    aws = W.Workspace(g.rowptr.device)
    est_i, est_a, t_i, t_a = [], [], [], []
    for r in range(args.alloc_seeds + 1):
        sd = args.seed + 5000 + r
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        so = W.sample_close(g, bi, hk, kg, sd)
        qi = W.to_host_u64(so.q).reshape(B + 1, 4)
        t1 = time.perf_counter()
        sa, tot = W.sample_alloc(g, bi, hk, kg, sd, ws=aws)
        qa = W.to_host_u64(sa.q).reshape(B + 1, 4)
        t2 = time.perf_counter()
        if r == 0:
            continue        # the first round pays one-time costs
        t_i.append(t1 - t0)
        t_a.append(t2 - t1)
        est_i.append(qi[:, 1:].sum(axis=1) / np.maximum(np.append(hk, kg), 1))
        est_a.append(qa[:, 1:].sum(axis=1) / np.maximum(tot, 1).astype(np.float64))
    ei, ea = np.array(est_i), np.array(est_a)
    rows_s = [r for r in range(B + 1) if (r == B and kg) or (r < B and hk[r])]
    alloc = {"seeds": args.alloc_seeds, "k": k,
             "iid_ms": round(1e3 * float(np.median(t_i)), 3),
             "alloc_ms": round(1e3 * float(np.median(t_a)), 3),
             "per_row": {("global" if r == B else str(r)):
                         {"var_ratio_alloc_over_iid":
                          round(float(ea[:, r].var(ddof=1) / max(ei[:, r].var(ddof=1), 1e-30)), 4),
                          "mean_iid": float(ei[:, r].mean()), "mean_alloc": float(ea[:, r].mean())}
                         for r in rows_s}}
    log(f"[bench] allocation form: {alloc['alloc_ms']} ms per sampling (i.i.d. "
        f"{alloc['iid_ms']} ms) over {args.alloc_seeds} seeds")
    return alloc


def closure_join(args, torch, W, g, bi, hk, kg, src, dst):
    """Closure of the step's wedges by a join against the unsorted edge list
    streamed from pinned host memory (no adjacency used)."""
    B = bi.max_bins
    dpb = int(max(int(hk.max()), kg))
    so = W.sample_close(g, bi, hk, kg, args.seed, dump_per_bin=dpb)
    dmp = so.dump.view(B + 1, dpb, 4)
    rows_s = [r for r in range(B) if hk[r]] + ([B] if kg else [])
    recs = torch.cat([dmp[r, : (kg if r == B else int(hk[r]))] for r in rows_s])
    qa, qc = recs[:, 1].contiguous(), recs[:, 2].contiguous()
    closed_ref = int((recs[:, 3] > 0).sum().item())
    del so, dmp, recs
    hs = torch.from_numpy(src.view(np.int32)).pin_memory()
    hd = torch.from_numpy(dst.view(np.int32)).pin_memory()
    jws = W.Workspace(g.rowptr.device)
    for _ in range(2):          # the second, warm run is reported
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        closed = W.closure_join(qa, qc, hs, hd, ws=jws)
        torch.cuda.synchronize()
        t_join = time.perf_counter() - t0
    nclosed = int(closed.sum().item())
    m_in = len(src)
    join = {"queries": int(qa.numel()), "edges_streamed": m_in, "seconds": round(t_join, 5),
            "closure_checks_per_s": qa.numel() / t_join,
            "edge_stream_GBps": round(8 * m_in / t_join / 1e9, 2),
            "closed": nclosed, "closed_by_search": closed_ref}
    if nclosed != closed_ref:
        raise RuntimeError(f"closure join disagrees with the sampler: {join}")
    log(f"[bench] closure join: {qa.numel()} wedges against {m_in} streamed edges in "
        f"{t_join * 1e3:.1f} ms")
    return join


def simple_edges_to_host(torch, g, seed):
    """The graph's simple edge list (each edge once, u < w before a random
    flip of orientation) in random order, in pinned host memory.  Below 2^31
    edges the order is a random permutation; above (torch's masked selection
    and randperm stop there) the rows are taken in slices of at most 2^30
    entries and edge e goes to position (a e + b) mod m for an a prime to m,
    which scatters neighbouring edges across the list."""
    n, m = g.n, g.m
    dev = g.col.device
    gen_ = torch.Generator(device=dev)
    gen_.manual_seed(seed)
    ha = torch.empty(m, dtype=torch.int32, pin_memory=True)
    hb = torch.empty(m, dtype=torch.int32, pin_memory=True)
    if m < (1 << 31):
        deg = g.rowptr[1:] - g.rowptr[:-1]
        rows = torch.repeat_interleave(torch.arange(n, dtype=torch.int32, device=dev), deg)
        col = g.col[: 2 * m]
        keep = col > rows
        u, w = rows[keep], col[keep]
        del rows, col, keep, deg
        perm = torch.randperm(m, device=dev, generator=gen_)
        u, w = u[perm], w[perm]
        del perm
        flip = torch.rand(m, device=dev, generator=gen_) < 0.5
        ha.copy_(torch.where(flip, w, u))
        hb.copy_(torch.where(flip, u, w))
        return ha, hb
    mult = 1_000_003
    while math.gcd(mult, m) != 1:
        mult += 2
    shift = int(torch.randint(0, m, (1,), device=dev, generator=gen_).item())
    A = torch.empty(m, dtype=torch.int32, device=dev)
    Bv = torch.empty(m, dtype=torch.int32, device=dev)
    rp = g.rowptr
    v0, off = 0, 0
    while v0 < n:
        lim = torch.tensor([int(rp[v0].item()) + (1 << 30)], dtype=torch.int64, device=dev)
        v1 = int(torch.searchsorted(rp, lim, right=True).item()) - 1
        v1 = min(max(v1, v0 + 1), n)
        r0, r1 = int(rp[v0].item()), int(rp[v1].item())
        deg = rp[v0 + 1:v1 + 1] - rp[v0:v1]
        rows = torch.repeat_interleave(torch.arange(v0, v1, dtype=torch.int32, device=dev), deg)
        col = g.col[r0:r1]
        keep = col > rows
        u, w = rows[keep], col[keep]
        del rows, col, keep, deg
        cnt = u.numel()
        pos = (torch.arange(off, off + cnt, dtype=torch.int64, device=dev) * mult + shift) % m
        flip = torch.rand(cnt, device=dev, generator=gen_) < 0.5
        A[pos] = torch.where(flip, w, u)
        Bv[pos] = torch.where(flip, u, w)
        del u, w, pos, flip
        off += cnt
        v0 = v1
    assert off == m, (off, m)
    ha.copy_(A)
    hb.copy_(Bv)
    del A, Bv
    return ha, hb


def stream_leg(args, torch, W, g, bi, k, kg, q_step):
    """The step's samples by the streamed path: the graph's simple edge list
    (each edge once, random order and orientation) in pinned host memory,
    degrees, draws, gathered rows and the closure join all from passes over
    it, no adjacency on the device; its counts against the step's."""
    n, m = g.n, g.m
    ha, hb = simple_edges_to_host(torch, g, args.seed)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    B = bi.max_bins
    hk_req = np.full(B, k, dtype=np.uint64)
    cap = m   # half the edge ends per gather round
    ws = W.Workspace(g.col.device)
    runs = []
    out = None
    for _ in range(2):          # the second, warm run is reported
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = W.sample_stream(ha, hb, n, hk_req, kg, args.seed, 2, 2, B, gather_cap=cap, ws=ws)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    q = W.to_host_u64(out.q).reshape(B + 1, 4)
    K = int(out.h_k.sum()) + out.k_global
    passes = 2 + out.rounds   # the degree pass, one per gather round, the join
    res = {"edges": m, "host_bytes": 8 * m, "gather_cap": cap, "rounds": out.rounds,
           "edge_ends_gathered": out.gathered, "edge_passes": passes,
           "seconds": round(runs[-1], 4), "seconds_first_run": round(runs[0], 4),
           "closure_checks_per_s": K / runs[-1],
           "host_link_GBps": round(passes * 8 * m / runs[-1] / 1e9, 2),
           "counts_equal_search": bool((q == q_step).all())}
    log(f"[bench] streamed path: {K} checks over {passes} passes of {m} edges in "
        f"{runs[-1]:.3f} s, counts equal {res['counts_equal_search']}")
    del ha, hb, ws, out
    torch.cuda.empty_cache()
    return res


def hash_probe(args, torch, W, g, bi, hk, kg, q_step, t_search_ms, search_probes):
    """The closure test by lookup in an edge table instead of the search on
    the same graph and samples: the table's build time (HIP events, it is not
    part of the step), the sampler launch with it, its slots read per sample,
    and its counts against the step's."""
    stream = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    build, samp = [], []
    h = None
    for r in range(3):
        e[0].record(stream)
        h = W.edge_hash(g, table=None if h is None else h.table)
        e[1].record(stream)
        out = W.sample_close_hashed(g, bi, h, hk, kg, args.seed)
        e[2].record(stream)
        torch.cuda.synchronize()
        if r > 0:
            build.append(e[0].elapsed_time(e[1]))
            samp.append(e[1].elapsed_time(e[2]))
    qh = W.to_host_u64(out.q).reshape(q_step.shape)
    K = int(hk.sum()) + kg
    res = {"table_bits": h.bits, "table_bytes": 8 << h.bits, "load": round(g.m / (1 << h.bits), 4),
           "keys_without_slot": int(h.full.item()),
           "build_ms": round(float(np.median(build)), 3),
           "sample_close_ms": round(float(np.median(samp)), 4),
           "search_sample_close_ms": round(t_search_ms, 4),
           "slots_per_sample": round(int(out.probe_loads.item()) / K, 4),
           "search_words_per_sample": round(search_probes / K, 4),
           "counts_equal_search": bool((qh == q_step).all())}
    log(f"[bench] edge table: built in {res['build_ms']} ms, sampler {res['sample_close_ms']} ms "
        f"(search {res['search_sample_close_ms']} ms), counts equal {res['counts_equal_search']}")
    del h, out
    torch.cuda.empty_cache()
    return res


def triangle_sample(args, torch, g, bi, est):
    from paper_1301_5887_amd import triangles as TR

    for _ in range(2):      # the second, warm run is reported
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts = TR.sample(g, bi, args.triangles, args.seed, max_bins=bi.max_bins,
                       keep_triangles=False)
        t_tri = time.perf_counter() - t0
    log(f"[bench] triangle sample: {ts.count} triangles from {args.triangles} wedges "
        f"in {t_tri * 1e3:.2f} ms")
    return {"k": args.triangles, "triangles": ts.count,
            "expected_k_times_c_global": args.triangles * est.glob["c_global"],
            "seconds": round(t_tri, 5),
            "assortativity": [[r["min_bin"], r["count"], r["q1"], r["median"], r["q3"]]
                              for r in ts.box]}


def cpu_baseline(args, torch, src, dst, n, B, k, hk, kg, workload, gpu):
    """The oracle, as it stands, on the same graph: its adjacency and bins
    (all host threads), then every sample of every sampled row and of the
    global stream (all host threads; this is `value`), then the first
    samples of every row on one thread.  Its rowptr/col, n_b/p_b, class
    counts and first DUMP_PER_ROW samples per row are compared element by
    element with the GPU's."""
    from oracle import oracle as O

    threads = O.num_threads()
    hi = host_info()
    t0 = time.time()
    og = O.build_graph(src, dst, n, progress=log)
    t_graph = time.time() - t0
    log(f"[bench] oracle graph: m={og.m} in {t_graph:.1f}s ({threads} threads)")
    # adjacency, element by element, in 2^28-entry chunks of the GPU's arrays
    csr_match = og.m == gpu["m"]
    if csr_match:
        rp = gpu["rowptr"].cpu().numpy().view(np.uint64)
        csr_match = bool(np.array_equal(rp, og.rowptr))
        del rp
    if csr_match:
        step = 1 << 28
        for a in range(0, 2 * og.m, step):
            b = min(a + step, 2 * og.m)
            ch = gpu["col"][a:b].cpu().numpy().view(np.uint32)
            if not np.array_equal(ch, og.col[a:b]):
                csr_match = False
                break
    log(f"[bench] oracle adjacency compared with the GPU's: match={csr_match}")
    t1 = time.time()
    n_b, p_b = O.bins(og, 2, 2, B)
    t_bins = time.time() - t1
    bins_match = bool((n_b == gpu["n_b"]).all() and (p_b == gpu["p_b"]).all())
    kb = O.k_for_bins(p_b, k)
    kgo = k if int(p_b.sum()) > 0 else 0
    rows_match = bool((kb == hk).all()) and kgo == kg
    t1 = time.perf_counter()
    s = O.sample(og, 2, 2, B, kb, kgo, args.seed, dump_per_bin=DUMP_PER_ROW)
    dt = time.perf_counter() - t1
    Ks = int(kb.sum()) + kgo
    counts_match = bool((s.q == gpu["q"]).all() and (s.q == gpu["q_dump_run"]).all())
    dmp = gpu["dump"]
    samples_match = True
    samples_compared = 0
    for r in range(B + 1):
        kr = kgo if r == B else int(kb[r])
        c = min(kr, DUMP_PER_ROW)
        if c == 0:
            continue
        samples_compared += c
        gv = dmp[r, :c]
        if not (np.array_equal(gv[:, 0], s.v[r, :c]) and np.array_equal(gv[:, 1], s.a[r, :c])
                and np.array_equal(gv[:, 2], s.c[r, :c])
                and np.array_equal(gv[:, 3], s.cls[r, :c].astype(np.uint32))):
            samples_match = False
    log(f"[bench] oracle sampled {Ks} wedges in {dt:.2f}s ({threads} threads): counts match="
        f"{counts_match}, first {DUMP_PER_ROW} samples of every row match={samples_match}")
    # the estimate phase (Alg. phase4c, Eq. global_est) on the oracle's counts
    t1 = time.perf_counter()
    _, glob = O.estimate(p_b, s.q, kb, kgo, args.delta)
    t_est = time.perf_counter() - t1
    est_match = all(abs(a - b) <= 1e-12 * max(1.0, abs(b)) for a, b in zip(gpu["est"], glob))
    # one thread, the first samples of every row (the thread count is
    # process-wide, so it is set back afterwards)
    k1 = np.minimum(kb, np.uint64(args.cpu_one_thread_per_row)).astype(np.uint64)
    kg1 = min(kgo, args.cpu_one_thread_per_row)
    t1 = time.perf_counter()
    s1 = O.sample(og, 2, 2, B, k1, kg1, args.seed, nthreads=1)
    dt1 = time.perf_counter() - t1
    O.set_num_threads(threads)
    K1 = int(k1.sum()) + kg1
    one_match = bool((s1.q[:B][k1 == kb] == s.q[:B][k1 == kb]).all())
    del og, s, s1
    gc.collect()
    return {"value": Ks / dt, "unit": "closure checks/s", "cores": threads, "kind": "oracle",
            "sample": f"every sample of the timed step: {int((kb > 0).sum())} bins x {k} and "
                      f"the global stream ({Ks} checks) on the same graph ({workload}); "
                      f"the oracle's adjacency and bins are built first, not timed in value",
            "seconds": round(dt, 3),
            "one_thread": {"value": K1 / dt1, "checks": K1, "seconds": round(dt1, 3),
                           "sample": f"first {args.cpu_one_thread_per_row} samples of every row"},
            "csr_seconds": round(t_graph, 3), "csr_threads": threads,
            "bins_seconds": round(t_bins, 3),
            "estimate_seconds": round(t_est, 6),
            "host": hi,
            "estimates_match": est_match,
            "gpu_counts_match": counts_match, "csr_match": csr_match, "bins_match": bins_match,
            "sample_counts_match": rows_match, "samples_match": samples_match,
            "samples_compared": samples_compared, "one_thread_rows_match": one_match}


def batch_block(args, torch):
    """The batched workload: G R-MAT graphs (Graph500 parameters, scale in
    [10, 20] and edge factor in [8, 32] drawn from the batch seed, seeds
    100 + g), 20,000 samples per bin and per global stream, launch shape from
    the autotuner, the whole pipeline captured into one HIP graph; timed by
    HIP events around replays and around the sampling launch alone.  The
    per-graph parity of this workload is a GPU test."""
    from paper_1301_5887_amd import wedge as W
    from paper_1301_5887_amd.synth import gen

    G = args.batch_graphs
    t0 = time.time()
    shapes = gen.batch_shapes(G, seed=100)
    graphs = []
    for g, (s, ef) in enumerate(shapes):
        n, src, dst = gen.rmat_graph500(s, ef, seed=100 + g)
        graphs.append((n, src, dst))
    m_tot = sum(len(x[1]) for x in graphs)
    log(f"[bench] batch: {G} graphs, {m_tot} edges generated in {time.time() - t0:.1f}s")
    tau, omega, B, k, seed, delta = 2, 2, 24, 20_000, 5, 1e-3
    bt = W.Batch(graphs, tau=tau, omega=omega, max_bins=B, k_per_bin=k, k_global=k, seed=seed)
    del graphs
    bt.prepare()
    cands = [W.make_shape(4, 4096, 0), W.make_shape(2, 2048, 0), W.make_shape(8, 8192, 0),
             W.make_shape(4, 16384, 2048), W.make_shape(4, 4096, 1024)]
    best, ms = bt.autotune(cands, reps=2)
    h = bt.host()
    K = int(h["q"].sum())
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    samp = []
    for _ in range(3):
        e0.record(stream)
        bt.sample(best, delta=delta)
        e1.record(stream)
        torch.cuda.synchronize()
        samp.append(e0.elapsed_time(e1))
    bt.capture(best, delta=delta)
    bt.replay()
    torch.cuda.synchronize()
    rep = []
    for _ in range(3):
        e0.record(stream)
        bt.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        rep.append(e0.elapsed_time(e1))
    h2 = bt.host()
    same = bool((h2["q"] == h["q"]).all())
    bt.destroy_graph()
    t_rep, t_samp = float(np.median(rep)), float(np.median(samp))
    log(f"[bench] batch: replay {t_rep:.2f} ms, sampling launch {t_samp:.2f} ms, "
        f"{K} checks, autotuner pick ({best.lanes_in_flight}, {best.samples_per_tile}, "
        f"{best.workgroups})")
    del bt
    return {"graphs": G, "edges_in": m_tot, "k_per_bin": k, "closure_checks": K,
            "pipeline_replay_ms": round(t_rep, 3), "sampling_launch_ms": round(t_samp, 3),
            "checks_per_s_replay": K / (t_rep / 1000.0),
            "checks_per_s_sampling": K / (t_samp / 1000.0),
            "replay_counts_equal_eager": same,
            "autotune": {"candidates": [[c.lanes_in_flight, c.samples_per_tile, c.workgroups]
                                        for c in cands],
                         "ms": [round(x, 3) for x in ms],
                         "pick": [best.lanes_in_flight, best.samples_per_tile, best.workgroups]}}


PMC_COUNTERS = ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
                "TCC_EA0_RDREQ_128B_sum", "TCC_BUBBLE_sum", "TCC_EA0_RDREQ_DRAM_sum",
                "TCC_HIT_sum", "TCC_MISS_sum", "TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum",
                "TCC_REQ_sum", "TCC_READ_SECTORS_sum"]


def _pmc_dispatches(dirs):
    """{dispatch id: {"kernel": name, counter: value}} from rocprofv3 csv
    output of one or more runs (each run's dispatch ids are its own; runs of
    the same command dispatch the same kernels in the same order)."""
    import csv
    import glob
    runs = []
    for d in dirs:
        disp = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    e = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": r["Kernel_Name"]})
                    e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        runs.append(disp)
    return runs


def _pmc_groups(disp):
    """Dispatch ids of the kernels the summary covers, from the order of one
    bench run: the sampler launches of the timed steps (before the
    calibration copy), the adjacency sort's first and later digit passes and
    its dedup (later passes: those between a first pass and the next dedup),
    the calibration copy and the calibration gather."""
    ids = sorted(disp)
    name = {i: disp[i]["kernel"] for i in ids}
    copies = [i for i in ids if "copyBuffer" in name[i]]
    big = lambda i: max(v for k, v in disp[i].items() if k != "kernel")
    cal = max(copies, key=big) if copies else None
    g = {"k_sample_close": [], "k_os_pass_first": [], "k_os_pass_later": [], "k_dedup": [],
         "calibration_copy": [cal] if cal is not None else [], "calibration_gather": []}
    in_sort = False
    for i in ids:
        nm = name[i]
        if "k_sample_close" in nm and (cal is None or i < cal):
            g["k_sample_close"].append(i)
        elif "k_os_pass<true" in nm:
            g["k_os_pass_first"].append(i)
            in_sort = True
        elif "k_os_pass<false" in nm and in_sort:
            g["k_os_pass_later"].append(i)
        elif "k_dedup" in nm:
            g["k_dedup"].append(i)
            in_sort = False
        elif "gather" in nm.lower() and cal is not None and i > cal:
            g["calibration_gather"].append(i)
    if g["calibration_gather"]:
        g["calibration_gather"] = [max(g["calibration_gather"], key=big)]
    return g


def pmc_summarize(dirs, workload_k: int, copy_gib: float, gather_lines: int, out_path: str):
    """Per-launch L2-to-memory traffic, request sizes and L2 hit rate of the
    sampler and the adjacency sort from rocprofv3 --pmc runs (each run
    collects a few TCC counters; every run is the same bench command).
    Read bytes = 32 n32 + 64 n64 + 128 n128 from the request counts by size;
    the calibration copy (known size) and the calibration gather (known
    number of random lines) show how these counts relate to real traffic."""
    runs = _pmc_dispatches(dirs)
    merged = {}
    for disp in runs:
        grp = _pmc_groups(disp)
        for gname, gids in grp.items():
            for c in PMC_COUNTERS:
                vals = [disp[i][c] for i in gids if c in disp[i]]
                if vals:
                    merged.setdefault(gname, {})[c] = sum(vals) / len(vals)
                    merged[gname].setdefault("dispatches", len(gids))

    def derive(c):
        out = {k: c[k] for k in PMC_COUNTERS if k in c}
        if all(k in c for k in ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
                                "TCC_EA0_RDREQ_128B_sum")):
            out["read_bytes"] = (32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
                                 + 128 * c["TCC_EA0_RDREQ_128B_sum"])
            tot = c.get("TCC_EA0_RDREQ_sum")
            if tot:
                out["request_mix"] = {"32B": round(c["TCC_EA0_RDREQ_32B_sum"] / tot, 4),
                                      "64B": round(c["TCC_EA0_RDREQ_64B_sum"] / tot, 4),
                                      "128B": round(c["TCC_EA0_RDREQ_128B_sum"] / tot, 4)}
        if all(k in c for k in ("TCC_BUBBLE_sum", "TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum")):
            out["fetch_size_formula_bytes"] = (
                128 * c["TCC_BUBBLE_sum"] + 32 * c["TCC_EA0_RDREQ_32B_sum"]
                + 64 * (c["TCC_EA0_RDREQ_sum"] - c["TCC_BUBBLE_sum"] - c["TCC_EA0_RDREQ_32B_sum"]))
        if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c and c["TCC_HIT_sum"] + c["TCC_MISS_sum"]:
            out["l2_hit_rate"] = round(c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"]), 4)
        if "TCC_EA0_WRREQ_sum" in c and "TCC_EA0_WRREQ_64B_sum" in c:
            out["write_bytes"] = (32 * (c["TCC_EA0_WRREQ_sum"] - c["TCC_EA0_WRREQ_64B_sum"])
                                  + 64 * c["TCC_EA0_WRREQ_64B_sum"])
        if "TCC_READ_SECTORS_sum" in c:
            out["l2_read_request_bytes"] = 32 * c["TCC_READ_SECTORS_sum"]
        out["dispatches"] = c.get("dispatches")
        return out

    groups = {g: derive(c) for g, c in merged.items()}
    out = {"sampler_hash": sampler_hash(), "csr_hash": csr_hash(), "workload_K": workload_k,
           "groups": groups, "runs": [str(d) for d in dirs]}
    cal = groups.get("calibration_copy", {})
    factor = None
    if cal.get("read_bytes"):
        factor = copy_gib * (1 << 30) / cal["read_bytes"]
        out["copy_read_factor"] = round(factor, 4)
    gat = groups.get("calibration_gather", {})
    if gather_lines and gat.get("TCC_EA0_RDREQ_sum"):
        # the gather also streams its 8-byte index array (in 128-byte lines)
        idx_lines = 8 * gather_lines / 128
        out["gather_requests_per_random_line"] = round(
            (gat["TCC_EA0_RDREQ_sum"] - idx_lines) / gather_lines, 4)
        if gat.get("read_bytes"):
            out["gather_read_bytes_per_random_line"] = round(
                (gat["read_bytes"] - 8 * gather_lines) / gather_lines, 2)
    samp = groups.get("k_sample_close", {})
    if samp.get("read_bytes") is not None:
        rb = samp["read_bytes"] * (factor if factor else 1.0)
        wb = samp.get("write_bytes", 0.0)
        out["hbm_bytes_per_launch"] = rb + wb
        out["traffic_by_requests"] = {"read_bytes": rb, "write_bytes": wb,
                                      "scaled_by_copy_factor": factor is not None}
        if "request_mix" in samp:
            out["request_mix"] = samp["request_mix"]
        if "l2_hit_rate" in samp:
            out["l2_hit_rate"] = samp["l2_hit_rate"]
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
