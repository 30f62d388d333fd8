"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a JSON message and exit code 2; the options the profiles use exist."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_profile_options_exist():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--no-cv", "--no-cpu-baseline", "--triangles",
                "--calibrate-copy-gib", "--pmc-summarize", "--graph", "--scale", "--join",
                "--alloc-seeds", "--stream", "--no-hash", "--no-batch", "--calibrate-gather"):
        assert opt in r.stdout, opt


def test_csr_traffic_follows_the_counter_summary(tmp_path, monkeypatch):
    """roofline_csr.traffic comes from the stored counter summary only while
    the build's sources and the workload match it: first pass + (digit passes
    - 1) later passes + dedup, plus the edge histogram's read of 8 B per edge."""
    sys.path.insert(0, ROOT)
    import bench
    gb = 10 ** 9
    groups = {"k_os_pass_first": {"read_bytes": 40 * gb, "write_bytes": 70 * gb},
              "k_os_pass_later": {"read_bytes": 75 * gb, "write_bytes": 72 * gb},
              "k_dedup": {"read_bytes": 66 * gb, "write_bytes": 33 * gb}}
    path = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "pmc_file", lambda scale: str(path))

    class Args:
        scale, graph = 28, "rmat"

    m_in, K = 1 << 32, 72_208_588
    path.write_text(json.dumps({"csr_hash": bench.csr_hash(), "workload_K": K,
                                "groups": groups}))
    rf = {"digit_passes": 7, "sort_bytes": 1000 * gb}
    bench.csr_traffic(Args, rf, m_in, K, 350.0)
    want = 110 * gb + 6 * 147 * gb + 99 * gb + 8 * m_in
    assert rf["traffic"] == want
    assert abs(rf["traffic_GBps"] - want / 0.35 / 1e9) < 0.1
    assert rf["traffic_over_sort_bytes"] == round(want / (1000 * gb), 3)
    # another build's sources or another workload: no traffic
    for bad in ({"csr_hash": "0" * 16, "workload_K": K}, {"csr_hash": bench.csr_hash(),
                                                         "workload_K": K + 1}):
        path.write_text(json.dumps({**bad, "groups": groups}))
        rf = {"digit_passes": 7, "sort_bytes": 1000 * gb}
        bench.csr_traffic(Args, rf, m_in, K, 350.0)
        assert rf["traffic"] is None


def test_bins_roofline_bytes():
    sys.path.insert(0, ROOT)
    import bench
    rf = bench.bins_roofline(1 << 28, 5.0)
    assert rf["min_bytes"] == 20 * (1 << 28) and rf["pass_bytes"] == 37 * (1 << 28)
    assert abs(rf["achieved_pass"] - 37 * (1 << 28) / 5e-3 / 1e9) < 0.01
