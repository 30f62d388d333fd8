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
