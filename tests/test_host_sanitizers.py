"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's host side (argument checks, workspace sizes, the FP64 estimates, the
control-variate arithmetic and bounds, the triangle box statistics) is rebuilt
with both sanitizers, device code untouched, and the ABI tests run against that
build in a child process with the ASan runtime preloaded.  Any sanitizer report
fails the test.  No device work is launched."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_abi_tests_pass_under_host_sanitizers():
    rt = asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime in this ROCm install")
    from paper_1301_5887_amd import build as pb

    lib = pb.build(sanitize=True)
    env = dict(os.environ, WEDGE_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
