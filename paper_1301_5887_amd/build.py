"""Build libwedge.so (hipcc, gfx950) in-tree.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection turned off and no floating-point contraction (the FP64 estimates
must round exactly as written).  build(sanitize=True) makes a second, checking
build under _build/san: the host code compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (each flag behind -Xarch_host, so no device code is
instrumented), for the host-sanitizer test only.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwedge.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["abi.cpp", "radix.hip", "csr.hip", "bins.hip", "sample.hip", "batch.hip", "mlp.hip",
           "census.hip", "triangles.hip", "join.hip", "cv_est.cpp", "validate.hip", "hash.hip", "stream.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]
FLAGS = ["-O3", *COMMON]
SAN_DIR = os.path.join(BUILD_DIR, "san")
SAN_LIB = os.path.join(SAN_DIR, "libwedge_san.so")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_FLAGS = ["-O1", "-g", *COMMON, *SAN_HOST]


def _compile(src: str, flags=FLAGS, out_dir: str = BUILD_DIR) -> str:
    out = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *flags, "-c", "-o", out]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd.append(os.path.join(CSRC, src))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    flags, out_dir, lib = (SAN_FLAGS, SAN_DIR, SAN_LIB) if sanitize else (FLAGS, BUILD_DIR, LIB)
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, flags, out_dir), SOURCES))
    tmp = lib + ".tmp"
    link = SAN_HOST if sanitize else []
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *link, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
