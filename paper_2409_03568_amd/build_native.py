"""Build the HIP library libckks_mi355x.so in-tree for gfx950 (hipcc cross-compiles without a GPU)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libckks_mi355x.so")
SOURCES = ["api.cpp", "host_math.cpp", "k_ntt_dispatch.cpp", "k_ops.hip", "k_cache.hip", "server.cpp", "batch.cpp",
           "pipeline.cpp", "tune_file.cpp"] + ["k_ntt_%d_%s.hip" % (n, part) for n in (13, 12, 14, 11) for part in ("fused", "enc", "mul")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # host tables (cos, Gaussian CDF) must round exactly as written
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


def _up_to_date(src: str, obj: str) -> bool:
    """True when obj is newer than src and every header of the source tree."""
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "ckks_mi355x.h"))
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not force and _up_to_date(src, obj):
        return obj
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force=False: only those older than their inputs) and link."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 8, 16, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, force), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    # roctx: the named ranges around the C-ABI calls (see TraceRange)
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread",
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
