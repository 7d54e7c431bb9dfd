"""Build libmsearch.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

Every source is compiled with FP contraction off (each FP64 operation
rounds once, as written) except where a kernel opts in locally with
`#pragma clang fp contract(fast)` (the Runge-Kutta map), and with packed
FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmsearch.so")
SOURCES = ["mesh.hip", "small_sort.hip", "search.hip", "rk8.hip", "refine.hip", "layers.hip", "pertbp.hip", "spectral.hip", "fourier_taylor.hip"]
ARCH = os.environ.get("MSEARCH_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-I", INCLUDE]


# Host-side checker build for the CPU sanitizer run (tests/test_sanitized_cpu.py):
# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the
# argument checks, planning and layouts); the device code is built as usual.
SAN_LIB = os.path.join(HERE, "libmsearch_san.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, jobs: int = 4, sanitize: bool = False) -> str:
    objs = []
    procs = []
    extra = HOST_SAN if sanitize else []
    out = SAN_LIB if sanitize else LIB
    tag = ".san.o" if sanitize else ".o"
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + tag)
        cmd = ["hipcc", *[f for f in FLAGS if f != "-shared"], *extra, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s}")
    for p, s in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra, *objs, "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
