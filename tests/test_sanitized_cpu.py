"""The CPU checks under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle's pins against a sanitizer build of the oracle, and the library's
host-side tests (argument checks, exports, the layer schedule) against a
build of the library whose host code is instrumented.  The two builds use
different sanitizer runtimes (gcc's for the oracle, clang's for the hipcc
build), so each runs in a process of its own with its runtime preloaded."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, files):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    return r.stdout


def test_oracle_pins_under_asan_ubsan():
    from oracle import build
    if not os.path.exists(build.SAN_LIB) or os.path.getmtime(build.SAN_LIB) < os.path.getmtime(build.SRC):
        build.build_sanitized()
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ub = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    files = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    out = _run({"ORACLE_LIB": build.SAN_LIB, "LD_PRELOAD": f"{rt}:{ub}"}, files)
    assert " passed" in out


def test_library_host_code_under_asan_ubsan():
    from paper_2109_14814_amd import build
    srcs = build.sources()
    if not os.path.exists(build.SAN_LIB) or os.path.getmtime(build.SAN_LIB) < max(map(os.path.getmtime, srcs)):
        build.build(sanitize=True)
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    files = [os.path.join(ROOT, "tests", f) for f in ("test_capi_load.py", "test_layers.py")]
    out = _run({"MSEARCH_LIB": build.SAN_LIB, "LD_PRELOAD": rts[0]}, files)
    assert " passed" in out
