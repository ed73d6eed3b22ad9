"""The host-side ABI checks (tests/test_abi.py) again, against a copy of libgr
whose host code is built with AddressSanitizer and UndefinedBehaviorSanitizer
(argument validation, size queries and workspace layout run with every
out-of-bounds access, use-after-free, overflow or misaligned access reported as
an error). Runs in a child process with the sanitizer runtime preloaded; no
GPU is needed."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def test_abi_checks_under_host_sanitizers():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm install")
    from paper_2602_01057_amd import build_lib
    lib = build_lib.LIB_SANITIZED
    if not os.path.exists(lib) or any(os.path.getmtime(os.path.join(build_lib.CSRC, s)) > os.path.getmtime(lib)
                                      for s in build_lib.SOURCES):
        build_lib.build(sanitize=True)
    undefined = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True).stdout
    assert "__asan_" in undefined and "__ubsan_" in undefined, "the library is not instrumented"
    env = dict(os.environ, LD_PRELOAD=rt, GR_LIB_PATH=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                        "-p", "no:cacheprovider", "-x"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
