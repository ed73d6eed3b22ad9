"""Compile libgr (the HIP kernels and the C ABI) for gfx950 into
paper_2602_01057_amd/libgr.so with hipcc.

Packed FP32 instructions are disabled at the target-feature level
(-packed-fp32-ops); float atomics compile to hardware atomics
(-munsafe-fp-atomics).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgr.so")
SOURCES = ["gr_api.hip", "gr_build.hip", "gr_project.hip", "gr_rays.hip", "gr_tof.hip", "gr_volume.hip"]
ARCH = os.environ.get("GR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


LIB_SANITIZED = os.path.join(PKG, "_build", "libgr_host_sanitized.so")


def build(verbose: bool = False, extra=None, sanitize: bool = False) -> str:
    """Compile libgr. sanitize=True builds a second copy whose HOST code is
    instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (the
    device code is built as usually) into _build/, for the host-side ABI tests;
    it is loaded only with the sanitizer runtime preloaded."""
    out = LIB_SANITIZED if sanitize else LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O1" if sanitize else "-O3", "-std=c++17", "-fPIC", "-shared",
           "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC, "-o", tmp]
    if sanitize:
        cmd += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
                "-shared-libasan"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if extra:
        cmd += list(extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    args = sys.argv[1:]
    san = "--sanitize" in args
    print(build(verbose=True, extra=[a for a in args if a != "--sanitize"], sanitize=san))
