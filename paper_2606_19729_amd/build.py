"""Builds libvoila.so (HIP kernels + C ABI) for gfx950 in-tree.

One hipcc invocation compiles the kernels and the ABI into a shared library
next to this file.  Packed FP32 instructions are disabled for the device code
(-packed-fp32-ops is turned off), the library is built at -O3 without fast-math
and without implicit contraction of multiply-adds (kernels that share device
functions then round identically; fused operations are written explicitly).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvoila.so")
SOURCES = ["kernels.hip", "grad.hip", "resample_large.hip", "abi.hip"]
ARCH = os.environ.get("VOILA_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include")]
    cmd += list(extra)
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libvoila.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
