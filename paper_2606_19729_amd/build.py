"""Builds libvoila.so (HIP kernels + C ABI) for gfx950 in-tree.

Each source compiles to an object in its own hipcc process (in parallel), and
the objects link into a shared library next to this file.  Packed FP32
instructions are disabled for the device code (-packed-fp32-ops is turned
off), the library is built at -O3 without fast-math and without implicit
contraction of multiply-adds (kernels that share device functions then round
identically; fused operations are written explicitly).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvoila.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["k_plan.hip", "k_plan_bf16.hip", "k_observe.hip", "k_search.hip", "k_nce.hip", "k_nce_grad.hip", "k_ddim.hip", "k_update.hip", "grad.hip",
           "resample_large.hip", "abi.hip"]
ARCH = os.environ.get("VOILA_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]
# Sources whose matrix instructions keep accumulators and results in VGPRs:
# their paired bfloat16 evaluations then hold the activations (B operands) in
# AGPRs and convert each finished accumulator pair with one AGPR write where
# the default form reads the pair out of AGPRs (measured faster for these
# two; the binary32 plan kernel, in k_plan.hip, and the contrastive scores
# kernels are not faster in that form).
VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
EXTRA = {"k_plan_bf16.hip": VGPR_FORM, "k_observe.hip": VGPR_FORM}


def _jobs():
    n = os.cpu_count() or 4
    cap = int(os.environ.get("MAX_JOBS", "16"))
    return max(1, min(n, cap, len(SOURCES)))


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(OBJ, exist_ok=True)
    base = ["hipcc", f"--offload-arch={ARCH}"] + FLAGS + ["-I", os.path.join(ROOT, "include")] + list(extra)

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = base + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    with concurrent.futures.ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [(s, r) for s, _, r in results if r.returncode != 0]
    for s, r in failed:
        sys.stderr.write(f"--- {s}\n" + r.stdout + r.stderr)
    if failed:
        raise RuntimeError("hipcc failed building libvoila.so: " + ", ".join(s for s, _ in failed))
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC"] + [o for _, o, _ in results] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libvoila.so failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
