"""Build step for the FP64 oracle library (test infrastructure only).

Compiles ``voila_oracle.c`` with gcc into ``liboracle.so`` next to it.  The
flags keep binary64 semantics plain: no fast-math, no contraction of a*b+c
into fused multiply-adds.  OpenMP only spreads independent rollouts and
particles over threads; every reduction runs afterwards in a fixed order, so
results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "voila_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
