"""Build the CPU oracle (test infrastructure) with gcc.

FP rules: -O2 with fused multiply-add contraction disabled and no fast-math,
so every rounding follows the source; OpenMP parallelises over blocks.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["oracle.c", "oracle_cs.c", "oracle_amr.c"]


def build(verbose=False):
    tmp = f"{LIB}.tmp{os.getpid()}"      # per process: concurrent test workers may build at once
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=gnu11", "-Wall", "-Wno-unknown-pragmas",
           "-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + ["forward_body.inc", "oracle.h"]
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
