"""Build libhydro.so (HIP, gfx950) in-tree with hipcc.

FP rules: -ffp-contract=off so that no multiply-add is fused unless fma() is
written (the bit-reproducible evaluation order of the method), no fast-math.
Packed FP32 instructions are disabled.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhydro.so")
SOURCES = ["hydro_fwd.hip", "hydro_vjp.hip", "hydro_api.hip", "hydro_noalloc.hip"]
HEADERS = ["hydro_common.h", "hydro_kernels.h"]
ARCH = os.environ.get("HYDRO_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _obj(src):
    return os.path.join(CSRC, "_build", src.replace(".hip", ".o"))


def _compile(src, verbose):
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    cmd = ["hipcc", "-c"] + FLAGS + [os.path.join(CSRC, src), "-o", _obj(src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return r.stderr


def build(verbose=False, jobs=None):
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, err in zip(SOURCES, ex.map(lambda s: _compile(s, verbose), SOURCES)):
            if verbose and err.strip():
                print(f"[{src}]\n{err}", flush=True)
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + [_obj(s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "hydro.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
