"""Build libhsweep.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled to an object in parallel, then the objects are
linked into paper_1007_4290_amd/libhsweep.so.

Usage: python -m paper_1007_4290_amd.build
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhsweep.so")

SOURCES = ["api.hip", "k_coeff.hip", "k_factor.hip", "k_factor_f64.hip", "k_sweep.hip", "k_sweep_a.hip",
           "k_sweep_b.hip", "k_sweep_c.hip", "k_sweep_g4.hip", "k_krylov.hip"]

ARCH = ["--offload-arch=gfx950"]
FLAGS = ARCH + [
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay disabled in every device compile
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    env = os.environ.get("HIPCC")
    if env:
        return env
    if os.path.exists("/opt/rocm/bin/hipcc"):
        return "/opt/rocm/bin/hipcc"
    return "hipcc"


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, res


def build(verbose=False, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, res in ex.map(lambda s: _compile(s, verbose), SOURCES):
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + ARCH + ["-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libhsweep.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
