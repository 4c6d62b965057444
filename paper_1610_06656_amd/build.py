"""Build libsmp.so (the C-ABI of include/smp.h) for gfx950 with hipcc.

    python -m paper_1610_06656_amd.build        # or build() from Python

Every source under csrc/ is compiled to an object in _build/ and linked into
paper_1610_06656_amd/libsmp.so, next to this file. Device code is compiled
with packed-FP32 instructions disabled.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsmp.so")
ARCH = os.environ.get("SMP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "server.cpp", "sketch.hip", "sketch_bf16.hip", "sketch_fp8.hip", "sketch_srht.hip", "sketch_sparse.hip", "sample.hip", "sample_multi.hip",
           "sort_scan.hip",
           "estimate.hip", "waltmin.hip", "baselines.cpp", "tune.cpp", "batch_group.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result", "-Wno-unused-value",
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src):
    hipcc = _hipcc()
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc, "-x", "hip", *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stderr}")
    return obj, res.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(jobs) as ex:
        outs = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in outs]
    if verbose:
        for src, (_, err) in zip(SOURCES, outs):
            warn = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if warn:
                print(f"[{src}]\n" + "\n".join(warn), file=sys.stderr)
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(_hipcc()))), "lib")
    # rocBLAS serves the LELA baseline's plain GEMM (the exact entries of A^T B)
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{rocm_lib}", "-lrocblas", f"-Wl,-rpath,{rocm_lib}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libsmp.so failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
