"""Build the HIP library libfmmlu.so for gfx950 with hipcc (in-tree).

Every source in csrc/ is compiled to an object in parallel, then linked into
paper_2201_07325_amd/libfmmlu.so. Packed-FP32 instructions are disabled for all device
code (-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfmmlu.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.cpp", "batch.cpp", "factor.cpp", "refine.cpp", "tree.cpp", "tune.cpp", "kernels_gen.hip", "kernels_la.hip",
           "kernels_solve.hip", "kernels_apply.hip", "kernels_blas1.hip", "kernels_far.hip", "kernels_gemm.hip"]
ARCH = os.environ.get("FMMLU_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
            "-Xclang", "-packed-fp32-ops", "-ffp-contract=fast", "-Wno-unused-result",
            "-Wno-unknown-warning-option"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [cc, *_flags(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if src == "tree.cpp":
            cmd.insert(1, "-ffp-contract=off")
        jobs.append((src, obj, cmd))

    def run(job):
        src, obj, cmd = job
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), max(1, (os.cpu_count() or 2)))) as ex:
        objs = list(ex.map(run, jobs))
    tmp = OUT + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
