"""Builds libsbfwi.so (the HIP/gfx950 library behind the C ABI) in-tree.

    python -m paper_2501_06748_amd.build

Every HIP source is compiled with hipcc for gfx950 (packed FP32 instructions
disabled); the host-only dense kernels of the coarse factorisation are plain
C++ (g++, no fused multiply-add); both are linked into
paper_2501_06748_amd/libsbfwi.so.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsbfwi.so")
SOURCES = ["api.cpp", "mesh.cpp", "profiler.cpp", "factor.hip", "step.hip", "coarse.hip", "adjoint.hip",
           "direct.hip", "fem.hip", "lfe.hip"]
HOST_SOURCES = ["dense_host.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        if src in HOST_SOURCES:
            cmd = [shutil.which("g++") or "g++", *HOST_FLAGS, "-c"]
        else:
            cmd = [hipcc, *FLAGS, "-c"]
            if src.endswith(".cpp"):
                cmd += ["-x", "hip"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose:
            print("compiled", src, flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES + HOST_SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
