"""Build libfpde.so (HIP kernels for gfx950 + host planner) in-tree with hipcc.

Usage: python -m paper_2302_02863_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfpde.so")
ARCH = os.environ.get("FPDE_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable"]
# device code: no hand-written or auto-generated packed FP32 instructions
HIP_FLAGS = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-munsafe-fp-atomics"]
# host planner: structure-deciding arithmetic must not be contracted into FMAs
HOST_FLAGS = ["-ffp-contract=off"]

SOURCES = [
    ("fpde_kernels.hip", HIP_FLAGS),
    ("fpde_near.hip", HIP_FLAGS),
    ("fpde_apply.hip", HIP_FLAGS),
    ("fpde_far1.hip", HIP_FLAGS),
    ("fpde_multi.hip", HIP_FLAGS),
    ("fpde_batched.hip", HIP_FLAGS),
    ("fpde_solve.hip", HIP_FLAGS),
    ("fpde_adjoint.hip", HIP_FLAGS),
    ("fpde_noalloc.hip", HIP_FLAGS),
    ("fpde_recompress.hip", HIP_FLAGS),
    ("fpde_host.cpp", HOST_FLAGS),
    ("fpde_plan.cpp", HOST_FLAGS),
    ("fpde_recompress.cpp", HOST_FLAGS),
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [hipcc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + flags
        jobs.append(cmd)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
        return r.stderr

    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        for err in ex.map(run, jobs):
            if verbose and err:
                print(err)
    tmp = LIB + ".tmp"
    run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
