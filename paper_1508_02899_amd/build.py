"""Build the HIP library liblattice.so in-tree for gfx950.

Each .hip source under csrc/ is compiled separately (in parallel) with
hipcc, then linked into paper_1508_02899_amd/liblattice.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "liblattice.so")
ARCH = os.environ.get("LATTICE_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    subprocess.check_call(["hipcc", *FLAGS, "-c", src, "-o", obj],
                          stderr=subprocess.STDOUT)
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip"))
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = SO + ".tmp"
    # rocBLAS: the plain GEMM of the 2D structure function (s1.hip)
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared",
                           "-fPIC", "-o", tmp, *objs, "-lrocblas"])
    os.replace(tmp, SO)
    if verbose:
        print("built", SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
