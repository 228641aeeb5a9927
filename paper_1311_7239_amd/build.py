"""Build the gfx950 HIP library libmrtlbm.so in-tree with hipcc.

Usage: python -m paper_1311_7239_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import pathlib
import subprocess
import sys

PKG = pathlib.Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libmrtlbm.so"
SOURCES = ["lbm_kernels.hip", "lbm_adjoint.hip", "lbm_abi.cpp"]

# -ffp-contract=off: every kernel variant (single domain, batch, schedules)
# evaluates the per-node arithmetic with the same rounding, which is what
# makes batched and single-domain results bitwise equal.
# -packed-fp32-ops: keep the compiler from forming packed FP32 instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> pathlib.Path:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    build_dir = PKG / "_build"
    build_dir.mkdir(exist_ok=True)
    procs = []
    # the translation units compile concurrently (one hipcc process each)
    for src in SOURCES:
        path = CSRC / src
        if not path.exists():
            continue
        obj = build_dir / (src + ".o")
        cmd = [hipcc, *FLAGS, "-x", "hip", "-I", str(ROOT / "include"), "-I", str(CSRC), "-c", str(path),
               "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(str(obj))
    failed = [cmd for cmd, proc in procs if proc.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
