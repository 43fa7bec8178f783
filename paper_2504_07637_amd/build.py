"""Build libboys.so (HIP, gfx950) in-tree.

    python -m paper_2504_07637_amd.build

Steps: regenerate csrc/boys_tables.inc from data/boys_coeffs.txt, then one hipcc call
that compiles csrc/boys_lib.hip (kernels, plans) and csrc/boys_serve.hip (serving loop)
into paper_2504_07637_amd/libboys.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(PKG, "libboys.so")
ARCH = os.environ.get("BOYS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # every + - * / sqrt stays one IEEE operation; fmas only where written
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def gen_tables() -> str:
    sys.path.insert(0, CSRC)
    try:
        import gen_tables  # noqa: E402  (the HIP side's own generator)
    finally:
        sys.path.pop(0)
    return gen_tables.main()


def build_lib(verbose: bool = False) -> str:
    gen_tables()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp,
           os.path.join(CSRC, "boys_lib.hip"), os.path.join(CSRC, "boys_serve.hip"), "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose=True))
