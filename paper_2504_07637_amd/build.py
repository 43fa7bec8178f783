"""Build libboys.so (HIP, gfx950) in-tree.

    python -m paper_2504_07637_amd.build

Steps: regenerate csrc/boys_tables.inc from data/boys_coeffs.txt; compile, in parallel,
the host side (csrc/boys_lib.hip), the serving loop (csrc/boys_serve.hip), the plain
kernels once per precision class (csrc/plain_inst.hip) and the batched kernels once per
(n_max bucket, launch shape) (csrc/batched_inst.hip), the two-approximation kernels
(csrc/split_inst.hip), the consumer kernels (csrc/eri_inst.hip) and the allocation-free
batched entry point (csrc/boys_noalloc.hip) into objects under
_build/; link them into paper_2504_07637_amd/libboys.so.  BOYS_BUILD_JOBS caps the parallel compiles
(default: the CPU count, at most 16).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(PKG, "libboys.so")
BUILD_DIR = os.path.join(PKG, "_build")

CLASSES = (0, 1, 2, 3, 4)       # boys_precision values
BUCKETS = 5                     # n_max buckets of the batched kernels
# (schedule, K): persistent; one workgroup per tile of K * block; one wave per tile of K * 64
SHAPES = ((0, 0), (1, 1), (1, 2), (1, 4), (2, 4))
ARCH = os.environ.get("BOYS_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
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


def _units():
    """(object name, source, extra flags) of every translation unit."""
    # the largest kernels (high buckets, large K) take longest: start them first
    units = [(f"batched_b{b}_s{sc}_k{k}", "batched_inst.hip",
              [f"-DBOYS_BUCKET={b}", f"-DBOYS_SCHED={sc}", f"-DBOYS_K={k}"])
             for b in reversed(range(BUCKETS))
             for sc, k in sorted(SHAPES, key=lambda t: -t[1])]
    units += [(f"plain_c{c}", "plain_inst.hip", [f"-DBOYS_CLASS={c}"]) for c in CLASSES]
    units += [("split", "split_inst.hip", []), ("eri", "eri_inst.hip", [])]
    units += [("boys_lib", "boys_lib.hip", []), ("boys_serve", "boys_serve.hip", []),
              ("boys_noalloc", "boys_noalloc.hip", [])]
    return units


def _jobs() -> int:
    env = os.environ.get("BOYS_BUILD_JOBS")
    if env:
        return max(1, int(env))
    return max(1, min(os.cpu_count() or 1, 16))


def build_lib(verbose: bool = False) -> str:
    gen_tables()
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    base = [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC]

    def compile_one(unit):
        name, src, extra = unit
        obj = os.path.join(BUILD_DIR, name + ".o")
        cmd = [*base, *extra, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return obj, cmd, r.returncode, r.stdout

    units = _units()
    with cf.ThreadPoolExecutor(max_workers=_jobs()) as pool:
        results = list(pool.map(compile_one, units))
    failed = [(cmd, out) for _, cmd, rc, out in results if rc != 0]
    for cmd, out in failed:
        sys.stderr.write(" ".join(cmd) + "\n" + out + "\n")
    if failed:
        raise RuntimeError(f"{len(failed)} of {len(units)} HIP compiles failed")
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[obj for obj, _, _, _ in results], "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose=True))
