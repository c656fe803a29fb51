"""Build libgfd.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgfd.so")
SOURCES = ["gfd_kernels.hip", "gfd_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


# the unit-counting build (measurement only): the same sources with the
# enumeration's unit counters compiled in
LIB_COUNT = os.path.join(PKG, "libgfd_count.so")


def _compile_jobs(out: str, extra, sub: str):
    bdir = os.path.join(PKG, "_build", sub)
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        jobs.append((obj, [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]))
    return out, jobs


def build(verbose: bool = False, counting: bool = True) -> str:
    """Compile every HIP source and link the shared library, and the
    unit-counting build beside it (always rebuilds; the compiles run in
    parallel)."""
    variants = [_compile_jobs(LIB, [], "main")]
    if counting:
        variants.append(_compile_jobs(LIB_COUNT, ["-DGFD_COUNT_UNITS"], "count"))
    procs = []
    for _, jobs in variants:
        for obj, cmd in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    for out, jobs in variants:
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs], "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
