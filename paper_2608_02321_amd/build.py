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


# roctx: named host ranges per phase for profilers
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]

# the unit-counting build (measurement only): the same sources with the
# enumeration's unit counters compiled in
LIB_COUNT = os.path.join(PKG, "libgfd_count.so")


# the host-sanitized build (tests only): the host code of the API source with
# AddressSanitizer and UndefinedBehaviorSanitizer (device code as in the main
# build), linked with the main build's kernels; it loads under
# LD_PRELOAD=<ASAN_RUNTIME>
LIB_ASAN = os.path.join(PKG, "libgfd_asan.so")
SAN = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]
ASAN_RUNTIME = "/opt/rocm/llvm/lib/clang/22/lib/linux/libclang_rt.asan-x86_64.so"


def _compile_jobs(out: str, extra, sub: str, sources=SOURCES, link=()):
    bdir = os.path.join(PKG, "_build", sub)
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src in sources:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        jobs.append((obj, [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]))
    return out, jobs, list(link)


def build(verbose: bool = False, counting: bool = True, sanitized: bool = True) -> str:
    """Compile every HIP source and link the shared library, and the
    unit-counting and host-sanitized builds beside it (always rebuilds; the
    compiles run in parallel)."""
    variants = [_compile_jobs(LIB, [], "main")]
    if counting:
        variants.append(_compile_jobs(LIB_COUNT, ["-DGFD_COUNT_UNITS"], "count"))
    if sanitized:
        variants.append(_compile_jobs(LIB_ASAN, SAN, "asan", ["gfd_api.hip"],
                                      [os.path.join(PKG, "_build", "main", "gfd_kernels.o"),
                                       "-shared-libsan", *SAN[1:]]))
    procs = []
    for _, jobs, _ in variants:
        for obj, cmd in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    for out, jobs, link in variants:
        tmp = out + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs], *link, *LIBS,
               "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
