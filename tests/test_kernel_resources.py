"""Compiler resource report of every device kernel (host-only: hipcc
cross-compiles for gfx950 without a GPU).  No kernel may use per-lane scratch
memory: a tuple held in a runtime-indexed private array ends up there, and
every enumeration attempt then stores and reloads it through the memory
hierarchy.  The exceptions are the enumeration kernels' 8-wave form and the
candidate pulls, whose registers are capped at 64 per lane on purpose (more
waves in flight pay for a few spilled values); their spills stay small.  The
enumeration kernels must also keep enough waves per SIMD to hide the latency
of their random loads."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2608_02321_amd import build as B

KERNELS = os.path.join(B.CSRC, "gfd_kernels.hip")


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("ru") / "k.o"
    flags = [f for f in B.FLAGS if f != "-Wall"]
    r = subprocess.run([B.HIPCC, *flags, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
                        "-c", KERNELS, "-o", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+(.*?)\s+\[-Rpass-analysis", line)
        if not m:
            continue
        key, _, val = m.group(1).partition(":")
        if key == "Function Name":
            cur = val.strip()
            kernels[cur] = {}
        elif cur is not None:
            kernels[cur][key.strip()] = val.strip()
    assert kernels, "no resource remarks"
    return kernels


def _eight_wave(name):
    return "k_ext_run" in name and name.split("ELi")[-1].startswith("8E")


def test_no_kernel_uses_scratch(report):
    bad = {k: v.get("ScratchSize [bytes/lane]") for k, v in report.items()
           if v.get("ScratchSize [bytes/lane]") != "0" and not _eight_wave(k)
           and "k_filter_pull" not in k}
    assert not bad, bad


def test_filter_pulls_keep_eight_waves(report):
    pulls = {k: v for k, v in report.items() if "k_filter_pull" in k}
    assert len(pulls) == 2, list(report)
    for k, v in pulls.items():
        assert int(v["Occupancy [waves/SIMD]"]) == 8, k
        assert int(v["ScratchSize [bytes/lane]"]) <= 16, (k, v["ScratchSize [bytes/lane]"])


def test_eight_wave_form_spills_little(report):
    eight = {k: v for k, v in report.items() if _eight_wave(k)}
    assert len(eight) == 3, list(report)
    for k, v in eight.items():
        assert int(v["Occupancy [waves/SIMD]"]) == 8, k
        assert int(v["ScratchSize [bytes/lane]"]) <= 512, (k, v["ScratchSize [bytes/lane]"])
    # the forms a default choice runs: inner levels and the plain last level
    plain = [k for k in eight if "ILb1ELb1" not in k]
    for k in plain:
        assert int(eight[k]["ScratchSize [bytes/lane]"]) <= 128, k


def test_enumeration_occupancy(report):
    ext = {k: int(v["Occupancy [waves/SIMD]"]) for k, v in report.items() if "k_ext_run" in k}
    # inner levels, last level plain and probing ahead; each in its two forms
    assert len(ext) == 6, list(report)
    for k, occ in ext.items():
        assert occ >= 4, (k, occ)


FLOAT2_SAMPLE = r"""
#include <hip/hip_runtime.h>
__global__ void axpy2(const float2* __restrict__ x, float2* __restrict__ y, float a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 v = x[i], w = y[i];
    w.x = a * v.x + w.x; w.y = a * v.y + w.y; w.x += v.y; w.y *= v.x;
    y[i] = w;
  }
}
"""
PACKED_F32 = re.compile(r"\bv_pk_(fma|add|mul)_f32\b")


def _device_asm(src, flags, out):
    r = subprocess.run([B.HIPCC, *flags, "--cuda-device-only", "-S", str(src), "-o", str(out)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def test_packed_fp32_ops_are_off(tmp_path):
    """The build's target-feature flag keeps packed FP32 instructions out of
    device code: a float2 kernel compiled with the library's flags has none,
    the same kernel without the flag has them, and the library's kernels have
    none."""
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "f2.hip"
    src.write_text(FLOAT2_SAMPLE)
    flags = [f for f in B.FLAGS if f != "-Wall"]
    i = flags.index("-packed-fp32-ops")
    plain = flags[:i - 3] + flags[i + 1:]  # without -Xclang -target-feature -Xclang -packed-fp32-ops
    assert len(plain) == len(flags) - 4
    assert not PACKED_F32.search(_device_asm(src, flags, tmp_path / "with_flag.s"))
    assert PACKED_F32.search(_device_asm(src, plain, tmp_path / "without_flag.s"))
    assert not PACKED_F32.search(_device_asm(KERNELS, flags, tmp_path / "kernels.s"))
