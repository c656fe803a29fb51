"""Host check of the leaf postponement count (no GPU): the library's
inclusion-exclusion over set partitions of the leaves, compiled for the host
from the same header the kernels use, equals a brute-force count of injective
leaf assignments over random small candidate sets, for one, two and three
leaves; and stays exact for list sizes near 2^32, where 64-bit products would
overflow."""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2608_02321_amd import build as B

SRC = r"""
#include "gfd_internal.h"
#include <cstdio>
int main() {
  int r;
  while (std::scanf("%d", &r) == 1) {
    int64_t c[gfd::LEAF_SUBSETS] = {};
    for (int b = 1; b < (1 << r); b++) std::scanf("%lld", (long long*)&c[b]);
    const __int128 v = gfd::leaf_injective(r, c);
    const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)(v >> 64);
    std::printf("%llu %llu\n", hi, lo);
  }
}
"""


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    if not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("leaf")
    src, exe = d / "leaf.cpp", d / "leaf"
    src.write_text(SRC)
    r = subprocess.run([B.HIPCC, f"-I{B.CSRC}", "-O2", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, cases):
    inp = "".join(f"{r} " + " ".join(str(c[b]) for b in range(1, 1 << r)) + "\n" for r, c in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    vals = []
    for line in out.split("\n")[:len(cases)]:
        hi, lo = (int(t) for t in line.split())
        v = (hi << 64) | lo
        vals.append(v - (1 << 128) if hi >> 63 else v)
    return vals


def _counts(sets):
    r = len(sets)
    return [len(set.intersection(*[sets[j] for j in range(r) if b >> j & 1])) if b else 0
            for b in range(1 << r)]


def test_matches_brute_force(prog):
    rng = np.random.default_rng(7)
    cases, want = [], []
    for _ in range(300):
        r = int(rng.integers(1, 4))
        n = int(rng.integers(0, 9))
        sets = [set(int(v) for v in np.nonzero(rng.random(n) < rng.random())[0]) for _ in range(r)]
        cases.append((r, _counts(sets)))
        want.append(sum(1 for t in itertools.product(*[sorted(s) for s in sets])
                        if len(set(t)) == r))
    assert _run(prog, cases) == want


def test_large_lists_stay_exact(prog):
    # three identical lists of 2^32 - 5 members: n (n - 1) (n - 2), past 2^64
    n = (1 << 32) - 5
    c = [0] + [n] * 7
    assert _run(prog, [(3, c), (2, c[:4]), (1, c[:2])]) == [n * (n - 1) * (n - 2), n * (n - 1), n]
