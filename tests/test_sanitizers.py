"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the oracle's pins run against a sanitized build of the oracle, and the host
ABI checks run against the library built with its host code sanitized
(libgfd_asan.so; device code cannot be sanitized here).  Either run fails on
the first report: a heap or stack overflow, a use after free, a signed
overflow, a misaligned or null access, a shift out of range."""
import os
import subprocess
import sys

import pytest

from paper_2608_02321_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("AddressSanitizer", "UndefinedBehaviorSanitizer", "runtime error")


def _pytest_under(preload, env_extra, test_file, tmp_path):
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", **env_extra)
    log = tmp_path / "run.log"
    with open(log, "w") as f:
        # -s: a sanitizer report goes to the process's own stderr, uncaptured
        rc = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:xdist",
                             "-p", "no:cacheprovider", os.path.join(ROOT, "tests", test_file)],
                            cwd=ROOT, env=env, stdout=f, stderr=subprocess.STDOUT,
                            timeout=600).returncode
    out = log.read_text()
    assert rc == 0 and not any(r in out for r in REPORTS), out[-3000:]
    assert " passed" in out, out[-2000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-shared", "-fPIC",
                    "-pthread", os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(lib)], check=True)
    rt = [subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True,
                         check=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    _pytest_under(":".join(rt), {"GFD_ORACLE_LIB": str(lib)}, "test_oracle_pins.py", tmp_path)


def test_host_abi_under_asan_ubsan(tmp_path):
    if not os.path.exists(B.LIB_ASAN):
        pytest.fail("libgfd_asan.so is not built (paper_2608_02321_amd/build.py builds it)")
    if not os.path.exists(B.ASAN_RUNTIME):
        pytest.skip("clang's ASan runtime is not installed")
    _pytest_under(B.ASAN_RUNTIME, {"GFD_LIBRARY": B.LIB_ASAN}, "test_abi_host.py", tmp_path)
