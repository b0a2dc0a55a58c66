"""The planner's host code (spec parsing and binding, GEMM view, family,
schedules, symbolic prediction) under AddressSanitizer and UBSan: random and
valid-by-construction specs from a seeded generator.  CPU only; built with g++
from the library's own sources."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1409_8608_amd", "csrc")


@pytest.fixture(scope="module")
def fuzz_bin(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("fuzz") / "host_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "host_fuzz.cpp"),
           os.path.join(CSRC, "spec.cpp"), os.path.join(CSRC, "family.cpp"), os.path.join(CSRC, "access.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in r.stderr.lower() and "cannot find" in r.stderr.lower():
            pytest.skip("sanitizer runtime not available")
        raise AssertionError(r.stderr[-2000:])
    return out


@pytest.mark.parametrize("seed", [11, 12])
def test_planner_under_sanitizers(fuzz_bin, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([fuzz_bin, str(seed), "20000"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    bound, members = [int(x) for x in r.stdout.replace(",", "").split()[1::2]]
    assert bound > 2000 and members > 10000
