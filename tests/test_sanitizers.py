"""AddressSanitizer + UndefinedBehaviorSanitizer builds on the CPU: the oracle
(oracle/ddo.c, plain and OpenMP builds) driven through every routine by
tests/asan/oracle_driver.c, and the library's host planning code
(csrc/dd_host.cpp) driven by tests/asan/host_driver.cpp.  Each build must exit 0 with no sanitizer report.
Only host compilers are used (gcc / g++); nothing here runs on a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _run(cmd_build, exe, tmp_path):
    r = subprocess.run(cmd_build, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, r.stdout + r.stderr
    # a library preloaded by the environment may come before the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
    return out


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_sanitizers(openmp, tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wno-unknown-pragmas", *SAN,
           *(["-fopenmp"] if openmp else []),
           os.path.join(ROOT, "oracle", "ddo.c"), os.path.join(ROOT, "tests", "asan", "oracle_driver.c"),
           "-lm", "-o", exe]
    out = _run(cmd, exe, tmp_path)
    assert "0 failures" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_planning_under_sanitizers(tmp_path):
    """The library's host-only planning code (csrc/dd_host.cpp: work split and
    Gauss-Legendre rule) driven by tests/asan/host_driver.cpp, which checks
    the plan invariants on many instance layouts."""
    exe = str(tmp_path / "host_asan")
    csrc = os.path.join(ROOT, "paper_2005_02498_amd", "csrc")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", *SAN, "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "dd_host.cpp"), os.path.join(ROOT, "tests", "asan", "host_driver.cpp"), "-o", exe]
    out = _run(cmd, exe, tmp_path)
    assert " 0 failures" in out
