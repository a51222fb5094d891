"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code (CPU only): the
host planner of the library (csrc/plan.cpp, g++, no device code) and the CPU oracle
(oracle/oracle.c, gcc), each driven by a small checking program in tests/sanitize/."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


def test_planner_under_sanitizers(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "plan_check")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
          os.path.join(ROOT, "tests", "sanitize", "plan_check.cpp"),
          os.path.join(ROOT, "paper_1901_07643_amd", "csrc", "plan.cpp"),
          f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib", "-o", exe])
    # the HIP runtime library is only linked for hipGetErrorString; its own start-up
    # allocations are not the planner's, so leak detection is off for this binary
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0")
    out = _run([exe], env)
    assert "0 failures" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c11", *SAN, "-pthread",
          os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    out = _run([exe], ENV)
    assert "0 failures" in out
