"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host planner (paper_1605_02178_amd/csrc/plan.cpp: coefficient fits in
binary128, conditioning, pivot plans, plane scales, parameter blocks,
recursive coefficients) and the plain-C oracle (oracle/c/oracle.c: the direct
filter of eq. 1 and the polynomial filter of Section II, with crops, radii
above the image side and degenerate shapes) are each built with g++/gcc and
-fsanitize=address,undefined into a small driver under tests/sanitize/ and
run; any sanitizer report aborts the driver.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, exe, tmp_path, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=str(tmp_path))
    if r.returncode != 0 and "sanitize" in r.stderr and "unrecognized" in r.stderr:
        pytest.skip("compiler without sanitizer support")
    assert r.returncode == 0, r.stderr[-2000:]
    e = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
             **(env or {}))
    r = subprocess.run([exe], capture_output=True, text=True, env=e, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout


def test_planner_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "plan_asan")
    out = _run(["g++", *SAN, "-std=gnu++17", "-I", os.path.join(ROOT, "paper_1605_02178_amd", "csrc"),
                os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"),
                os.path.join(ROOT, "paper_1605_02178_amd", "csrc", "plan.cpp"), "-lquadmath", "-o", exe],
               exe, tmp_path)
    assert "0 failed checks" in out


def test_oracle_c_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan")
    out = _run(["gcc", *SAN, "-std=c11", "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                os.path.join(ROOT, "oracle", "c", "oracle.c"), "-lm", "-o", exe], exe, tmp_path,
               env={"OMP_NUM_THREADS": "4"})
    assert "0 failed checks" in out
