"""The CPU oracle and the library's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and run on random and
edge-case inputs: no sanitizer report, every call returns what it should."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fopenmp"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def build_and_run(cmd, exe):
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    out = build_and_run(["gcc", "-std=c11", "-ffp-contract=off", *SAN, os.path.join(ROOT, "oracle", "mgs_oracle.c"),
                         os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm", "-o", exe], exe)
    assert "ok" in out


def test_host_ilp_under_sanitizers(tmp_path):
    exe = str(tmp_path / "ilp_driver")
    out = build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                         os.path.join(ROOT, "paper_2604_26799_amd", "csrc", "ilp.cpp"),
                         os.path.join(ROOT, "tests", "sanitize", "ilp_driver.cpp"), "-o", exe], exe)
    assert "ok" in out
