"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host code -- the binned-SAH builder, the 4-wide collapse and
  the serving pool allocator -- built with g++ -fsanitize=address,undefined
  together with tests/sanitize/host_checks.cpp, which builds trees over
  random and degenerate scenes and checks their invariants, and runs a
  random allocation sequence through the pool allocator.
* The C oracle built the same way, with the oracle pin tests run against it
  in a child Python process (the sanitizer runtime preloaded).
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_01304_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    path = subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def test_host_code_under_asan_ubsan(tmp_path):
    _runtime("libasan.so")
    exe = tmp_path / "host_checks"
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                           os.path.join(CSRC, "bvh_build.cpp"), os.path.join(CSRC, "bvh_wide.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks passed" in r.stdout


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", *SAN, "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
                           "-o", str(lib), os.path.join(ROOT, "oracle", "hrpp_oracle.c")])
    env = dict(os.environ, HRPP_ORACLE_LIB=str(lib), LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       capture_output=True, text=True, timeout=900, env=env, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-4000:] + r.stderr[-4000:])
    assert "passed" in r.stdout
