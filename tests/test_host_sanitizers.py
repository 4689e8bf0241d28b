"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle/squeeze_oracle.c) is rebuilt with both sanitizers and the
  oracle pins (tests/test_oracle_pins.py) run against that build in a child
  process (libasan preloaded into the interpreter; leak checking off, since
  the interpreter itself is not instrumented).
* The library's host-only table builders (paper_2201_00613_amd/csrc/
  host_tables.cpp, compiled by g++ into libsqueeze as well) are built with
  both sanitizers together with a check program (tests/host/check_host_tables.cpp)
  that compares them with brute force on the CPU.

Any sanitizer report aborts the child (-fno-sanitize-recover), so a report is
a failed test.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _need_gcc():
    if not shutil.which("gcc") or not shutil.which("g++"):
        pytest.skip("gcc/g++ not available")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    return asan


def test_oracle_pins_under_sanitizers():
    asan = _need_gcc()
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "liboracle_san.so")
    subprocess.run(["gcc", *SAN, "-std=c11", "-fopenmp", "-fPIC", "-shared", os.path.join(ROOT, "oracle", "squeeze_oracle.c"),
                    "-o", lib], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", SQZ_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "passed" in res.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    # the instrumentation is live: a neighbour table with an index far past the end
    # (a planted mistake, on the CPU) makes the sanitized build abort with a report
    probe = ("import numpy as np, oracle\n"
             "O = oracle.Fractal(2, [(0, 0), (1, 0), (0, 1)], 6)\n"
             "nb = O.neighbour_table(); nb[5, 0] = 10 ** 9\n"
             "O.life_steps(O.fill_compact(1, 0.5), 1, nb)\n")
    res = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0 and "AddressSanitizer" in res.stderr, res.stderr[-2000:]


def test_host_table_builders_under_sanitizers():
    _need_gcc()
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "check_host_tables")
    csrc = os.path.join(ROOT, "paper_2201_00613_amd", "csrc")
    subprocess.run(["g++", *SAN, "-std=c++17", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "host", "check_host_tables.cpp"), os.path.join(csrc, "host_tables.cpp"),
                    "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, ASAN_OPTIONS="abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    assert "all checks passed" in res.stdout
