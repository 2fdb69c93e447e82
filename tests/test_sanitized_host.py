"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: the oracle (liboracle, liboracle_mt) and the host side of every
translation unit of the library (argument checks, workspace and tuning
logic, the host backend) are rebuilt with both sanitizers (the library
without device code), and the CPU tests that exercise them -- the oracle's
pins, the C-ABI boundary checks, the host backend -- run against those builds
with the sanitizer runtime preloaded.  Any report fails the run."""
import os
import subprocess
import sys

import oracle
from paper_2309_03912_amd import build as hdc_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_asan_and_ubsan():
    lib = hdc_build.build_sanitized()
    olib, omt = oracle.build_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": hdc_build.asan_runtime(),
        # the interpreter and torch are not instrumented: no leak report for them
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "HDC_LIBRARY": lib,
        "HDC_ORACLE_LIBRARY": olib,
        "HDC_ORACLE_MT_LIBRARY": omt,
    })
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-s", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           "tests/test_oracle.py", "tests/test_boundary.py", "tests/test_host_side.py"]
    proc = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (proc.stdout + proc.stderr)[-4000:]
    assert proc.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in proc.stderr and "runtime error:" not in proc.stderr, tail
