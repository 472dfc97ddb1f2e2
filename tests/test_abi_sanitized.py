"""The C ABI's host-side argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): the library's host code is rebuilt
with both sanitizers (device code unchanged) and tests/test_abi.py runs
against that build in a child process with the sanitizer runtime preloaded.
Any sanitizer report aborts the child, which fails this test."""

import os
import subprocess
import sys

import pytest

from paper_2602_18741_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


def test_abi_validation_is_clean_under_asan_and_ubsan():
    lib = build.build(sanitize=True)
    env = dict(os.environ, HC_LIBRARY=lib, LD_PRELOAD=build.asan_runtime(),
               # the interpreter itself is not instrumented: its allocations
               # are not leak-checked; every other report aborts
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-p", "no:xdist",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
    assert " passed" in out
