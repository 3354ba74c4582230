"""The library's host code (validation, planning, pass compilation,
bindings) under AddressSanitizer and UndefinedBehaviorSanitizer: a g++ build
of the host sources, linked with the device objects, drives
tests/sanitized_driver.py in a child process with the sanitizer runtime
preloaded.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2203_08826_amd import build as B
    lib = B.build_sanitized(verbose=False)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), asan
    env = dict(os.environ, LD_PRELOAD=asan, QSV_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_driver.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "sanitized host workout:" in r.stdout
