"""The FP64 reference built with the address and undefined-behaviour
sanitizers (host code only, g++), every entry point driven on small random
cases of all four geometries by tests/oracle_asan_driver.cpp: no invalid
memory access, leak or undefined operation may be reported."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_reference_is_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
               os.path.join(ROOT, "oracle", "oracle.cpp"),
               os.path.join(ROOT, "tests", "oracle_asan_driver.cpp"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
