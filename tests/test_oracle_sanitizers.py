"""The oracle's C library built with AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only, gcc) and run through a driver that calls every exported
function on all three sample formats, including rejected arguments.  A
memory error, an overflow or a mismatch between the oracle's own routes fails
the test."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    src = [os.path.join(ROOT, "oracle", "gnss_oracle.c"), os.path.join(ROOT, "tests", "csrc", "oracle_san_driver.c")]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-Wall", "-o", exe] + src + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "ERROR" not in res.stderr and "runtime error" not in res.stderr, res.stderr
    assert "all checks passed" in res.stdout
