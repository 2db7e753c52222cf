"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
oracle/asan_driver.c runs build, matvec, GMRES, export and free on edge
cases (one point, ragged and deep trees, cell-boundary points, zero
tolerance, duplicates, bad sizes); any invalid access, leak or undefined
operation makes the sanitized run fail."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = tmp_path / "orc_asan"
    src = [os.path.join(ROOT, "oracle", "h2d_oracle.c"), os.path.join(ROOT, "oracle", "asan_driver.c")]
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           *src, "-o", str(exe), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp_path / "o.h2dx")], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert "sanitizer driver done" in r.stdout
