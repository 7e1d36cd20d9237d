"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, g++) and driven through every mode on tiny channels by
oracle/sanitize_check.cpp: predictor-corrector with each kernel, EOS, AV
form and disk law, scheme 1, the axisymmetric form, and the building blocks
the pins call. The sanitizers abort on any out-of-bounds access, use after
free, signed overflow or other undefined behaviour; the driver also fails on
a non-finite state."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


@pytest.mark.slow
def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "sanitize_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE,
           os.path.join(ORACLE, "wcsph_oracle.cpp"), os.path.join(ORACLE, "sanitize_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitizer runs clean" in r.stdout
