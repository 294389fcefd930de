"""The library's host-side logic (circulant frequency selection, the small
dense factorisations of the randomized SVD's host path, the overlap test of
pitched operands) built from its own source with a plain C++ compiler under
AddressSanitizer and UndefinedBehaviorSanitizer, and checked against brute
force (tests/host/host_logic_test.cpp).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_19308_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic_test")
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
    cmd = ["g++", *flags, "-I", CSRC, os.path.join(ROOT, "tests", "host", "host_logic_test.cpp"),
           os.path.join(CSRC, "host_logic.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
