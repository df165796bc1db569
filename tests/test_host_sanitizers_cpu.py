"""The library's host rules (host_rules.cpp) built with the host compiler under
AddressSanitizer and UndefinedBehaviorSanitizer and driven through valid and
invalid inputs (tests/sanitize/host_rules_driver.cpp): no leak, no
out-of-bounds access, no undefined behaviour, every expectation met."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2512_12151_amd", "csrc", "host_rules.cpp")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "host_rules_driver.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_host_rules_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_rules_asan")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", SRC, DRIVER, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
