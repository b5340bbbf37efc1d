"""The serving scheduler's host logic (csrc/serve_core.hpp: arena, resident-factor
LRU, admission, stage machine, refinement decisions) under a fake executor and
clock, compiled with g++ and run under AddressSanitizer and
UndefinedBehaviorSanitizer.  No device is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_1812_02056_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serve_core_under_sanitizers(tmp_path):
    exe = str(tmp_path / "serve_core_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Wall", "-Wextra",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-I", INC, SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "all checks passed" in res.stdout
