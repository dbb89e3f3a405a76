"""Host-only tests of the served-stream scheduler (admission by memory, continuous batching,
failure paths, a multi-threaded stream): compiles tests/cpp/server_core_test.cpp with g++
against the scheduler header, plain and under AddressSanitizer/UBSan and ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "server_core_test.cpp")
INC = os.path.join(ROOT, "paper_1002_4464_amd", "csrc")


@pytest.mark.parametrize("flags", [[], ["-fsanitize=address,undefined"], ["-fsanitize=thread"]],
                         ids=["plain", "asan-ubsan", "tsan"])
def test_scheduler_core(tmp_path, flags):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sct")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-Wall", *flags,
                           "-I", INC, SRC, "-o", exe])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "WARNING" not in r.stderr, r.stderr
