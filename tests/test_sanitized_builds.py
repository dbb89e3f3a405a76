"""Host-only builds of the oracle (oracle/dss_oracle.c), of the planner (csrc/plan.cpp, the HIP
pipeline replaced by stubs) and of the autotuner's result file (csrc/tune_cache.cpp), plainly and
under AddressSanitizer/UBSan, each driven by a small checker in tests/cpp (oracle: output against
its stable sort and the trace's bookkeeping over many random inputs; planner: every geometry
inside the plan's workspace, regions disjoint, Section 4's bound for the chosen (L, s); tuning
file: round trips and replacement by key)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPP = os.path.join(ROOT, "tests", "cpp")
FLAGS = {"plain": [], "asan-ubsan": ["-fsanitize=address,undefined",
                                     "-fno-sanitize-recover=undefined"]}


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "runtime error" not in r.stderr, r.stderr


@pytest.mark.parametrize("mode", sorted(FLAGS))
def test_oracle_sanitized(tmp_path, mode):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-Wall", *FLAGS[mode],
                           os.path.join(CPP, "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "dss_oracle.c"), "-o", exe])
    _run(exe)


@pytest.mark.parametrize("mode", sorted(FLAGS))
def test_planner_sanitized(tmp_path, mode):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "plan_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-pthread", *FLAGS[mode],
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1002_4464_amd", "csrc"),
                           os.path.join(CPP, "plan_check.cpp"),
                           os.path.join(ROOT, "paper_1002_4464_amd", "csrc", "plan.cpp"),
                           "-o", exe])
    _run(exe)


@pytest.mark.parametrize("mode", sorted(FLAGS))
def test_tune_cache_sanitized(tmp_path, mode):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tune_cache_test")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall", *FLAGS[mode],
                           "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1002_4464_amd", "csrc"),
                           os.path.join(CPP, "tune_cache_test.cpp"),
                           os.path.join(ROOT, "paper_1002_4464_amd", "csrc", "tune_cache.cpp"),
                           "-o", exe])
    _run(exe, str(tmp_path))
