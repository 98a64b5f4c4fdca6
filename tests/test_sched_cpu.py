"""The serving scheduler's policies on the CPU: builds tests/sched_test.cpp
(the scheduler header with a stand-in executor) with g++ and runs it, and
again under ThreadSanitizer with LLVM's clang++ (GCC 11's ThreadSanitizer
runtime does not intercept pthread_cond_clockwait, which timed condition
waits use, and reports false races there)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "sched_test.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1004_0014_amd", "csrc")]


CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(tmp_path, extra, cxx="g++"):
    exe = str(tmp_path / "sched_test")
    cc = subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-pthread", "-Wall", "-Werror", *extra,
                         *INC, SRC, "-o", exe], capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_scheduler_policies(tmp_path):
    _build_and_run(tmp_path, [])


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no LLVM clang++")
def test_scheduler_policies_tsan(tmp_path):
    probe = subprocess.run([CLANG, "-fsanitize=thread", "-x", "c++", "-", "-o", str(tmp_path / "p")],
                           input="int main(){}", capture_output=True, text=True)
    if probe.returncode != 0:
        pytest.skip("no ThreadSanitizer runtime")
    r = _build_and_run(tmp_path, ["-fsanitize=thread"], CLANG)
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
