"""The serving scheduler's host logic (rs_sched.h: admission with bounded
overtaking, slice shares, arena, retirement, launch and device failures),
driven with synthetic completions by tests/csrc/sched_host_test.cpp, built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer.  No GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "csrc", "sched_host_test.cpp")
INC = os.path.join(ROOT, "paper_2307_09226_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduler_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sched_host_test")
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            "-Wall", "-Wextra", "-Werror", "-I", INC, SRC, "-o", exe],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "ALL OK" in run.stdout
