"""Host tests of the serving policy (FIFO queue, first-fit arena, admission by
memory footprint and slots, batching by kernel class), compiled from the
library's own sk_sched.cpp with g++ and the address / undefined-behaviour
sanitizers, and run against a fake executor (tests/sched/sched_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_20966_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_policy(tmp_path):
    exe = str(tmp_path / "sched_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "sched", "sched_check.cpp"), os.path.join(CSRC, "sk_sched.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "scheduler checks passed" in r.stdout
