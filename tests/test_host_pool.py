"""The host worker pool that builds and checks patch-set tables
(csrc/host_pool.hpp), on the CPU: built with g++ and run as its own program
(host_pool_check.cpp): every task of a call runs exactly once, two threads
can call at once, and a forked child completes its calls and exits."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2606_12162_amd", "csrc")


def test_host_pool_runs_every_task_once_across_threads_and_fork(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "host_pool_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", "-I", CSRC, "-o", exe,
                    os.path.join(HERE, "host_pool_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "forked child ok 1" in r.stdout
