"""CPU test of the serving admission logic: the arena and FIFO admitter of the
serving loop are compiled with g++ against a test driver (no GPU involved)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_admission_logic(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = tmp_path / "sched_test"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", os.path.join(HERE, "native", "sched_test.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "OK" in out.stdout
