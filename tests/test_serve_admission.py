"""Admission bookkeeping of the served form on the CPU: the first-fit arena
and the admit / not-now / never decision, driven by a footprint-only fake
device and a fake clock (tests/cpp/arena_check.cpp, built with g++)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_and_admission(tmp_path):
    exe = str(tmp_path / "arena_check")
    src = os.path.join(HERE, "cpp", "arena_check.cpp")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-fsanitize=address,undefined",
                    "-o", exe, src], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
