"""CPU tests of the serving runtime's host logic (arena allocator, admission order).

The allocator and the admission rule are host-only C++ (paper_2409_03568_amd/csrc/
arena.hpp); tests/native/runtime_host_test.cpp checks them against a unit bitmap and a
simulated job stream.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "runtime_host_test.cpp")


def test_arena_and_admission(tmp_path):
    exe = str(tmp_path / "runtime_host_test")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-fsanitize=address,undefined", "-o", exe, SRC],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "OK"
