"""The request scheduler's host logic (admission by memory budget, FIFO order,
batch/slot limits, completion and release) on the CPU with a fake executor:
compiles tests/serve_core_test.cpp against the library's scheduler header."""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_core(tmp_path):
    exe = tmp_path / "serve_core_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "paper_2505_12425_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_core_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "OK"
