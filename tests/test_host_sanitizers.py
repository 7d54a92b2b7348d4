"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer on the CPU:
the C ABI's argument validation (csrc/api.cpp, compiled with the host
compiler against stub kernel launchers) and every function of the oracle
(oracle/kro.c) on small and degenerate inputs.  Each driver prints "OK"."""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_12425_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _run(exe):
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "OK"


def test_api_validation_sanitized(tmp_path):
    exe = tmp_path / "api_sanitize_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC] + SAN +
                   [os.path.join(ROOT, "tests", "api_sanitize_test.cpp"), os.path.join(CSRC, "api.cpp"),
                    "-o", str(exe)], check=True)
    _run(exe)


def test_oracle_sanitized(tmp_path):
    exe = tmp_path / "oracle_sanitize_test"
    subprocess.run(["gcc", "-std=c11", "-O1", "-ffp-contract=off", "-Wno-unknown-pragmas"] + SAN +
                   [os.path.join(ROOT, "tests", "oracle_sanitize_test.c"), os.path.join(ROOT, "oracle", "kro.c"),
                    "-lm", "-o", str(exe)], check=True)
    _run(exe)
