"""The CPU oracle and the serving policy's simulator built with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc / g++, host code only)
and run on seeded inputs: any out-of-bounds access, leak or undefined
operation fails the test.  CPU only."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _have(tool):
    return shutil.which(tool) is not None


def _build_and_run(tmp_path, compiler, sources, flags, name):
    exe = str(tmp_path / name)
    cmd = [compiler] + SAN + flags + sources + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip(f"sanitizer runtime unavailable: {r.stderr[-300:]}")
    assert r.returncode == 0, r.stderr
    run = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.skipif(not _have("gcc"), reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc",
                         [os.path.join(HERE, "sanitize", "oracle_driver.c"),
                          os.path.join(ROOT, "oracle", "sw_oracle.c")],
                         ["-std=c99", "-D_POSIX_C_SOURCE=200809L", "-lpthread"], "oracle_san")
    assert "0 failures" in out


@pytest.mark.skipif(not _have("g++") or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the ROCm headers not found")
def test_serving_simulator_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1208_6350_amd", "csrc")
    out = _build_and_run(tmp_path, "g++",
                         [os.path.join(HERE, "sanitize", "sim_driver.cpp"),
                          os.path.join(csrc, "simulate.cpp")],
                         ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + csrc],
                         "sim_san")
    assert "0 failures" in out
