"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: its C++
source, compiled into tests/oracle_sanitize_driver.cpp with both sanitizers
(every report fatal), runs small 1D, 2D and 3D solves with all side kinds,
active limiters, the first-order scheme and Dirichlet rows."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

from helpers import ROOT


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "oracle_sanitize"
    build = subprocess.run(
        [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
         os.path.join(ROOT, "tests", "oracle_sanitize_driver.cpp"), "-o", str(exe)],
        capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower() and "cannot find" in build.stderr:
        pytest.skip("no sanitizer runtime for g++")
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "fails=0" in run.stdout
    assert "FAILED" not in run.stdout
