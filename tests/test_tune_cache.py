"""The autotuner's persistent cache (csrc/tune_cache.cpp), compiled on the host
with g++ and run: a stored choice reads back; a missing, corrupt or stale file
and out-of-range values read as "no entry", so a plan tunes afresh (or keeps
its defaults) instead of taking a bad layout."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tune_cache_round_trip_and_fallbacks(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "tune_cache_test"
    csrc = os.path.join(ROOT, "paper_1604_03155_amd", "csrc")
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", csrc,
                        os.path.join(ROOT, "tests", "cpp", "tune_cache_test.cpp"),
                        os.path.join(csrc, "tune_cache.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
