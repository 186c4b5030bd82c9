"""The batched apply's cache policy (csrc/batch_cache.h), compiled on the host
with g++ and run: batches recorded into a caller's stream capture are pinned
and never evicted (the caller's graph points into their device descriptors
and workspace); they go only with a plan they use."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pinned_entries_are_never_evicted(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "batch_cache_test"
    src = os.path.join(ROOT, "tests", "cpp", "batch_cache_test.cpp")
    inc = os.path.join(ROOT, "paper_1604_03155_amd", "csrc")
    r = subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
