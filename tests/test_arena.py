"""The server's HBM arena (first-fit carving of one allocation, paper_2304_09409_amd/csrc/arena.h):
host logic only, checked by a small C++ program built with g++ (and the host sanitizers) against a
brute-force granule map
(a carve succeeds exactly when a run of free granules holds it; no overlap; holes exact, merged)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2304_09409_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_arena_carving(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I" + CSRC, os.path.join(HERE, "arena_check.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "arena ok" in r.stdout
