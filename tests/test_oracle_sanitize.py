"""Host code under the sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer): the C oracle
(gcc, no OpenMP) on a small random model of every descriptor kind -- periodic cell smaller than
2 r_c, both neighbour searches (which must agree), the table, an open cluster and a ghost domain
(tests/oracle_sanitize.c) -- and the model file's header parser on truncated and mutated headers
(tests/json_fuzz.cpp, g++). Any out-of-bounds access, leak or undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                            os.path.join(HERE, "oracle_sanitize.c"), "-o", exe, "-lm"],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitizer run ok" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_model_header_parser_under_sanitizers(tmp_path):
    exe = str(tmp_path / "json_fuzz")
    csrc = os.path.join(HERE, "..", "paper_2304_09409_amd", "csrc")
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I" + csrc,
                            os.path.join(HERE, "json_fuzz.cpp"), "-o", exe],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "json header fuzz ok" in r.stdout
