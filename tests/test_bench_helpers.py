"""Host-side checks of bench.py's reporting helpers (no GPU): the end-to-end ceilings and the
one-GPU guard."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_e2e_reports_both_ceilings_for_mixed_water():
    b = _bench()
    r = b.e2e("water", "mixed", 2.0e7)
    assert r["ceiling"] == b.CEILING[("water", "mixed")]
    assert r["frac"] == pytest.approx(2.0e7 / r["ceiling"])
    assert r["calibrated"]["ceiling"] > r["ceiling"]          # the measured tanh is cheaper
    assert r["calibrated"]["frac"] == pytest.approx(2.0e7 / r["calibrated"]["ceiling"])


def test_e2e_without_calibrated_ceiling_and_unknown_workload():
    b = _bench()
    r = b.e2e("water", "fp64", 5.0e6)
    assert "calibrated" not in r and r["frac"] == pytest.approx(5.0e6 / 1.73e7)
    assert b.e2e("no such workload", "mixed", 1.0) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""
