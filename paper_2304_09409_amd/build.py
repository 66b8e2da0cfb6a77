"""Build libdpk.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2304_09409_amd.build   (or __graft_entry__.build()).
Every call recompiles; objects go to paper_2304_09409_amd/_build/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdpk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-I" + CSRC]
# Geometry kernels: no FMA contraction, so distances are bitwise reproducible sums of products.
SOURCES = {
    "kernels_geom.hip": ["-ffp-contract=off"],
    "kernels_nn.hip": [],
    "kernels_fit.hip": [],
    # the table kernels keep their MFMA accumulators in VGPRs (no AGPR copies around the loops)
    "kernels_tab.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "api.cpp": ["-ffp-contract=off"],
    "model_file.cpp": [],
    "kernels_train.hip": [],
    "trainer.cpp": [],
}


def _compile(src: str, extra: list[str]) -> str:
    obj = os.path.join(OUT, src + ".o")
    cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(*kv), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-Wl,--no-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    # the vector-ALU calibration program (a standalone executable; not part of the library)
    probe = os.path.join(HERE, "calib", "valu_rates.hip")
    cmd = [HIPCC] + COMMON + [probe, "-o", os.path.join(OUT, "valu_rates")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for calib/valu_rates.hip:\n{r.stderr}")
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
