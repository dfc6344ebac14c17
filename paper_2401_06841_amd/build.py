"""Build libdg.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2401_06841_amd.build [--resource-usage]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libdg.so")
SOURCES = ["dg_api.hip", "dg_sensor.hip", "dg_stats.hip", "dg_forcing.cpp"]
# hipFFT for the spectrum of the flow statistics
LIBS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lhipfft"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed FP32 (v_pk_*_f32) off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if resource_usage:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    tmp = SO + ".tmp"
    cmd += ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + LIBS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True, resource_usage="--resource-usage" in sys.argv)
