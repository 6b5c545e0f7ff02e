"""Build libsympix.so in-tree: host geometry with g++ (no FP contraction, so
the latitude arithmetic is evaluated exactly as written), HIP kernels and the
C ABI with hipcc for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsympix.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return res


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    geo_o = os.path.join(BUILD, "geometry.o")
    ker_o = os.path.join(BUILD, "kernels.o")
    sht_o = os.path.join(BUILD, "sht.o")
    pre_o = os.path.join(BUILD, "precond.o")
    api_o = os.path.join(BUILD, "api.o")
    _run(["g++", "-std=c++17", "-O2", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra",
          "-c", os.path.join(CSRC, "geometry.cpp"), "-o", geo_o], verbose)
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", ker_o], verbose)
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "sht.hip"), "-o", sht_o], verbose)
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "precond.hip"), "-o", pre_o], verbose)
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "api.cpp"), "-o", api_o], verbose)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, geo_o, ker_o, sht_o, pre_o, api_o], verbose)
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
