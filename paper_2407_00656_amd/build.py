"""Builds libhgks.so (HIP kernels for gfx950 + host precompute + C ABI) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhgks.so")
BUILD = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

# Packed FP32 instructions stay off: all float arithmetic is issued as scalar-lane ops.
HIP_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__",
             f"-I{ROCM}/include"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    return r


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    objs = []
    ku = os.path.join(BUILD, "kernels.o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    r = _run([hipcc, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, "kernels.hip"), "-o", ku], verbose)
    if resource_usage:
        sys.stdout.write(r.stderr)
    objs.append(ku)
    for src in ("mesh_build.cpp", "mesh_hex.cpp", "capi.cpp"):
        o = os.path.join(BUILD, src.replace(".cpp", ".o"))
        _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv)
