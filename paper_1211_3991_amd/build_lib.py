"""Builds libxylevy.so (HIP kernels for gfx950 + host graph code) in-tree.

Device code is compiled for gfx950 only, with packed-FP32 instruction
generation disabled.  The FP64 kernels are compiled with -ffp-contract=off so
that their arithmetic is evaluated exactly as written (no fused multiply-add);
the host graph code likewise, so its prefix sums are plain sequential adds.
"""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxylevy.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIP_COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-command-line-argument"]
HIP_SOURCES = {
    "kernels_fp64.hip": ["-ffp-contract=off"],
    "kernels_fix16.hip": [],
    "kernels_phase.hip": [],
    "kernels_walk.hip": [],
    "runtime.hip": ["-ffp-contract=off"],
}
CXX_SOURCES = {"graph.cpp": ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra"]}


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, extra in HIP_SOURCES.items():
        obj = os.path.join(BUILD, src + ".o")
        cmd = [_hipcc(), "-c", *HIP_COMMON, *extra, "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    for src, flags in CXX_SOURCES.items():
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["g++", "-c", *flags, "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
