"""Builds libhhg.so (HIP kernels for gfx950 + host hierarchy builder) in place.

    python paper_1511_02134_amd/build.py
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhhg.so")
BUILD = os.path.join(HERE, "_build")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(BUILD, exist_ok=True)
    host_obj = os.path.join(BUILD, "hierarchy.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c",
          os.path.join(CSRC, "hierarchy.cpp"), "-o", host_obj])
    dev_obj = os.path.join(BUILD, "hhg.o")
    _run([hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, "hhg.hip"), "-o", dev_obj])
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", host_obj, dev_obj, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
