"""Build libabea.so (HIP, gfx950) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libabea.so")
SOURCES = [
    os.path.join(CSRC, "abea_kernels.hip"),
    os.path.join(CSRC, "abea_host.cpp"),
    os.path.join(CSRC, "abea_server.cpp"),
    os.path.join(CSRC, "abea_detect.hip"),
    os.path.join(CSRC, "abea_detect_host.cpp"),
    os.path.join(CSRC, "abea_meth.hip"),
    os.path.join(CSRC, "abea_meth_host.cpp"),
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the cell arithmetic must round every operation as the CPU reference does
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # 16-byte LDS reads as one ds_read_b128 (contiguous across the lanes,
    # free of bank conflicts) rather than a pair of 8-byte reads
    "-Xclang", "-target-feature", "-Xclang", "+enable-ds128",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-pthread",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
