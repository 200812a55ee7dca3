"""Build libpermgpu.so in-tree with hipcc for gfx950.

    python -m paper_1802_02779_amd.build

The library is one device translation unit (``csrc/perm_device.hip``) plus
host-only C++ (``csrc/perm_host.cpp``, ``csrc/perm_server.cpp``), linked
against the HIP runtime.  Packed-FP32 instructions are disabled for the
device code; FP contraction is off (every fused multiply-add in the kernels
is written explicitly).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libpermgpu.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["perm_device.hip", "perm_host.cpp", "perm_server.cpp", "perm_multi.cpp", "perm_order.cpp"]
ARCH = os.environ.get("PERM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", INCLUDE, "-I", CSRC,
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError(f"hipcc failed with exit code {proc.returncode}")
    if verbose and proc.stdout.strip():
        # hipcc's host pass warns that it does not know the packed-fp32 feature
        lines = [ln for ln in proc.stdout.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            print("\n".join(lines))
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
