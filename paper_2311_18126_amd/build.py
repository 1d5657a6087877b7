"""Build libdmrod.so (the HIP kernels and the C++ host runtime) and the dm_peaks measurement
program for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdmrod.so")
PEAKS = os.path.join(HERE, "dm_peaks")
FLOPS = os.path.join(HERE, "dm_flops")
SOURCES = ["dm_kernels.hip", "dm_mlp.hip", "dm_contact.hip", "dm_runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# gfx950 with XNACK off (the code object for GPUs without page-fault retry, the MI355X's
# default): the compiler need not keep memory clauses' address registers live for a replay,
# 0.9 % faster on the rod batch than a code object that also runs with XNACK on
FLAGS = ["--offload-arch=gfx950:xnack-", "-O3", "-std=c++17", "-fPIC", "-shared",
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # instruction scheduling for latency hiding over occupancy: the step kernel runs two
         # waves per SIMD at 256 VGPRs, and this order measured 2.3 % faster on the rod batch
         "-mllvm", "-amdgpu-sched-strategy=max-ilp",
         "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False) -> str:
    """Compile every source into libdmrod.so next to this file and return its path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libdmrod.so")
    os.replace(tmp, LIB)
    build_peaks(verbose)
    build_flops(verbose)
    return LIB


def build_flops(verbose: bool = False) -> str:
    """Compile the operation counter of the element math (a host program, no GPU code)."""
    tmp = FLOPS + ".tmp"
    cmd = [HIPCC, "--cuda-host-only", "-O2", "-std=c++17", os.path.join(CSRC, "dm_flops.cpp"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building dm_flops")
    os.replace(tmp, FLOPS)
    return FLOPS


def build_peaks(verbose: bool = False) -> str:
    """Compile the standalone ceiling-measurement program (FP64 FMA, HBM copy, BF16 MFMA)."""
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    tmp = PEAKS + ".tmp"
    cmd = [HIPCC, *flags, os.path.join(CSRC, "dm_peaks.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building dm_peaks")
    os.replace(tmp, PEAKS)
    return PEAKS


def build_hostcheck(out: str, verbose: bool = False) -> str:
    """Compile the host check of the element math (csrc/dm_hostcheck.cpp) with AddressSanitizer
    and UndefinedBehaviorSanitizer on the host code (the program has no GPU code)."""
    cmd = [HIPCC, "--cuda-host-only", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", os.path.join(CSRC, "dm_hostcheck.cpp"), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building dm_hostcheck")
    return out


if __name__ == "__main__":
    print(build(verbose=True))
