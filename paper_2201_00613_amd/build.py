"""Compile libsqueeze.so (HIP, gfx950) in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsqueeze.so")
SOURCES = ["api.hip", "maps.hip", "mfma_maps.hip", "blocks.hip", "bb.hip", "life_tile.hip", "xtile.hip", "bitbox.hip", "batch.hip"]
ARCH = os.environ.get("SQZ_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libsqueeze)")


def compile_command(out: str, defines=()) -> list[str]:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        *[f"-D{d}" for d in defines],
        "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
        # keep the compiler from forming packed-FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out,
    ]


CALIB_SRC = os.path.join(PKG, "calib", "valu_issue.hip")
CALIB_BIN = os.path.join(PKG, "calib", "valu_issue")


def calib_command(out: str) -> list[str]:
    """The vector-ALU issue-rate calibration program (a measurement aid, not part of the library)."""
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", CALIB_SRC, "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = compile_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    cmd = calib_command(CALIB_BIN + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB_BIN + ".tmp", CALIB_BIN)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
