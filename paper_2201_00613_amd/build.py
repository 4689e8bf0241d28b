"""Compile libsqueeze.so (HIP, gfx950) in-tree.

Each HIP source is compiled to its own object in parallel (no cross-file
device code, so no relocatable device code is needed), then the objects are
linked into the shared library.  The vector-ALU calibration program is a
measurement aid with a build function of its own (``build_calib``); the
library build does not depend on it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsqueeze.so")
OBJDIR = os.path.join(ROOT, "_build", "obj")
SOURCES = ["api.hip", "maps.hip", "mfma_maps.hip", "blocks.hip", "bb.hip", "life_tile.hip", "xtile.hip", "bitbox.hip",
           "batch.hip"]
HOST_SOURCES = ["host_tables.cpp"]
ARCH = os.environ.get("SQZ_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libsqueeze)")


def _common_flags(defines=()) -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", *[f"-D{d}" for d in defines],
            "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
            # keep the compiler from forming packed-FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC]


def object_commands(objdir: str, defines=()) -> list[tuple[list[str], str]]:
    """(command, object path) for every source: HIP sources through hipcc, the
    host-only table builders through g++ (no device code)."""
    cmds = []
    for s in SOURCES:
        obj = os.path.join(objdir, s + ".o")
        cmds.append(([hipcc(), *_common_flags(defines), "-c", os.path.join(CSRC, s), "-o", obj], obj))
    for s in HOST_SOURCES:
        obj = os.path.join(objdir, s + ".o")
        cmds.append((["g++", "-O2", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wextra",
                      "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, s), "-o", obj], obj))
    return cmds


def compile_command(out: str, defines=()) -> list[str]:
    """One hipcc command that builds the whole library (serial; used for variants)."""
    return [hipcc(), *_common_flags(defines), "-shared",
            *[os.path.join(CSRC, s) for s in SOURCES + HOST_SOURCES], "-o", out]


def build(verbose: bool = False, jobs: int | None = None, defines=(), out: str = LIB) -> str:
    objdir = OBJDIR if not defines else OBJDIR + "_" + "_".join(d.replace("=", "") for d in defines)
    os.makedirs(objdir, exist_ok=True)
    cmds = object_commands(objdir, defines)
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))

    def run(c):
        if verbose:
            print(" ".join(c[0]), flush=True)
        subprocess.run(c[0], check=True)
        return c[1]

    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(run, cmds))
    tmp = out + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


CALIB_SRC = os.path.join(PKG, "calib", "valu_issue.hip")
CALIB_BIN = os.path.join(PKG, "calib", "valu_issue")


def calib_command(out: str) -> list[str]:
    """The vector-ALU issue-rate calibration program (a measurement aid, not part of the library)."""
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", CALIB_SRC, "-o", out]


def build_calib(verbose: bool = False) -> str:
    """Build the calibration program (profiling path only; `python -m paper_2201_00613_amd.build calib`)."""
    cmd = calib_command(CALIB_BIN + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB_BIN + ".tmp", CALIB_BIN)
    return CALIB_BIN


if __name__ == "__main__":
    import sys

    if len(sys.argv) > 1 and sys.argv[1] == "calib":
        print(build_calib(verbose=True))
    else:
        print(build(verbose=True))
