"""The compile-time block plans of the bit-sliced tiled Life kernels (the
brute-force micro-fractal of Section "Moving from Thread-level to
Block-level", turned into bit moves): a host program built from the kernels'
own header checks, on the CPU, that the plan of every tiled pattern gives each
cell of a block exactly its number of live Moore neighbours, for random block
and adjacent-block words (tests/host/check_block_plan.hip)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_block_plans_count_moore_neighbours():
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if not hipcc:
        pytest.skip("hipcc not available")
    out = os.path.join(ROOT, "_build", "host")
    os.makedirs(out, exist_ok=True)
    exe = os.path.join(out, "check_block_plan")
    csrc = os.path.join(ROOT, "paper_2201_00613_amd", "csrc")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I",
                    csrc, os.path.join(ROOT, "tests", "host", "check_block_plan.hip"),
                    os.path.join(csrc, "host_tables.cpp"), "-o", exe], check=True, capture_output=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "all checks passed" in res.stdout, res.stdout
