"""Shared helpers for the GPU parity tests (device side through the C ABI,
expected values from the CPU oracle only)."""
import numpy as np
import pytest

import fractals as FR


def torch_or_skip():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a HIP device")
    return torch


def gpu_fractal(name, r):
    import paper_2201_00613_amd as sqz

    s, offs = FR.ALL[name]
    return sqz.Fractal(s, offs, r)


def oracle_fractal(name, r):
    import oracle

    s, offs = FR.ALL[name]
    return oracle.Fractal(s, offs, r)


def to_np(t):
    return t.detach().cpu().numpy()


def mismatch(got, want, what=""):
    got, want = np.asarray(got), np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    bad = np.flatnonzero(got.reshape(-1) != want.reshape(-1))
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:8].tolist()}"
