"""GPU parity of the bit-row expanded tiles (SQZ_IMPL_BITS, the Sierpinski
carpet): one step and multi-step runs bit-exact against the oracle, against
the expanded-tile kernel, and with the result in the documented buffer."""
import ctypes

import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


def test_no_bit_rows_below_level_3():
    """A level-2 tile is narrower than the four-block border: such carpets use the
    expanded tiles."""
    torch_or_skip()
    for r in (0, 1, 2):
        assert gpu_fractal("carpet", r).bits_level == 0


@pytest.mark.parametrize("r", [3, 4, 5, 6])
def test_step_matches_oracle(r):
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", r), oracle_fractal("carpet", r)
    assert F.bits_level == min(r, 5) and F.run_steps_per_launch == 10
    nb = O.neighbour_table()
    for seed, p in ((2201, 0.5), (7, 0.3), (11, 0.8)):
        start = O.fill_compact(seed, p)
        a = F.fill_bernoulli(seed, p)
        b = torch.empty_like(a)
        F.compact_step(a, b, impl="bits")
        mismatch(to_np(b), O.life_steps(start, 1, nb), f"bits r={r} seed={seed}")


@pytest.mark.parametrize("r", [2, 3, 4, 5, 6, 7])
def test_run_equals_single_steps_and_oracle(r):
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", r), oracle_fractal("carpet", r)
    start = O.fill_compact(2201, 0.5)
    nb = O.neighbour_table() if F.cells <= 300_000 else None
    for steps in range(0, 24):
        a = F.fill_bernoulli(2201, 0.5)
        b = torch.zeros_like(a)
        res = F.compact_run(a, b, steps)
        assert res is (a if steps % 2 == 0 else b)
        x, y = F.fill_bernoulli(2201, 0.5), torch.empty_like(a)
        for _ in range(steps):
            F.compact_step(x, y, impl="xtile")
            x, y = y, x
        assert torch.equal(res, x), (r, steps)
        if nb is not None and steps in (2, 5, 6, 7, 10, 13, 21):
            mismatch(to_np(res), O.life_steps(start, steps, nb), f"carpet r={r} {steps} steps")


@pytest.mark.parametrize("steps", [1, 3, 6, 10, 12, 21])
def test_all_alive(steps):
    """Every cell alive at t = 0: border cells change in the first step."""
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 5), oracle_fractal("carpet", 5)
    a = torch.ones(F.cells, dtype=torch.uint8, device="cuda")
    res = F.compact_run(a, torch.empty_like(a), steps)
    mismatch(to_np(res), O.life_steps(np.ones(F.cells, np.uint8), steps), f"all alive, {steps} steps")


def test_r9_run_equals_expanded_tiles():
    """The benchmark level (134,217,728 cells, 4,096 tiles): a 23-step run (launches
    of 10, 10 and 3) equals 23 one-step expanded-tile launches."""
    torch = torch_or_skip()
    F = gpu_fractal("carpet", 9)
    a = F.fill_bernoulli(2201, 0.5)
    r1 = F.compact_run(a.clone(), torch.empty_like(a), 23)
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(23):
        F.compact_step(x, y, impl="xtile")
        x, y = y, x
    assert torch.equal(r1, x)
    del a, r1, x, y
    torch.cuda.empty_cache()


def test_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    T = gpu_fractal("triangle", 6)
    assert T.bits_level == 0
    a = T.fill_bernoulli(1, 0.5)
    with pytest.raises(sqz.SqueezeError) as e:
        T.compact_step(a, torch.empty_like(a), impl="bits")
    assert e.value.status == 5
    C1 = gpu_fractal("carpet", 1)
    assert C1.bits_level == 0
    F = gpu_fractal("carpet", 4)
    L = sqz._lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = torch.zeros(2 * F.cells + 64, dtype=torch.uint8, device="cuda")
    src, dst = big[4:4 + F.cells], big[F.cells + 32:2 * F.cells + 32]
    assert L.sqz_compact_step_impl(F._h, 5, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), s) == 1
    # AUTO falls back to the expanded tiles for 4-byte aligned buffers
    src.copy_(F.fill_bernoulli(3, 0.5))
    assert L.sqz_compact_step_impl(F._h, 0, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), s) == 0
    want = torch.empty_like(src)
    F.compact_step(src.clone(), want, impl="xtile")
    assert torch.equal(dst, want)
