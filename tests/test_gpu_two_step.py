"""GPU parity of the multi-step tiled kernels used by sqz_compact_run, in both
run forms: "launches" (up to ten Life steps per launch) and "resident" (one
launch, tiles held in LDS, ring cells exchanged every ten steps).
Every step count, every tiled pattern, bit-exact against one-step launches and
the oracle, with the result in the documented buffer."""
import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

CASES = [("triangle", 3), ("triangle", 5), ("triangle", 8), ("triangle", 9), ("triangle", 11),
         ("triangle_paper", 4), ("triangle_paper", 9), ("vicsek", 2), ("vicsek", 3), ("vicsek", 6),
         ("vicsek", 8)]


FORMS = ["launches", "resident"]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("name,r", CASES)
def test_run_equals_single_steps_and_oracle(name, r, form):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    assert F.has_tile
    assert F.resident_run  # at most 3^3 level-8 tiles here: all fit on the chip
    # ring slots exist even for a single tile (all absent); ring cells must lie in the
    # adjacent tiles, so a launch takes fewer than s^M steps
    assert F.run_steps_per_launch == min(10, F.s ** F.tile_level - 1)
    start = O.fill_compact(2201, 0.5)
    nb = O.neighbour_table() if F.cells <= 3 ** 11 else None
    for steps in range(0, 23):
        a = F.fill_bernoulli(2201, 0.5)
        b = torch.zeros_like(a)
        res = F.compact_run(a, b, steps, form=form)
        assert res is (a if steps % 2 == 0 else b)
        x, y = F.fill_bernoulli(2201, 0.5), torch.empty_like(a)
        for _ in range(steps):
            F.compact_step(x, y, impl="tile")
            x, y = y, x
        assert torch.equal(res, x), (name, r, form, steps)
        if nb is not None and steps in (2, 3, 4, 7, 10, 12, 15, 21):
            mismatch(to_np(res), O.life_steps(start, steps, nb), f"{name} r={r} {steps} steps")


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("steps", [2, 3, 4, 5, 6, 7, 8, 9, 10, 14, 20])
def test_all_alive_multi_step(steps, form):
    """All cells alive at t = 0: ring cells change state in the first step, so later
    steps depend on their recomputed states."""
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 10), oracle_fractal("triangle", 10)
    a = torch.ones(F.cells, dtype=torch.uint8, device="cuda")
    res = F.compact_run(a, torch.empty_like(a), steps, form=form)
    mismatch(to_np(res), O.life_steps(np.ones(F.cells, np.uint8), steps), f"all alive, {steps} steps ({form})")


@pytest.mark.parametrize("form", FORMS)
def test_r16_run_equals_single_steps(form):
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 16)
    a = F.fill_bernoulli(9, 0.5)
    r1 = F.compact_run(a.clone(), torch.empty_like(a), 20, form=form)
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(20):
        F.compact_step(x, y, impl="tile")
        x, y = y, x
    assert torch.equal(r1, x)


@pytest.mark.parametrize("r", [15, 16, 17])
def test_large_triangle_tiles_equal_thread_level(r):
    """From level 16 the triangle runs level-10 tiles in 512-lane workgroups (below
    it level-8 tiles): a 13-step run (launches of 10 and 3) equals 13 thread-level
    steps.  The thread-level kernel computes every cell with one lambda and eight
    nu; the tiles evaluate no map per cell (the same device maps only locate each
    tile's ring cells at set-up), so the two paths differ in everything but those
    maps.  The oracle itself checks the level-10 tiles in test_gpu_headline_parity."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", r)
    assert F.tile_level == (10 if r >= 16 else 8) and F.run_steps_per_launch == 10
    assert F.resident_run == (r == 16)  # 729 level-10 tiles fit the chip; 2,187 tiles do not
    a = F.fill_bernoulli(31, 0.4)
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(13):
        F.compact_step(x, y, impl="cell")
        x, y = y, x
    for form in ["launches"] + (["resident"] if F.resident_run else []):
        r1 = F.compact_run(a.clone(), torch.empty_like(a), 13, form=form)
        assert torch.equal(r1, x), form
        del r1
    del a, x, y
    torch.cuda.empty_cache()
