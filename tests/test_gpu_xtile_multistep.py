"""GPU parity of the multi-step expanded tiles (up to three steps per launch with
a border of three cells): Life and diffusion runs equal one-step launches bit for
bit (binary32 and bfloat16 storage with stochastic rounding), and the oracle."""
import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

WIDE = (4, ((0, 0), (1, 0), (3, 0), (0, 1), (2, 1), (3, 1), (1, 2), (2, 2), (0, 3), (3, 3)))


def pair(name, r):
    if name == "wide":
        import oracle
        import paper_2201_00613_amd as sqz

        return sqz.Fractal(*WIDE, r), oracle.Fractal(*WIDE, r)
    return gpu_fractal(name, r), oracle_fractal(name, r)


@pytest.mark.parametrize("name,r", [("carpet", 5), ("carpet", 6), ("carpet", 7), ("wide", 5)])
def test_life_run_equals_single_steps_and_oracle(name, r):
    torch = torch_or_skip()
    F, O = pair(name, r)
    assert not F.has_tile and F.run_steps_per_launch >= 2
    start = O.fill_compact(2201, 0.5)
    nb = O.neighbour_table() if F.cells <= 300_000 else None
    for steps in range(0, 10):
        a = F.fill_bernoulli(2201, 0.5)
        b = torch.zeros_like(a)
        res = F.compact_run(a, b, steps)
        assert res is (a if steps % 2 == 0 else b)
        x, y = F.fill_bernoulli(2201, 0.5), torch.empty_like(a)
        for _ in range(steps):
            F.compact_step(x, y, impl="xtile")
            x, y = y, x
        assert torch.equal(res, x), (name, r, steps)
        if nb is not None and steps in (3, 7):
            mismatch(to_np(res), O.life_steps(start, steps, nb), f"{name} r={r} {steps} steps")


def test_life_all_alive_three_steps():
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 5), oracle_fractal("carpet", 5)
    a = torch.ones(F.cells, dtype=torch.uint8, device="cuda")
    res = F.compact_run(a, torch.empty_like(a), 3)
    mismatch(to_np(res), O.life_steps(np.ones(F.cells, np.uint8), 3), "carpet all alive, 3 steps")


def xt_steps(F):
    """Steps per launch of the fractal's expanded tiles (the Life runs report the
    bit-sliced kernel's for triangle and Vicsek, so ask the library directly)."""
    import paper_2201_00613_amd as sqz

    for k in (3, 2):
        u = F.fill_uniform(0)
        try:
            F.diffuse_run(u, sqz_empty(u), 1, 0.1, steps_per_launch=k)
            return k
        except sqz.SqueezeError:
            continue
    return 1


def sqz_empty(u):
    import torch

    return torch.empty_like(u)


@pytest.mark.parametrize("name,r", [("carpet", 5), ("carpet", 6), ("vicsek", 5), ("triangle", 8), ("wide", 5)])
@pytest.mark.parametrize("dtype,rounding", [("f32", "nearest"), ("bf16", "stochastic"), ("bf16", "nearest")])
def test_diffusion_run_equals_single_steps(name, r, dtype, rounding):
    torch = torch_or_skip()
    F, _ = pair(name, r)
    k = xt_steps(F)
    u = F.fill_uniform(11)
    mean = float(F.mass_f64(u)) / F.cells
    start = u if dtype == "f32" else F.bf16_encode(u, mean)
    for steps, first in ((1, 0), (2, 3), (3, 0), (5, 7), (8, 100)):
        res = F.diffuse_run(start.clone(), torch.empty_like(start), steps, 0.1, dtype=dtype, first_step=first,
                            rounding=rounding, seed=17, steps_per_launch=k)
        x, y = start.clone(), torch.empty_like(start)
        for i in range(steps):
            F.diffuse_step(x, y, 0.1, dtype=dtype, step=first + i, rounding=rounding, seed=17, impl="xtile")
            x, y = y, x
        assert torch.equal(res, x), (name, r, dtype, rounding, steps, first)


def test_diffusion_run_matches_oracle_carpet_r6():
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 6), oracle_fractal("carpet", 6)
    u0 = O.fill_uniform_compact(5)
    u = F.fill_uniform(5)
    got = F.diffuse_run(u, torch.empty_like(u), 50, 0.1, steps_per_launch=3)
    want = O.diffuse_steps(u0, 0.1, 50)
    assert float(np.max(np.abs(to_np(got) - want)) / np.max(np.abs(want))) < 1e-5


def test_r9_runs_equal_single_steps():
    """The diffusion workload's level: 7 binary32 steps and 7 Life steps."""
    torch = torch_or_skip()
    F = gpu_fractal("carpet", 9)
    u = F.fill_uniform(2201)
    r1 = F.diffuse_run(u.clone(), torch.empty_like(u), 7, 0.1, steps_per_launch=3)
    x, y = u.clone(), torch.empty_like(u)
    for i in range(7):
        F.diffuse_step(x, y, 0.1, step=i, impl="xtile")
        x, y = y, x
    assert torch.equal(r1, x)
    del u, r1, x, y
    a = F.fill_bernoulli(3, 0.5)
    l1 = F.compact_run(a.clone(), torch.empty_like(a), 7)
    x, y = a.clone(), torch.empty_like(a)
    for i in range(7):
        F.compact_step(x, y, impl="xtile")
        x, y = y, x
    assert torch.equal(l1, x)
    del a, l1, x, y
    torch.cuda.empty_cache()


def test_diffusion_steps_per_launch_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    F = gpu_fractal("carpet", 6)
    u = F.fill_uniform(1)
    for bad, status in ((4, 5), (-1, 1)):
        with pytest.raises(sqz.SqueezeError) as e:
            F.diffuse_run(u, torch.empty_like(u), 3, 0.1, steps_per_launch=bad)
        assert e.value.status == status
    with pytest.raises(sqz.SqueezeError) as e:
        F.diffuse_run(u, torch.empty_like(u), 3, 0.1, impl="cell", steps_per_launch=2)
    assert e.value.status == 5
