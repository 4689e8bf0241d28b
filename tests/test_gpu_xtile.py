"""GPU parity of the expanded-tile kernels (Life on any pattern, diffusion in
binary32 and bfloat16 storage) and of the binary64 mass reduction."""
import math

import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

A = 0.1  # dt * alpha of the diffusion workload

LIFE = [("carpet", 1), ("carpet", 2), ("carpet", 4), ("carpet", 5), ("carpet", 6), ("vicsek", 1), ("vicsek", 4),
        ("vicsek", 6), ("triangle", 1), ("triangle", 6), ("triangle", 9), ("triangle_paper", 8)]


@pytest.mark.parametrize("name,r", LIFE)
def test_xtile_life_matches_oracle(name, r):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    assert F.xtile_level >= 1
    seed, p = 2201, 0.5
    start = O.fill_compact(seed, p)
    a = F.fill_bernoulli(seed, p)
    b = torch.empty_like(a)
    F.compact_step(a, b, impl="xtile")
    mismatch(to_np(b), O.life_compact(start), f"xtile {name} r={r}")
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(6):
        F.compact_step(x, y, impl="xtile")
        x, y = y, x
    mismatch(to_np(x), O.life_steps(start, 6), f"xtile {name} r={r} 6 steps")


def test_carpet_auto_uses_xtile_and_matches_cell_r8():
    """Level-8 carpet (16.8M cells, 4096-cell tiles): AUTO (expanded tile) equals the
    thread-level kernel over 20 steps and the oracle on one step of two ranges."""
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 8), oracle_fractal("carpet", 8)
    assert not F.has_tile and F.xtile_level == 4
    a = F.fill_bernoulli(7, 0.5)
    b = torch.empty_like(a)
    F.compact_step(a, b)
    start = O.fill_compact(7, 0.5)
    for c0 in (0, F.cells - 1_000_000):
        mismatch(to_np(b[c0:c0 + 1_000_000]), O.life_compact(start, c0, c0 + 1_000_000), f"carpet r8 {c0}")
    x1, y1 = a.clone(), torch.empty_like(a)
    x2, y2 = a.clone(), torch.empty_like(a)
    for _ in range(20):
        F.compact_step(x1, y1)
        F.compact_step(x2, y2, impl="cell")
        x1, y1, x2, y2 = y1, x1, y2, x2
    assert torch.equal(x1, x2)
    rng = np.random.default_rng(8)
    c = rng.integers(0, F.cells, 1500)
    mismatch(to_np(x1[torch.from_numpy(c).cuda()]), O.light_cone(7, 0.5, O.lam(c), 20), "carpet r8 20 steps")


def rel_inf(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


@pytest.mark.parametrize("name,r", [("carpet", 1), ("carpet", 3), ("carpet", 5), ("vicsek", 4), ("triangle", 6)])
@pytest.mark.parametrize("impl", ["xtile", "cell"])
def test_diffusion_f32_matches_f64_oracle(name, r, impl):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    u0 = O.fill_uniform_compact(5)
    a = F.fill_uniform(5)
    mismatch(to_np(a).astype(np.float64), u0, "uniform start")
    b = torch.empty_like(a)
    nb = O.neighbour_table()
    for t in (1, 10, 200):
        x = F.diffuse_run(a.clone(), b, t, A, impl=impl)
        err = rel_inf(to_np(x).astype(np.float64), O.diffuse_steps(u0, A, t, nb))
        assert err < 1e-5, (name, r, impl, t, err)


def test_diffusion_xtile_equals_cell_bitwise():
    torch = torch_or_skip()
    F = gpu_fractal("carpet", 6)
    a = F.fill_uniform(3)
    x = F.diffuse_run(a.clone(), torch.empty_like(a), 25, A, impl="xtile")
    y = F.diffuse_run(a.clone(), torch.empty_like(a), 25, A, impl="cell")
    assert torch.equal(x, y)


def test_diffusion_bf16_offset_storage():
    """bfloat16 storage of u - mean (mean from the binary64 mass), binary32 update,
    stochastic rounding: within 2e-2 (relative infinity norm) of the binary64 oracle
    after 500 steps.  Round-to-nearest-even storage is measured too: small updates
    below half an ulp are lost, so it drifts further (about 3e-2 here) and does not
    meet the bar; the test records that it is the worse of the two."""
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 5), oracle_fractal("carpet", 5)
    u0 = O.fill_uniform_compact(9)
    want = O.diffuse_steps(u0, A, 500)
    u = F.fill_uniform(9)
    mean = float(F.mass_f64(u)) / F.cells
    assert abs(mean * F.cells - math.fsum(u0)) < 1e-9 * F.cells
    errs = {}
    for rounding in ("stochastic", "nearest"):
        d = F.bf16_encode(u, mean)
        res = F.diffuse_run(d, torch.empty_like(d), 500, A, dtype="bf16", rounding=rounding, seed=17)
        errs[rounding] = rel_inf(to_np(F.bf16_decode(res, mean)).astype(np.float64), want)
        if rounding == "stochastic":
            m1 = float(F.mass_f64(res, dtype="bf16", offset=mean))
            assert abs(m1 - math.fsum(u0)) / math.fsum(u0) < 1e-3
    assert errs["stochastic"] < 2e-2, errs
    assert errs["stochastic"] < errs["nearest"] < 0.2, errs


def test_bf16_encode_decode_roundtrip():
    torch = torch_or_skip()
    F = gpu_fractal("carpet", 3)
    u = F.fill_uniform(4)
    b = F.bf16_encode(u, 0.5)
    back = to_np(F.bf16_decode(b, 0.5)).astype(np.float64)
    u64 = to_np(u).astype(np.float64)
    assert np.max(np.abs(back - u64)) <= 2 ** -9 * 0.5 + 1e-12  # |u - 0.5| < 0.5, bf16 keeps 8 bits


def test_mass_f64_matches_exact_sum():
    torch = torch_or_skip()
    F = gpu_fractal("carpet", 7)
    u = F.fill_uniform(12)
    exact = math.fsum(to_np(u).astype(np.float64).tolist())
    got = float(F.mass_f64(u))
    assert abs(got - exact) <= F.cells * 2.0 ** -53 * 1.0 * 4
    again = float(F.mass_f64(u))
    assert got == again  # deterministic reduction tree
    assert float(F.mass_f64(u, offset=0.25)) == pytest.approx(exact + 0.25 * F.cells, rel=1e-15)


def test_diffusion_r9_light_cones_and_mass():
    """Level-9 carpet (134M cells, the diffusion workload's size): 10 binary32 steps
    compared with the binary64 light cone at sampled cells; mass drift after 100 steps."""
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 9), oracle_fractal("carpet", 9)
    u = F.fill_uniform(2201)
    m0 = float(F.mass_f64(u))
    v = torch.empty_like(u)
    res = F.diffuse_run(u, v, 10, A)
    rng = np.random.default_rng(9)
    c = rng.integers(0, F.cells, 3000)
    c[:2] = [0, F.cells - 1]
    got = to_np(res[torch.from_numpy(c).cuda()]).astype(np.float64)
    want = O.diffuse_cone(2201, A, O.lam(c), 10)
    assert np.max(np.abs(got - want)) < 1e-5 * np.max(np.abs(want))
    res = F.diffuse_run(res, u if res is v else v, 90, A, first_step=10)
    m1 = float(F.mass_f64(res))
    assert abs(m1 - m0) / m0 < 1e-5
    del u, v, res
    torch.cuda.empty_cache()


def test_diffusion_argument_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    F = gpu_fractal("carpet", 3)
    a = F.fill_uniform(1)
    with pytest.raises(sqz.SqueezeError) as e:
        F.diffuse_step(a, torch.empty_like(a), 0.2)  # unstable coefficient
    assert e.value.status == 1
    with pytest.raises(sqz.SqueezeError) as e:
        F.diffuse_step(a, a, 0.1)
    assert e.value.status == 1
    with pytest.raises(sqz.SqueezeError) as e:
        F.diffuse_step(a, torch.empty_like(a), 0.1, impl="tile")
    assert e.value.status == 1
