"""GPU parity of the lambda / nu maps and the seeded starts against the oracle."""
import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

EXHAUSTIVE = [("triangle", 0), ("triangle", 1), ("triangle", 2), ("triangle", 10), ("triangle_paper", 8),
              ("carpet", 1), ("carpet", 5), ("vicsek", 1), ("vicsek", 6)]


@pytest.mark.parametrize("name,r", EXHAUSTIVE)
def test_lambda_exhaustive(name, r):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    idx = torch.arange(F.cells + 3, dtype=torch.int64, device="cuda")
    idx[-1] = -1  # UINT64_MAX
    xy = to_np(F.lambda_map(idx))
    mismatch(xy[:F.cells], O.order(), f"lambda {name} r={r}")
    assert (xy[F.cells:] == -1).all()


@pytest.mark.parametrize("name,r", EXHAUSTIVE)
def test_nu_exhaustive_with_ring(name, r):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    n = F.n
    ys, xs = np.mgrid[-1:n + 1, -1:n + 1]
    pts = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
    got = to_np(F.nu_map(torch.from_numpy(pts).cuda()))
    dense = np.full((n + 2, n + 2), -1, dtype=np.int64)
    dense[1:-1, 1:-1] = O.dense_inverse()
    mismatch(got, dense.ravel(), f"nu {name} r={r}")
    # nu(lambda(c)) = c on the device alone
    idx = torch.arange(F.cells, dtype=torch.int64, device="cuda")
    mismatch(to_np(F.nu_map(F.lambda_map(idx))), np.arange(F.cells), "nu o lambda")


@pytest.mark.parametrize("name,r", [("triangle", 16), ("triangle", 20), ("triangle", 22), ("carpet", 9),
                                    ("carpet", 12), ("vicsek", 14)])
def test_maps_sampled_large(name, r):
    """Random indices and points at levels where N may exceed 2^32 (64-bit paths)."""
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    rng = np.random.default_rng(r)
    c = rng.integers(0, F.cells, 200_000, dtype=np.uint64)
    c[:4] = [0, 1, F.cells - 2, F.cells - 1]
    xy = to_np(F.lambda_map(torch.from_numpy(c.view(np.int64)).cuda()))
    mismatch(xy, O.lam(c), f"lambda {name} r={r}")
    mismatch(to_np(F.nu_map(torch.from_numpy(xy).cuda())), c.view(np.int64), "nu o lambda")
    pts = rng.integers(-1, F.n + 1, (200_000, 2)).astype(np.int32)
    pts[:6] = [[0, 0], [F.n - 1, 0], [0, F.n - 1], [F.n - 1, F.n - 1], [-2 ** 31, 5], [2 ** 31 - 1, 0]]
    got = to_np(F.nu_map(torch.from_numpy(pts).cuda()))
    mismatch(got, O.nu(pts.astype(np.int64)), f"nu {name} r={r}")


@pytest.mark.parametrize("name,r,seed,p", [("triangle", 10, 2201, 0.5), ("triangle", 12, 1, 0.3),
                                           ("carpet", 4, 77, 0.5), ("vicsek", 5, 123456789, 0.5),
                                           ("triangle", 3, 2201, 0.0), ("triangle", 3, 2201, 1.0)])
def test_fill_bernoulli(name, r, seed, p):
    torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    mismatch(to_np(F.fill_bernoulli(seed, p)), O.fill_compact(seed, p), "compact fill")
    if F.n <= 4096:
        mismatch(to_np(F.fill_bernoulli(seed, p, layout="expanded")).reshape(F.n, F.n),
                 O.fill_expanded(seed, p), "expanded fill")


def test_fill_bernoulli_r20_sampled():
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 20), oracle_fractal("triangle", 20)
    st = F.fill_bernoulli(2201, 0.3)
    rng = np.random.default_rng(0)
    c = rng.integers(0, F.cells, 100_000)
    c[:2] = [0, F.cells - 1]
    got = to_np(st[torch.from_numpy(c).cuda()])
    want = np.array([O.fill_compact(2201, 0.3, int(ci), int(ci) + 1)[0] for ci in c[:2000]])
    mismatch(got[:2000], want, "fill r=20")
    assert abs(got.mean() - 0.3) < 0.01
    del st
    torch.cuda.empty_cache()


def test_fill_uniform():
    torch_or_skip()
    F, O = gpu_fractal("carpet", 5), oracle_fractal("carpet", 5)
    got = to_np(F.fill_uniform(9)).astype(np.float64)
    mismatch(got, O.fill_uniform_compact(9), "uniform fill")
