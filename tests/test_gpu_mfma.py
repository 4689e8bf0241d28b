"""GPU parity of the matrix-core map variants (lambda and nu as int8 MFMA digit
sums) and of the thread-level Life step that uses them: bit-exact against the
oracle and against the scalar look-up-table maps."""
import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

# A 4x4 pattern with 10 replicas (k > 8: tau from LDS; s = 4: division path)
# and a 12x12 pattern with 127 replicas (the largest digit int8 holds).
WIDE = (4, ((0, 0), (1, 0), (3, 0), (0, 1), (2, 1), (3, 1), (1, 2), (2, 2), (0, 3), (3, 3)))
K127 = (12, tuple((i % 12, i // 12) for i in range(144) if i % 9 != 4)[:127])
EXTRA = {"wide": WIDE, "k127": K127}


def fractal_pair(name, r):
    if name in EXTRA:
        import oracle
        import paper_2201_00613_amd as sqz

        s, offs = EXTRA[name]
        return sqz.Fractal(s, offs, r), oracle.Fractal(s, offs, r)
    return gpu_fractal(name, r), oracle_fractal(name, r)


EXHAUSTIVE = [("triangle", 0), ("triangle", 1), ("triangle", 2), ("triangle", 10), ("triangle_paper", 8),
              ("carpet", 1), ("carpet", 5), ("vicsek", 1), ("vicsek", 6), ("wide", 1), ("wide", 5),
              ("k127", 1), ("k127", 2)]


def test_k127_pattern_is_valid():
    s, offs = K127
    assert len(offs) == 127 and len(set(offs)) == 127


@pytest.mark.parametrize("name,r", EXHAUSTIVE)
def test_lambda_mfma_exhaustive(name, r):
    torch = torch_or_skip()
    F, O = fractal_pair(name, r)
    idx = torch.arange(F.cells + 70, dtype=torch.int64, device="cuda")
    idx[-1] = -1  # UINT64_MAX
    got = F.lambda_map(idx, impl="mfma")
    xy = to_np(got)
    mismatch(xy[:F.cells], O.order(), f"lambda mfma {name} r={r}")
    assert (xy[F.cells:] == -1).all()
    assert torch.equal(got, F.lambda_map(idx, impl="scalar"))


@pytest.mark.parametrize("name,r", EXHAUSTIVE)
def test_nu_mfma_exhaustive_with_ring(name, r):
    torch = torch_or_skip()
    F, O = fractal_pair(name, r)
    n = F.n
    ys, xs = np.mgrid[-1:n + 1, -1:n + 1]
    pts = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
    got = to_np(F.nu_map(torch.from_numpy(pts).cuda(), impl="mfma"))
    dense = np.full((n + 2, n + 2), -1, dtype=np.int64)
    dense[1:-1, 1:-1] = O.dense_inverse()
    mismatch(got, dense.ravel(), f"nu mfma {name} r={r}")
    idx = torch.arange(F.cells, dtype=torch.int64, device="cuda")
    mismatch(to_np(F.nu_map(F.lambda_map(idx, impl="mfma"), impl="mfma")), np.arange(F.cells), "nu o lambda")


@pytest.mark.parametrize("name,r", [("triangle", 16), ("triangle", 17), ("triangle", 20), ("triangle", 22),
                                    ("carpet", 9), ("carpet", 12), ("vicsek", 14), ("wide", 11), ("k127", 4)])
def test_maps_mfma_sampled_large(name, r):
    """Levels past 16 (two instructions per product) and N above 2^32 (64-bit digits)."""
    torch = torch_or_skip()
    F, O = fractal_pair(name, r)
    rng = np.random.default_rng(r + 100)
    c = rng.integers(0, F.cells, 100_000, dtype=np.uint64)
    c[:4] = [0, 1, F.cells - 2, F.cells - 1]
    ct = torch.from_numpy(c.view(np.int64)).cuda()
    xy = F.lambda_map(ct, impl="mfma")
    mismatch(to_np(xy), O.lam(c), f"lambda mfma {name} r={r}")
    mismatch(to_np(F.nu_map(xy, impl="mfma")), c.view(np.int64), "nu o lambda")
    pts = rng.integers(-1, F.n + 1, (100_000, 2)).astype(np.int32)
    pts[:6] = [[0, 0], [F.n - 1, 0], [0, F.n - 1], [F.n - 1, F.n - 1], [-2 ** 31, 5], [2 ** 31 - 1, 0]]
    pt = torch.from_numpy(pts).cuda()
    got = F.nu_map(pt, impl="mfma")
    mismatch(to_np(got), O.nu(pts.astype(np.int64)), f"nu mfma {name} r={r}")
    assert torch.equal(got, F.nu_map(pt, impl="scalar"))


LIFE = [("triangle", 0), ("triangle", 1), ("triangle", 5), ("triangle", 10), ("triangle_paper", 9), ("carpet", 2),
        ("carpet", 5), ("vicsek", 3), ("vicsek", 7), ("wide", 4)]


@pytest.mark.parametrize("name,r", LIFE)
def test_life_cell_mfma_matches_oracle(name, r):
    torch = torch_or_skip()
    F, O = fractal_pair(name, r)
    start = O.fill_compact(2201, 0.5)
    a = F.fill_bernoulli(2201, 0.5)
    b = torch.empty_like(a)
    F.compact_step(a, b, impl="cell_mfma")
    nb = O.neighbour_table()
    mismatch(to_np(b), O.life_steps(start, 1, nb), f"cell_mfma {name} r={r}")
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(5):
        F.compact_step(x, y, impl="cell_mfma")
        x, y = y, x
    mismatch(to_np(x), O.life_steps(start, 5, nb), f"cell_mfma {name} r={r} 5 steps")


@pytest.mark.parametrize("r", [16, 17])
def test_life_cell_mfma_equals_tile_large(r):
    """The benchmark level (r=16, one instruction per product) and r=17 (two)."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", r)
    a = F.fill_bernoulli(2201, 0.5)
    x1, y1 = a.clone(), torch.empty_like(a)
    x2, y2 = a.clone(), torch.empty_like(a)
    for _ in range(3):
        F.compact_step(x1, y1, impl="cell_mfma")
        F.compact_step(x2, y2, impl="tile")
        x1, y1, x2, y2 = y1, x1, y2, x2
    assert torch.equal(x1, x2)
    del a, x1, y1, x2, y2
    torch.cuda.empty_cache()


def test_mfma_unsupported_and_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    offs = tuple((i % 12, i // 12) for i in range(128))
    F = sqz.Fractal(12, offs, 1)  # k = 128: digits do not fit int8
    idx = torch.arange(10, dtype=torch.int64, device="cuda")
    with pytest.raises(sqz.SqueezeError) as e:
        F.lambda_map(idx, impl="mfma")
    assert e.value.status == 5
    with pytest.raises(sqz.SqueezeError) as e:
        F.nu_map(torch.zeros((4, 2), dtype=torch.int32, device="cuda"), impl="mfma")
    assert e.value.status == 5
    a = F.fill_bernoulli(1, 0.5)
    with pytest.raises(sqz.SqueezeError) as e:
        F.compact_step(a, torch.empty_like(a), impl="cell_mfma")
    assert e.value.status == 5
    # the scalar maps still serve this pattern
    mismatch(to_np(F.lambda_map(idx)), np.array([[i % 12, i // 12] for i in range(10)]), "scalar lambda k=128")
    import ctypes

    L = sqz._lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = torch.empty((10, 2), dtype=torch.int32, device="cuda")
    assert L.sqz_lambda_map_impl(F._h, 7, ctypes.c_void_p(idx.data_ptr()), 10, ctypes.c_void_p(out.data_ptr()), s) == 1
