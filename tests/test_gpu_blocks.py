"""GPU parity of the block-level layouts: the lambda(omega) approach (expanded
array, workgroups over the compact grid of blocks) and micro-block storage
(block-level Squeeze memory), against the oracle and against the compact and
bounding-box kernels."""
import os

import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WIDE = (4, ((0, 0), (1, 0), (3, 0), (0, 1), (2, 1), (3, 1), (1, 2), (2, 2), (0, 3), (3, 3)))


def pair(name, r):
    if name == "wide":
        import oracle
        import paper_2201_00613_amd as sqz

        return sqz.Fractal(*WIDE, r), oracle.Fractal(*WIDE, r)
    return gpu_fractal(name, r), oracle_fractal(name, r)


def expected_blocks(O, compact, m):
    """Micro-block layout written out from the oracle's order: block t = c // k^m
    holds cell c at (y mod s^m) * s^m + (x mod s^m); every other byte is 0."""
    B, km = O.s ** m, O.k ** m
    xy = O.order()
    c = np.arange(O.N)
    out = np.zeros(O.N // km * B * B, dtype=np.uint8)
    out[(c // km) * B * B + (xy[:, 1] % B) * B + xy[:, 0] % B] = compact
    return out


CASES = [("triangle", 1, 0), ("triangle", 1, 1), ("triangle", 6, 0), ("triangle", 6, 2), ("triangle", 6, 3),
         ("triangle", 9, 4), ("triangle", 9, 5), ("triangle", 10, 6), ("triangle_paper", 8, 3), ("carpet", 3, 1),
         ("carpet", 5, 2), ("carpet", 5, 3), ("vicsek", 4, 1), ("vicsek", 6, 3), ("wide", 3, 1), ("wide", 4, 2),
         ("wide", 4, 3)]


@pytest.mark.parametrize("name,r,m", CASES)
def test_microblock_pack_unpack_step(name, r, m):
    torch = torch_or_skip()
    F, O = pair(name, r)
    start = O.fill_compact(2201, 0.5)
    a = F.fill_bernoulli(2201, 0.5)
    assert F.microblock_bytes(m) == O.N // O.k ** m * O.s ** (2 * m)
    blk = F.microblock_pack(a, m)
    mismatch(to_np(blk), expected_blocks(O, start, m), f"pack {name} r={r} m={m}")
    mismatch(to_np(F.microblock_unpack(blk, m)), start, "unpack")
    nb = O.neighbour_table()
    x, y = blk, torch.empty_like(blk)
    for t in range(1, 5):
        F.microblock_step(x, y, m)
        x, y = y, x
        mismatch(to_np(x), expected_blocks(O, O.life_steps(start, t, nb), m), f"microblock step {t} {name} r={r} m={m}")


@pytest.mark.parametrize("name,r,m", CASES)
def test_lambda_omega_matches_oracle_and_bb(name, r, m):
    torch = torch_or_skip()
    import oracle

    F, O = pair(name, r)
    a = F.fill_bernoulli(2201, 0.5, layout="expanded")
    want = O.fill_expanded(2201, 0.5)
    member = O.member()
    x, y = a.clone(), torch.zeros_like(a)
    bx, by = a.clone(), torch.empty_like(a)
    for t in range(1, 5):
        F.lambda_omega_step(x, y, m)
        F.expanded_step(bx, by)
        x, y, bx, by = y, x, by, bx
        want = oracle.life_expanded(member, want)
        mismatch(to_np(x).reshape(F.n, F.n), want, f"lambda(omega) step {t} {name} r={r} m={m}")
        assert torch.equal(x, bx)


def test_microblock_r16_equals_tile():
    """Benchmark level, blocks of side 16 and 64: three steps equal the tiled kernel's."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 16)
    a = F.fill_bernoulli(2201, 0.5)
    ref, tmp = a.clone(), torch.empty_like(a)
    for _ in range(3):
        F.compact_step(ref, tmp, impl="tile")
        ref, tmp = tmp, ref
    for m in (4, 6):
        x = F.microblock_pack(a, m)
        y = torch.empty_like(x)
        for _ in range(3):
            F.microblock_step(x, y, m)
            x, y = y, x
        assert torch.equal(F.microblock_unpack(x, m), ref), m
    del a, ref, tmp, x, y
    torch.cuda.empty_cache()


def test_lambda_omega_r16_equals_compact():
    """Benchmark level: two lambda(omega) steps on the 4.3 GB expanded array, gathered
    through lambda, equal two compact steps."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 16)
    a = F.fill_bernoulli(2201, 0.5, layout="expanded")
    b = torch.zeros_like(a)
    F.lambda_omega_step(a, b, 4)
    F.lambda_omega_step(b, a, 4)
    c = F.fill_bernoulli(2201, 0.5)
    d = torch.empty_like(c)
    F.compact_step(c, d)
    F.compact_step(d, c)
    xy = F.lambda_map(torch.arange(F.cells, dtype=torch.int64, device="cuda")).long()
    assert torch.equal(a[xy[:, 1] * F.n + xy[:, 0]], c)
    assert int(a.sum()) == int(c.sum())  # nothing written outside the fractal
    del a, b, c, d, xy
    torch.cuda.empty_cache()


def test_microblock_memory_matches_paper_table():
    """Micro-block bytes at r=16 for rho = 1..32 reproduce the printed table (4 bytes
    per cell there, 1 here)."""
    torch_or_skip()
    F = gpu_fractal("triangle", 16)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "memory_table_r16.txt")) if l[0] != "#"]
    for rho, bb, sq, mrf in rows:
        m = int(rho).bit_length() - 1
        nbytes = F.microblock_bytes(m)
        assert abs(nbytes * 4 / 2 ** 30 - float(sq)) <= 0.01
        assert round(F.n * F.n / nbytes, 1) == float(mrf)


def test_block_layout_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    F = gpu_fractal("triangle", 8)
    with pytest.raises(sqz.SqueezeError) as e:
        F.microblock_bytes(9)
    assert e.value.status == 2
    with pytest.raises(sqz.SqueezeError) as e:
        F.microblock_bytes(7)  # side 128
    assert e.value.status == 5
    a = F.fill_bernoulli(1, 0.5, layout="expanded")
    with pytest.raises(sqz.SqueezeError) as e:
        F.lambda_omega_step(a, a, 2)
    assert e.value.status == 1
    big = torch.zeros(F.n * F.n + 4, dtype=torch.uint8, device="cuda")
    import ctypes

    L = sqz._lib.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sqz_lambda_omega_step(F._h, 2, ctypes.c_void_p(big.data_ptr() + 1), ctypes.c_void_p(a.data_ptr()), s) == 1
    blk = F.microblock_pack(F.fill_bernoulli(1, 0.5), 3)
    with pytest.raises(sqz.SqueezeError):
        F.microblock_step(blk, blk, 3)
