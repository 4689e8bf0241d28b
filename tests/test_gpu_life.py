"""GPU parity of the Life step (thread-level, tiled, bounding box) against the oracle."""
import ctypes

import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

SMALL = [("triangle", r) for r in range(0, 11)] + [("triangle_paper", 5), ("triangle_paper", 9),
                                                   ("carpet", 1), ("carpet", 3), ("carpet", 5),
                                                   ("vicsek", 1), ("vicsek", 2), ("vicsek", 4), ("vicsek", 7)]


def impls(F):
    return ["cell", "tile"] if F.has_tile else ["cell"]


@pytest.mark.parametrize("name,r", SMALL)
@pytest.mark.parametrize("seed,p", [(2201, 0.5), (77, 0.3)])
def test_step_and_run_match_oracle(name, r, seed, p):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    start = O.fill_compact(seed, p)
    want1 = O.life_compact(start)
    want7 = O.life_steps(start, 7)
    for impl in impls(F):
        a = F.fill_bernoulli(seed, p)
        b = torch.empty_like(a)
        F.compact_step(a, b, impl=impl)
        mismatch(to_np(b), want1, f"{name} r={r} {impl} 1 step")
        x, y = a.clone(), torch.empty_like(a)
        for i in range(7):
            F.compact_step(x, y, impl=impl)
            x, y = y, x
        mismatch(to_np(x), want7, f"{name} r={r} {impl} 7 steps")


@pytest.mark.parametrize("name,r", [("triangle", 10), ("carpet", 4)])
def test_all_alive_and_empty(name, r):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    for fill in (0, 1):
        a = torch.full((F.cells,), fill, dtype=torch.uint8, device="cuda")
        want = O.life_compact(np.full(F.cells, fill, np.uint8))
        for impl in impls(F):
            b = torch.empty_like(a)
            F.compact_step(a, b, impl=impl)
            mismatch(to_np(b), want, f"{name} all={fill} {impl}")
    if name == "triangle":
        assert want.sum() == 26245


def test_compact_run_parity_and_placement():
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 9), oracle_fractal("triangle", 9)
    start = O.fill_compact(5, 0.5)
    for steps in (0, 1, 4, 5):
        a = F.fill_bernoulli(5, 0.5)
        b = torch.zeros_like(a)
        res = F.compact_run(a, b, steps)
        assert res is (a if steps % 2 == 0 else b)
        mismatch(to_np(res), O.life_steps(start, steps) if steps else start, f"run {steps}")


def test_r16_one_step_ranges_and_light_cones():
    """Level-16 triangle (43M cells): one step compared on the first, a middle and the
    last 3M cells; 100 steps (tiled) compared on light-cone samples."""
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 16), oracle_fractal("triangle", 16)
    seed, p = 2201, 0.5
    a = F.fill_bernoulli(seed, p)
    b = torch.empty_like(a)
    start = O.fill_compact(seed, p)
    mismatch(to_np(a), start, "fill r=16")
    F.compact_step(a, b, impl="tile")
    got = to_np(b)
    for c0 in (0, F.cells // 2, F.cells - 3_000_000):
        mismatch(got[c0:c0 + 3_000_000], O.life_compact(start, c0, c0 + 3_000_000), f"r16 range {c0}")
    res = F.compact_run(a, b, 100)
    rng = np.random.default_rng(16)
    c = rng.integers(0, F.cells, 600)
    c[:3] = [0, F.cells // 2, F.cells - 1]
    xy = O.lam(c)
    mismatch(to_np(res[torch.from_numpy(c).cuda()]), O.light_cone(seed, p, xy, 100), "r16 100 steps")


def test_r16_tile_equals_cell_and_bb():
    """Three GPU kernels on the level-16 triangle agree after 10 steps: tiled, thread-level,
    and the bounding-box grid gathered through lambda."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 16)
    a = F.fill_bernoulli(3, 0.5)
    t1, t2 = a.clone(), torch.empty_like(a)
    c1, c2 = a.clone(), torch.empty_like(a)
    rt = F.compact_run(t1, t2, 10)
    for i in range(10):
        F.compact_step(c1, c2, impl="cell")
        c1, c2 = c2, c1
    assert torch.equal(rt, c1)
    e1 = F.fill_bernoulli(3, 0.5, layout="expanded")
    e2 = torch.empty_like(e1)
    for i in range(10):
        F.expanded_step(e1, e2)
        e1, e2 = e2, e1
    xy = F.lambda_map(torch.arange(F.cells, dtype=torch.int64, device="cuda")).long()
    gathered = e1[xy[:, 1] * F.n + xy[:, 0]]
    assert torch.equal(gathered, rt)
    assert int(e1.sum()) == int(rt.sum())  # holes stayed 0
    del e1, e2, xy, gathered
    torch.cuda.empty_cache()


def test_r20_light_cones():
    """Level-20 triangle (3.49e9 cells, expanded form 1.1 TB): one step and 20 steps
    (tiled) checked on light-cone samples."""
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 20), oracle_fractal("triangle", 20)
    seed, p = 2201, 0.3
    a = F.fill_bernoulli(seed, p)
    b = torch.empty_like(a)
    rng = np.random.default_rng(20)
    c = rng.integers(0, F.cells, 4000)
    c[:4] = [0, 1, F.cells - 2, F.cells - 1]
    ct = torch.from_numpy(c).cuda()
    xy = O.lam(c)
    F.compact_step(a, b)
    mismatch(to_np(b[ct]), O.light_cone(seed, p, xy, 1), "r20 1 step")
    # a contiguous range across many tile boundaries, exhaustively
    c0 = 1_234_567_891
    mismatch(to_np(b[c0:c0 + 200_000]), _range_step(O, seed, p, c0, 200_000), "r20 range")
    res = F.compact_run(a, b, 20)
    mismatch(to_np(res[ct]), O.light_cone(seed, p, xy, 20), "r20 20 steps")
    del a, b, res
    torch.cuda.empty_cache()


def test_r21_indices_past_2_32():
    """Level-21 triangle (10,460,353,203 cells, 10.5 GB buffers): compact indices
    past 2^32 and tile starts past 2^32 bytes.  One step exhaustively over a range
    across index 2^32, and the thread-level step equal to it over the whole array;
    twelve steps (a ten-step launch and a two-step launch) on
    windows along the tile edges of the tiles around index 2^32 and of the last
    tiles, and on light-cone samples over the whole array."""
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 21), oracle_fractal("triangle", 21)
    assert F.cells > 2 ** 33 and F.tile_level == 10 and not F.resident_run
    seed, p, t = 2201, 0.3, 12
    side = 2 ** F.tile_level
    print("r21: fill and one step", flush=True)
    a = F.fill_bernoulli(seed, p)
    b = torch.empty_like(a)
    F.compact_step(a, b)
    c0 = 2 ** 32 - 100_000
    want1 = _range_step(O, seed, p, c0, 200_000)
    mismatch(to_np(b[c0:c0 + 200_000]), want1, "r21 one step across 2^32")
    print("r21: one thread-level step", flush=True)
    d = torch.empty_like(a)
    F.compact_step(a, d, impl="cell")  # 64-bit lambda, in-chunk neighbours from 64-bit indices
    mismatch(to_np(d[c0:c0 + 200_000]), want1, "r21 one thread-level step across 2^32")
    assert torch.equal(d, b), "r21: thread-level and tiled steps differ"
    del d
    print("r21: twelve steps", flush=True)
    res = F.compact_run(a, b, t)
    assert res is a
    per_tile = 3 ** F.tile_level
    ntiles = F.cells // per_tile
    t32 = 2 ** 32 // per_tile
    tiles = np.array([t32 - 1, t32, t32 + 1, ntiles - 2, ntiles - 1, 0], dtype=np.int64)
    tiles_xy = oracle_fractal("triangle", F.r - F.tile_level).lam(tiles)
    idx, want = [], []
    horiz = [(X * side - 10, Y * side - 10) for X, Y in tiles_xy]
    vert = [(X * side - 10, Y * side + 10) for X, Y in tiles_xy]
    for corners, w, h in ((horiz, side + 20, 20), (vert, 20, side)):
        win = O.life_windows(seed, p, corners, w, h, t)
        for q, (x0, y0) in enumerate(corners):
            yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
            c = O.nu(np.stack([xx.ravel(), yy.ravel()], 1))
            keep = c >= 0
            idx.append(c[keep])
            want.append(win[q].ravel()[keep])
    rng = np.random.default_rng(21)
    c = rng.integers(0, F.cells, 3000)
    c[:6] = [0, 2 ** 32 - 1, 2 ** 32, 2 ** 32 + 1, F.cells - 2, F.cells - 1]
    idx.append(c)
    want.append(O.light_cone(seed, p, O.lam(c), t))
    idx, want = np.concatenate(idx), np.concatenate(want)
    assert int((idx >= 2 ** 32).sum()) > idx.size // 2
    print(f"r21: {idx.size} samples", flush=True)
    mismatch(to_np(res[torch.from_numpy(idx).cuda()]), want, "r21 twelve steps")
    del a, b, res
    torch.cuda.empty_cache()


def _range_step(O, seed, p, c0, count):
    """Oracle one-step states of cells [c0, c0+count) from the seeded start, without
    materialising all N cells: each cell's one-step light cone."""
    xy = O.lam(np.arange(c0, c0 + count, dtype=np.uint64))
    return O.light_cone(seed, p, xy, 1)


@pytest.mark.parametrize("name,r", [("triangle", 4), ("triangle", 10), ("triangle_paper", 7), ("carpet", 3),
                                    ("carpet", 5), ("vicsek", 5)])
def test_expanded_step_matches_oracle(name, r):
    torch = torch_or_skip()
    import oracle

    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    member = O.member()
    grid = O.fill_expanded(11, 0.5)
    a = F.fill_bernoulli(11, 0.5, layout="expanded")
    mismatch(to_np(a).reshape(F.n, F.n), grid, "expanded fill")
    b = torch.empty_like(a)
    F.expanded_step(a, b)
    mismatch(to_np(b).reshape(F.n, F.n), oracle.life_expanded(member, grid), f"BB {name} r={r}")


def test_deterministic_and_checkpoint_resume():
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 14)
    a = F.fill_bernoulli(8, 0.5)
    x1, y1 = a.clone(), torch.empty_like(a)
    full = F.compact_run(x1, y1, 12).clone()
    x2, y2 = a.clone(), torch.empty_like(a)
    again = F.compact_run(x2, y2, 12)
    assert torch.equal(full, again)
    x3, y3 = a.clone(), torch.empty_like(a)
    half = F.compact_run(x3, y3, 6).cpu()  # checkpoint to host
    x4 = half.cuda()
    y4 = torch.empty_like(x4)
    assert torch.equal(F.compact_run(x4, y4, 6), full)


def test_error_paths():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    L = sqz._lib.lib()
    F = gpu_fractal("triangle", 6)
    a = F.fill_bernoulli(1, 0.5)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = ctypes.c_void_p(a.data_ptr())
    assert L.sqz_compact_step(F._h, p, p, s) == 1  # aliasing
    assert L.sqz_compact_step(F._h, p, ctypes.c_void_p(a.data_ptr() + 5), s) == 1  # overlap
    assert L.sqz_compact_step(F._h, None, p, s) == 1
    assert L.sqz_lambda_map(F._h, p, -1, p, s) == 1
    assert L.sqz_lambda_map(F._h, None, 0, None, s) == 0
    assert L.sqz_compact_run(F._h, p, p, 3, s) == 1
    assert L.sqz_compact_run(F._h, p, ctypes.c_void_p(a.data_ptr() + 4096), -1, s) == 1
    assert L.sqz_fill_bernoulli(F._h, 1, 1.5, 0, p, s) == 1
    # misaligned buffers: the tiled kernel refuses, AUTO takes the thread-level path
    big = torch.zeros(2 * F.cells + 64, dtype=torch.uint8, device="cuda")
    src = big[1:1 + F.cells]
    src.copy_(a)
    dst = big[F.cells + 33:2 * F.cells + 33]
    assert L.sqz_compact_step_impl(F._h, 2, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), s) == 1
    F.compact_step(src, dst)
    ref = torch.empty_like(a)
    F.compact_step(a, ref, impl="cell")
    assert torch.equal(dst, ref)
    # patterns without a tiled kernel
    C = gpu_fractal("carpet", 3)
    assert not C.has_tile
    c = C.fill_bernoulli(1, 0.5)
    with pytest.raises(sqz.SqueezeError) as e:
        C.compact_step(c, torch.empty_like(c), impl="tile")
    assert e.value.status == 5
    # bounding box at r=20 cannot fit: refused before any allocation or launch
    T20 = gpu_fractal("triangle", 20)
    q = ctypes.c_void_p(16)
    assert L.sqz_expanded_step(T20._h, q, ctypes.c_void_p(32), s) == 2
    assert b"exceed" in L.sqz_last_error()
    # a handle used on the wrong device is refused (only one device here: nothing to test)
    info = sqz._lib.Info()
    assert L.sqz_fractal_info(F._h, ctypes.byref(info)) == 0 and info.cells == 3 ** 6


# A 4 x 4 frame: the twelve border cells of the box are the replicas.
FRAME4 = (4, tuple((x, y) for y in range(4) for x in range(4) if x in (0, 3) or y in (0, 3)))


def test_thread_level_step_and_nu_with_large_map_tables():
    """The thread-level step copies all four map tables into LDS and the nu kernel its
    two: on the 4 x 4 frame at level 6 (2,985,984 cells) they are 11,648 words (46.6 KB)
    and 8,192 words (32 KB).  One and three thread-level steps over the whole array
    against the oracle's neighbour-table steps; nu over every point of a 1,030 x 1,030
    window of the box and its surroundings against the oracle's nu, and nu(lambda(c)) = c
    for every cell."""
    torch = torch_or_skip()
    import oracle
    import paper_2201_00613_amd as sqz

    s, offs = FRAME4
    F, O = sqz.Fractal(s, offs, 6), oracle.Fractal(s, offs, 6)
    assert F.cells == 12 ** 6
    start = O.fill_compact(5, 0.35)
    a = F.fill_bernoulli(5, 0.35)
    mismatch(to_np(a), start, "frame fill")
    nb = O.neighbour_table()
    b = torch.empty_like(a)
    F.compact_step(a, b, impl="cell")
    mismatch(to_np(b), O.life_steps(start, 1, nb), "frame: one thread-level step")
    x, y = b, a
    for _ in range(2):
        F.compact_step(x, y, impl="cell")
        x, y = y, x
    mismatch(to_np(x), O.life_steps(start, 3, nb), "frame: three thread-level steps")
    del nb
    idx = torch.arange(F.cells, dtype=torch.int64, device="cuda")
    mismatch(to_np(F.nu_map(F.lambda_map(idx))), np.arange(F.cells), "frame: nu o lambda")
    ys, xs = np.mgrid[-1:1029, F.n - 1029:F.n + 1]
    pts = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
    got = to_np(F.nu_map(torch.from_numpy(pts).cuda()))
    mismatch(got, O.nu(pts.astype(np.int64)), "frame: nu over a window")
