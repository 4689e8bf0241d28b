"""Oracle parity of the kernels behind the headline figures: the bit-sliced
level-10 triangle tiles that sqz_compact_run uses from level 16 up (Section
"Moving from Thread-level to Block-level"; the Life workload of Section
"Experimental Setup and Results"), in both run forms: the resident run (one
launch, all 729 tiles of the level-16 triangle held in LDS at once, ring
cells exchanged every ten steps; the default at level 16 from 10 steps) and
launches of ten steps (the form of every larger level).

* Level 16, seed 2201, Bernoulli(0.5): all 43,046,721 cells after 20 steps
  and after 100 steps, in each run form, against the oracle's neighbour-table
  steps, and the bounding-box grid after the same steps gathered through the
  oracle's replication order.
* Level 20, seed 2201, Bernoulli(0.3), 20 steps: more than a million cells
  against the oracle's window light cones, more than half of them within
  distance 10 of their tile's box edge (where the ring cells that a
  ten-step launch advances in LDS sit) and the rest in uniformly drawn
  level-7 subtrees.
"""
import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu


_R16 = {}


def r16_oracle():
    """The oracle's level-16 start (seed 2201, Bernoulli(0.5)) and its states after 20
    and 100 steps, computed once per session."""
    if not _R16:
        O = oracle_fractal("triangle", 16)
        start = O.fill_compact(2201, 0.5)
        print("r16: oracle neighbour table", flush=True)
        nb = O.neighbour_table()
        _R16[0] = start
        _R16[20] = O.life_steps(start, 20, nb)
        _R16[100] = O.life_steps(_R16[20], 80, nb)
        del nb
    return _R16


@pytest.mark.parametrize("form", ["resident", "launches"])
def test_r16_full_array_20_and_100_steps(form):
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 16), oracle_fractal("triangle", 16)
    assert F.tile_level == 10 and F.run_steps_per_launch == 10 and F.resident_run
    seed, p = 2201, 0.5
    want = r16_oracle()
    a = F.fill_bernoulli(seed, p)
    mismatch(to_np(a), want[0], "fill r=16")
    for steps in (20, 100):
        print(f"r16: {steps} steps, full array, {form}", flush=True)
        x, y = a.clone(), torch.empty_like(a)
        res = F.compact_run(x, y, steps, form=form)
        assert res is x  # even step count: result in the first buffer
        mismatch(to_np(res), want[steps], f"r16 {steps} steps ({form})")
        del x, y, res
    if form != "launches":
        return
    # the bounding-box kernel over the same steps, gathered through the oracle's order
    order = torch.from_numpy(O.order().astype(np.int64)).cuda()
    gidx = order[:, 1] * F.n + order[:, 0]
    del order
    e1 = F.fill_bernoulli(seed, p, layout="expanded")
    e2 = torch.empty_like(e1)
    done = 0
    for steps in (20, 100):
        print(f"r16: bounding box to {steps} steps", flush=True)
        for _ in range(steps - done):
            F.expanded_step(e1, e2)
            e1, e2 = e2, e1
        done = steps
        mismatch(to_np(e1[gidx]), want[steps], f"r16 bounding box {steps} steps")
        assert int(e1.sum()) == int(want[steps].sum())  # holes stayed dead
    del e1, e2, gidx
    torch.cuda.empty_cache()


def _strip_samples(O, tiles_xy, side):
    """Rectangles covering the points within distance 10 of each tile's box edges at
    local x = 0 and y = 0, including the contact points at the box corners where
    the tile meets its neighbours.  Every member of a triangle tile within distance
    10 of its other two edges has local x < 10 or y < 10, so the rectangles hold
    them too.  Returns (corners, width, height) per rectangle shape."""
    horiz = [(X * side - 10, Y * side - 10) for X, Y in tiles_xy]  # (side + 20) x 20
    vert = [(X * side - 10, Y * side + 10) for X, Y in tiles_xy]   # 20 x side
    return [(horiz, side + 20, 20), (vert, 20, side)]


def test_r20_ring_weighted_windows():
    torch = torch_or_skip()
    F, O = gpu_fractal("triangle", 20), oracle_fractal("triangle", 20)
    M = F.tile_level
    assert M == 10 and F.run_steps_per_launch == 10
    side = 2 ** M
    seed, p, t = 2201, 0.3, 20
    a = F.fill_bernoulli(seed, p)
    b = torch.empty_like(a)
    print("r20: 20 steps (two ten-step launches)", flush=True)
    res = F.compact_run(a, b, t)
    assert res is a
    rng = np.random.default_rng(2020)
    Otile = oracle_fractal("triangle", F.r - M)
    tiles = rng.choice(Otile.N, size=200, replace=False)
    tiles[:3] = [0, Otile.N // 2, Otile.N - 1]
    tiles_xy = Otile.lam(tiles)
    idx, want, near = [], [], []
    print("r20: oracle strips along tile edges", flush=True)
    for corners, w, h in _strip_samples(O, tiles_xy, side):
        win = O.life_windows(seed, p, corners, w, h, t)
        for q, (x0, y0) in enumerate(corners):
            yy, xx = np.mgrid[y0:y0 + h, x0:x0 + w]
            xy = np.stack([xx.ravel(), yy.ravel()], 1)
            c = O.nu(xy)
            keep = c >= 0
            idx.append(c[keep])
            want.append(win[q].ravel()[keep])
            lx, ly = xy[keep, 0] % side, xy[keep, 1] % side
            near.append(np.minimum(np.minimum(lx, ly), np.minimum(side - 1 - lx, side - 1 - ly)) < 10)
    # uniformly drawn level-7 subtrees: each fills its own 128 x 128 box
    print("r20: oracle windows over random level-7 subtrees", flush=True)
    m7 = 7
    O7 = oracle_fractal("triangle", F.r - m7)
    sub = rng.choice(O7.N, size=600, replace=False)
    box = 2 ** m7
    corners = O7.lam(sub) * box
    win = O.life_windows(seed, p, corners, box, box, t)
    for q, tq in enumerate(sub):
        c = np.arange(int(tq) * 3 ** m7, (int(tq) + 1) * 3 ** m7, dtype=np.int64)
        xy = O.lam(c)
        idx.append(c)
        want.append(win[q][xy[:, 1] - corners[q, 1], xy[:, 0] - corners[q, 0]])
        lx, ly = xy[:, 0] % side, xy[:, 1] % side
        near.append(np.minimum(np.minimum(lx, ly), np.minimum(side - 1 - lx, side - 1 - ly)) < 10)
    idx, want, near = np.concatenate(idx), np.concatenate(want), np.concatenate(near)
    print(f"r20: {idx.size} samples, {int(near.sum())} within distance 10 of a tile edge", flush=True)
    assert idx.size >= 1_000_000 and 2 * int(near.sum()) >= idx.size
    got = to_np(res[torch.from_numpy(idx).cuda()])
    mismatch(got, want, "r20 20 steps, ring-weighted windows")
    del a, b, res
    torch.cuda.empty_cache()
