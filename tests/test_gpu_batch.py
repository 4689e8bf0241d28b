"""GPU parity of batched Life: every instance of a mixed batch equals the oracle
(small levels) or its own single-fractal run (large levels); graph replays equal
eager steps; autotuning does not change results."""
import numpy as np
import pytest

from gpu_common import mismatch, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

MIX_SMALL = [("triangle", 0), ("triangle", 2), ("triangle", 3), ("triangle", 7), ("carpet", 0), ("carpet", 1),
             ("carpet", 3), ("carpet", 4), ("vicsek", 1), ("vicsek", 2), ("vicsek", 5), ("triangle_paper", 6),
             ("triangle", 9), ("carpet", 5), ("vicsek", 6)]


def build(names_levels):
    import fractals as FR
    import paper_2201_00613_amd as sqz

    fr = [sqz.Fractal(*FR.ALL[n], r) for n, r in names_levels]
    return fr, sqz.Batch(fr)


def test_small_mixed_batch_matches_oracle():
    torch = torch_or_skip()
    import fractals as FR
    import oracle

    fr, B = build(MIX_SMALL)
    seeds = [1000 + i for i in range(len(fr))]
    a = B.fill_bernoulli(seeds, 0.5)
    b = B.empty_state()
    starts, nbs = [], []
    for i, (n, r) in enumerate(MIX_SMALL):
        O = oracle.Fractal(*FR.ALL[n], r)
        starts.append(O.fill_compact(seeds[i], 0.5))
        nbs.append((O, O.neighbour_table()))
        mismatch(to_np(B.instance(a, i)), starts[-1], f"fill {n} r={r}")
    B.step(a, b)
    for i, (n, r) in enumerate(MIX_SMALL):
        O, nb = nbs[i]
        mismatch(to_np(B.instance(b, i)), O.life_steps(starts[i], 1, nb), f"batch step {n} r={r}")
    x = B.fill_bernoulli(seeds, 0.5)
    res = B.run(x, torch.empty_like(x), 9)
    for i, (n, r) in enumerate(MIX_SMALL):
        O, nb = nbs[i]
        mismatch(to_np(B.instance(res, i)), O.life_steps(starts[i], 9, nb), f"batch run {n} r={r}")


def test_multi_step_runs_equal_eager_steps():
    """Every instance is in a group of a multi-step kernel (single-tile ones
    included): triangle and Vicsek tiles and carpet bit rows take up to ten
    steps per launch; any step count equals that many one-step launches."""
    torch = torch_or_skip()
    spec = [("triangle", 9), ("carpet", 5), ("vicsek", 6), ("carpet", 3), ("triangle", 12), ("vicsek", 3),
            ("triangle_paper", 10), ("carpet", 6)]
    fr, B = build(spec)
    assert B.steps_per_launch == 10
    seeds = [31 * i + 1 for i in range(len(fr))]
    for steps in (1, 2, 3, 4, 5, 6, 7, 9, 10, 11, 13, 14, 20, 21, 23):
        a, b = B.fill_bernoulli(seeds, 0.5), B.empty_state()
        res = B.run(a, b, steps)
        assert res is (a if steps % 2 == 0 else b)
        x, y = B.fill_bernoulli(seeds, 0.5), B.empty_state()
        for _ in range(steps):
            B.step(x, y)
            x, y = y, x
        assert torch.equal(res, x), steps


def test_large_batch_equals_single_instance_runs():
    torch = torch_or_skip()
    spec = [("triangle", 12), ("carpet", 6), ("vicsek", 8), ("triangle", 14), ("carpet", 7), ("vicsek", 9),
            ("triangle", 1), ("carpet", 2)]
    fr, B = build(spec)
    seeds = [7 * i + 3 for i in range(len(fr))]
    a = B.fill_bernoulli(seeds, 0.5)
    res = B.run(a, B.empty_state(), 12)
    for i, F in enumerate(fr):
        x = F.fill_bernoulli(seeds[i], 0.5)
        y = F.compact_run(x, torch.empty_like(x), 12)
        assert torch.equal(B.instance(res, i), y), spec[i]


def test_graph_replays_equal_eager_steps():
    torch = torch_or_skip()
    spec = [("triangle", 11), ("carpet", 5), ("vicsek", 7), ("triangle", 4)]
    fr, B = build(spec)
    seeds = [5, 6, 7, 8]
    # eager reference: 6 single steps
    e = B.fill_bernoulli(seeds, 0.4)
    f = B.empty_state()
    for k in range(6):
        B.step(e, f) if k % 2 == 0 else B.step(f, e)
    want = e.clone()
    # the same 6 steps as one captured graph, replayed 3 times with eager work between
    for rep in range(3):
        g = B.fill_bernoulli(seeds, 0.4)
        h = B.empty_state()
        res = B.run(g, h, 6)
        torch.cuda.synchronize()
        assert torch.equal(res, want), rep
        scratch = B.fill_bernoulli([1, 2, 3, 4], 0.5)
        B.step(scratch, B.empty_state())
        torch.cuda.synchronize()
    # re-running on the same buffers replays the cached graph
    g2 = B.fill_bernoulli(seeds, 0.4)
    g.copy_(g2)
    h.zero_()
    assert torch.equal(B.run(g, h, 6), want)


def test_mixed_groups_and_persistent_launch():
    """Groups (tiles, bit rows) and instances of the persistent launch (expanded
    tiles of another pattern, thread-level cells) in one batch: runs of several
    lengths equal the instances' own single-fractal runs."""
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    wide = (4, ((0, 0), (1, 0), (3, 0), (0, 1), (2, 1), (3, 1), (1, 2), (2, 2), (0, 3), (3, 3)))
    import fractals as FR

    fr = [sqz.Fractal(*FR.ALL["triangle"], 11), sqz.Fractal(*wide, 5), sqz.Fractal(*FR.ALL["carpet"], 1),
          sqz.Fractal(*FR.ALL["carpet"], 6), sqz.Fractal(*FR.ALL["vicsek"], 7), sqz.Fractal(*FR.ALL["triangle"], 2)]
    B = sqz.Batch(fr)
    seeds = [3, 4, 5, 6, 7, 8]
    for steps in (1, 4, 7, 10):
        a = B.fill_bernoulli(seeds, 0.5)
        res = B.run(a, B.empty_state(), steps)
        for i, F in enumerate(fr):
            x = F.fill_bernoulli(seeds[i], 0.5)
            y = F.compact_run(x, torch.empty_like(x), steps)
            assert torch.equal(B.instance(res, i), y), (i, steps)


@pytest.mark.parametrize("form,steps_per_launch,wg", [("persistent", 0, 0), ("persistent", 3, 2),
                                                     ("persistent", 6, 4), ("persistent", 1, 1),
                                                     ("per_tile", 0, 0), ("per_tile", 4, 0), ("per_tile", 1, 0)])
def test_single_tiled_launch_equals_groups(form, steps_per_launch, wg):
    """The tiled instances as one launch over all of them (persistent with any grid,
    or a workgroup per tile; any steps per launch) give the same states as the
    per-group launches, next to instances of the other persistent launch."""
    torch = torch_or_skip()
    spec = [("triangle", 9), ("carpet", 5), ("vicsek", 6), ("carpet", 2), ("triangle", 12), ("vicsek", 3),
            ("triangle_paper", 10), ("carpet", 6), ("triangle", 1), ("carpet", 0)]
    fr, B = build(spec)
    seeds = [17 * i + 5 for i in range(len(fr))]
    for steps in (1, 5, 12):
        a = B.fill_bernoulli(seeds, 0.5)
        want = B.run(a, B.empty_state(), steps).clone()
        B.set_tiled_launch(form, steps_per_launch, wg)
        if steps_per_launch:
            assert B.steps_per_launch <= steps_per_launch
        x = B.fill_bernoulli(seeds, 0.5)
        got = B.run(x, B.empty_state(), steps)
        assert torch.equal(got, want), steps
        B.set_tiled_launch(False)


def test_tiled_launch_query():
    torch_or_skip()
    fr, B = build([("triangle", 9), ("carpet", 5), ("vicsek", 6)])
    assert B.tiled_launch["form"] == "groups"
    B.set_tiled_launch("persistent", 3, 2)
    assert B.tiled_launch == {"form": "persistent", "steps_per_launch": 3, "wg_per_cu": 2}
    B.set_tiled_launch("per_tile", 5)
    assert B.tiled_launch == {"form": "per_tile", "steps_per_launch": 5, "wg_per_cu": 0}
    assert B.steps_per_launch == 5
    import paper_2201_00613_amd as sqz

    wide = (4, ((0, 0), (1, 0), (3, 0), (0, 1), (2, 1), (3, 1), (1, 2), (2, 2), (0, 3), (3, 3)))
    C = sqz.Batch([sqz.Fractal(*wide, 3)])  # expanded tiles only: no tiled instance
    assert C.tiled_launch["form"] is None


def test_tiled_launch_arguments():
    torch_or_skip()
    import paper_2201_00613_amd as sqz

    fr, B = build([("triangle", 9), ("carpet", 5)])
    for bad in ((3, 0, 0), (-1, 0, 0), (1, -1, 0), (1, 11, 0), (1, 0, -1), (1, 0, 1000)):
        with pytest.raises(sqz.SqueezeError) as e:
            B.set_tiled_launch(*bad)
        assert e.value.status == 1
    B.set_tiled_launch(True, 6, 2)
    assert B.steps_per_launch == 6


def test_autotune_keeps_results():
    torch = torch_or_skip()
    spec = [("triangle", 13), ("carpet", 6), ("vicsek", 8)]
    fr, B = build(spec)
    a = B.fill_bernoulli([1, 2, 3], 0.5)
    ref = B.run(a.clone(), B.empty_state(), 4).clone()
    w = B.autotune(B.fill_bernoulli([9, 9, 9], 0.5), B.empty_state())
    assert w >= 1
    assert torch.equal(B.run(a.clone(), B.empty_state(), 4), ref)


def test_batched_workload_512_instances():
    """The batched workload (512 instances drawn from seed, 7.9e8 cells): 50 steps in
    one graph equal the instances' own single-fractal runs; sampled cells of a few
    instances equal the oracle's light cones."""
    torch = torch_or_skip()
    import oracle
    import paper_2201_00613_amd as sqz
    from paper_2201_00613_amd import workloads as W

    inst = W.batch_instances(512, 2201)
    cache = {}
    fr = []
    for name, s, offs, r, seed in inst:
        if (name, r) not in cache:
            cache[(name, r)] = sqz.Fractal(s, offs, r)
        fr.append(cache[(name, r)])
    B = sqz.Batch(fr)
    seeds = [x[4] for x in inst]
    a = B.fill_bernoulli(seeds, 0.5)
    res = B.run(a, B.empty_state(), 50)
    torch.cuda.synchronize()
    for i in range(0, 512, 37):
        F = fr[i]
        x = F.fill_bernoulli(seeds[i], 0.5)
        y = F.compact_run(x, torch.empty_like(x), 50)
        assert torch.equal(B.instance(res, i), y), inst[i][:4]
    rng = np.random.default_rng(4)
    for i in (0, 1, 2, 511):
        name, s, offs, r, seed = inst[i]
        O = oracle.Fractal(s, offs, r)
        c = rng.integers(0, O.N, 200)
        got = to_np(B.instance(res, i)[torch.from_numpy(c).cuda()])
        mismatch(got, O.light_cone(seed, 0.5, O.lam(c), 50), f"instance {i} {name} r={r}")
    del a, res, B
    torch.cuda.empty_cache()


def test_batch_argument_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    fr, B = build([("triangle", 5), ("carpet", 3)])
    a = B.empty_state()
    with pytest.raises(sqz.SqueezeError):
        B.step(a, a)
    big = torch.zeros(B.total_bytes + 16, dtype=torch.uint8, device="cuda")
    L = sqz._lib.lib()
    import ctypes

    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sqz_batch_step(B._h, ctypes.c_void_p(big.data_ptr() + 1), ctypes.c_void_p(a.data_ptr()), s) == 1
    assert L.sqz_batch_create(0, None, ctypes.byref(ctypes.c_void_p())) == 1


def test_large_triangle_in_a_batch():
    """A level-16 triangle (level-10 tiles of its own kernel) in a batch runs in the
    batch's expanded-tile launch; its states equal its own compact_run."""
    torch = torch_or_skip()
    spec = [("triangle", 16), ("carpet", 5), ("vicsek", 6), ("triangle", 10)]
    fr, B = build(spec)
    seeds = [5, 6, 7, 8]
    for steps in (1, 7, 12):
        a = B.fill_bernoulli(seeds, 0.5)
        res = B.run(a, B.empty_state(), steps)
        for i, F in enumerate(fr):
            x = F.fill_bernoulli(seeds[i], 0.5)
            y = F.compact_run(x, torch.empty_like(x), steps)
            assert torch.equal(B.instance(res, i), y), (i, steps)
    del B, fr
    torch.cuda.empty_cache()
