"""The resident run form of sqz_compact_run_form (one launch, one
workgroup per level-M subtree, every subtree held in LDS for the whole run,
ring cells exchanged through the caller buffers at a grid barrier every
run_steps_per_launch steps; the Life iterations of Section "Experimental Setup
and Results" on the tiles of Section "Moving from Thread-level to
Block-level").  Bit-exact against the oracle and the launches form around
every exchange boundary, over repeated runs, and its argument errors."""
import ctypes

import numpy as np
import pytest

from gpu_common import gpu_fractal, mismatch, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

EDGE_STEPS = [1, 2, 3, 9, 10, 11, 12, 19, 20, 21, 29, 30, 31, 45]


@pytest.mark.parametrize("name,r", [("triangle", 11), ("triangle", 12), ("triangle_paper", 11), ("vicsek", 7)])
def test_exchange_boundaries_against_oracle(name, r):
    torch = torch_or_skip()
    F, O = gpu_fractal(name, r), oracle_fractal(name, r)
    assert F.resident_run
    K = F.run_steps_per_launch
    start = O.fill_compact(77, 0.45)
    nb = O.neighbour_table()
    want, t = {}, 0
    state = start
    for steps in sorted(EDGE_STEPS):
        state = O.life_steps(state, steps - t, nb)
        t = steps
        want[steps] = state
    for steps in EDGE_STEPS:
        a = F.fill_bernoulli(77, 0.45)
        b = torch.full_like(a, 7)  # scratch contents must not matter
        res = F.compact_run(a, b, steps, form="resident")
        assert res is (a if steps % 2 == 0 else b)
        mismatch(to_np(res), want[steps], f"{name} r={r} K={K} {steps} steps (resident)")


@pytest.mark.parametrize("name,r", [("triangle", 13), ("triangle_paper", 12), ("vicsek", 8)])
def test_resident_equals_launches(name, r):
    torch = torch_or_skip()
    F = gpu_fractal(name, r)
    assert F.resident_run
    for seed, p, steps in ((5, 0.5, 33), (6, 0.2, 40), (7, 0.8, 17)):
        a = F.fill_bernoulli(seed, p)
        r1 = F.compact_run(a.clone(), torch.empty_like(a), steps, form="resident")
        r2 = F.compact_run(a.clone(), torch.empty_like(a), steps, form="launches")
        assert torch.equal(r1, r2), (name, r, seed, steps)


def test_back_to_back_runs_equal_one_run():
    """The grid-barrier counts carry over from run to run: six runs of 7 steps in a row
    on one stream equal one run of 42 steps (and the launches form)."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 16)
    assert F.resident_run
    a = F.fill_bernoulli(2201, 0.5)
    whole = F.compact_run(a.clone(), torch.empty_like(a), 42, form="resident")
    x, y = a.clone(), torch.empty_like(a)
    for _ in range(6):
        x = F.compact_run(x, y, 7, form="resident")
        y = torch.empty_like(x)
    assert torch.equal(x, whole)
    ref = F.compact_run(a.clone(), torch.empty_like(a), 42, form="launches")
    assert torch.equal(whole, ref)
    del a, whole, x, y, ref
    torch.cuda.empty_cache()


def test_runs_of_mixed_lengths_in_a_row():
    """Runs of 1, 2, 9, 10, 11, 25, 0, 3 and 20 steps in a row (each passing a different
    number of barriers, the 0-step run one) equal the launches form over the same
    steps, after every run."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 12)
    assert F.resident_run
    a = F.fill_bernoulli(91, 0.4)
    x, y = a.clone(), torch.empty_like(a)
    u, v = a.clone(), torch.empty_like(a)
    for steps in (1, 2, 9, 10, 11, 25, 0, 3, 20):
        x1 = F.compact_run(x, y, steps, form="resident")
        y = x if x1 is y else y
        x = x1
        u1 = F.compact_run(u, v, steps, form="launches")
        v = u if u1 is v else v
        u = u1
        assert torch.equal(x, u), steps


def test_graph_replays_of_a_resident_run():
    """A resident run of 20 steps captured once into a graph and replayed three times,
    with eager work and synchronisation between the replays: after replay k the
    state equals 20 k steps of the launches form."""
    torch = torch_or_skip()
    F = gpu_fractal("triangle", 12)
    assert F.resident_run
    a = F.fill_bernoulli(17, 0.5)
    x, y = a.clone(), torch.empty_like(a)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture, then restore the start
        F.compact_run(x, y, 20, form="resident")
        x.copy_(a)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = F.compact_run(x, y, 20, form="resident")
    assert res is x
    torch.cuda.synchronize()
    assert torch.equal(x, a)  # capture records, it does not run
    u, v = a.clone(), torch.empty_like(a)
    for k in range(1, 4):
        g.replay()
        torch.cuda.synchronize()
        u = F.compact_run(u, v, 20, form="launches")  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(x, u), k
    del g


def _launch_count(steps, K):
    """Launches of the launches form: full groups of K, the rest, and one more
    one-step launch when their count's parity differs from the step count's."""
    n = steps // K + (1 if steps % K else 0)
    return n + (1 if steps >= 1 and (n & 1) != (steps & 1) else 0)


def test_zero_steps_and_auto_choice():
    """The auto form is the resident run for 10 steps and more, and below that where the
    launches form needs an extra one-step launch for the result's buffer (never for
    fewer than two steps); either way the results equal the explicit forms'."""
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    F = gpu_fractal("triangle", 10)
    assert F.resident_run
    K = F.run_steps_per_launch
    a = F.fill_bernoulli(3, 0.5)
    keep = a.clone()
    assert F.compact_run(a, torch.empty_like(a), 0, form="resident") is a
    assert torch.equal(a, keep)
    for steps in range(0, 61):
        want = steps >= 2 and (steps >= 10 or _launch_count(steps, K) > -(-steps // K))
        assert F.auto_run_form(steps) == ("resident" if want else "launches"), steps
    for steps in (5, 9, 10, 11, 20, 25, 31):
        r_auto = F.compact_run(a.clone(), torch.empty_like(a), steps)
        r_res = F.compact_run(a.clone(), torch.empty_like(a), steps, form="resident")
        r_lau = F.compact_run(a.clone(), torch.empty_like(a), steps, form="launches")
        assert torch.equal(r_auto, r_res) and torch.equal(r_auto, r_lau), steps
    G = gpu_fractal("triangle", 20)  # no resident run: always launches
    assert not G.resident_run and all(G.auto_run_form(t) == "launches" for t in (2, 30, 100))
    L = sqz._lib.lib()
    form = ctypes.c_int(-1)
    assert L.sqz_run_form_auto(F._h, -1, ctypes.byref(form)) == 1 and form.value == -1
    assert L.sqz_run_form_auto(F._h, 4, None) == 1
    assert L.sqz_run_form_auto(None, 4, ctypes.byref(form)) == 1


def test_argument_errors():
    torch = torch_or_skip()
    import paper_2201_00613_amd as sqz

    L = sqz._lib.lib()
    F = gpu_fractal("triangle", 20)  # 59,049 level-10 tiles: more than the chip holds at once
    assert not F.resident_run and F.run_steps_per_launch == 10
    a = torch.zeros(16, dtype=torch.uint8, device="cuda")  # never touched: the calls fail first
    s = torch.cuda.current_stream().cuda_stream
    p, q = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr() + (1 << 40))
    assert L.sqz_compact_run_form(F._h, 2, p, q, 4, ctypes.c_void_p(s)) == 5  # unsupported
    G = gpu_fractal("triangle", 10)
    assert G.resident_run
    x = torch.zeros(G.cells + 64, dtype=torch.uint8, device="cuda")
    y = torch.zeros(G.cells + 64, dtype=torch.uint8, device="cuda")
    px, py = ctypes.c_void_p(x.data_ptr() + 1), ctypes.c_void_p(y.data_ptr())
    assert L.sqz_compact_run_form(G._h, 2, px, py, 4, ctypes.c_void_p(s)) == 1  # unaligned
    px = ctypes.c_void_p(x.data_ptr())
    assert L.sqz_compact_run_form(G._h, 7, px, py, 4, ctypes.c_void_p(s)) == 1  # unknown form
    assert L.sqz_compact_run_form(G._h, 2, px, py, -1, ctypes.c_void_p(s)) == 1  # negative steps
    assert L.sqz_compact_run_form(G._h, 2, px, px, 4, ctypes.c_void_p(s)) == 1  # overlap
    torch.cuda.synchronize()
    assert int(x.sum()) == 0 and int(y.sum()) == 0
