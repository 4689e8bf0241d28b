"""Accuracy of the diffusion forms over the full 1000-step horizon, against the
binary64 oracle on the level-7 carpet (2,097,152 cells; the level-9 workload is
checked through light cones and mass in test_gpu_xtile).  Errors are the
relative infinity norm at t = 1, 10, 100, 1000."""
import numpy as np
import pytest

from gpu_common import gpu_fractal, oracle_fractal, to_np, torch_or_skip

pytestmark = pytest.mark.gpu

A = 0.1
CHECKPOINTS = (1, 10, 100, 1000)


def rel_inf(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def test_carpet_r7_1000_steps(record_property):
    torch = torch_or_skip()
    F, O = gpu_fractal("carpet", 7), oracle_fractal("carpet", 7)
    u0 = O.fill_uniform_compact(2201)
    nb = O.neighbour_table()
    want, t_prev = {}, 0
    w = u0
    for t in CHECKPOINTS:
        w = O.diffuse_steps(w, A, t - t_prev, nb)
        want[t], t_prev = w, t
    u = F.fill_uniform(2201)
    mean = float(F.mass_f64(u)) / F.cells
    errs = {}
    for form in ("f32", "bf16_stochastic", "bf16_nearest"):
        if form == "f32":
            x, kw = u.clone(), {}
        else:
            x = F.bf16_encode(u, mean)
            kw = {"dtype": "bf16", "rounding": form.split("_")[1], "seed": 17}
        y, t_prev = torch.empty_like(x), 0
        for t in CHECKPOINTS:
            x = F.diffuse_run(x, y, t - t_prev, A, first_step=t_prev, **kw)
            y = torch.empty_like(x)
            got = to_np(x).astype(np.float64) if form == "f32" else to_np(F.bf16_decode(x, mean)).astype(np.float64)
            errs[(form, t)] = rel_inf(got, want[t])
            t_prev = t
    for k, v in errs.items():
        record_property(f"{k[0]}_t{k[1]}", v)
    print({f"{k[0]} t={k[1]}": f"{v:.2e}" for k, v in errs.items()})
    for t in CHECKPOINTS:
        assert errs[("f32", t)] < 1e-5, errs
        assert errs[("bf16_stochastic", t)] < 2e-2, errs
    assert errs[("bf16_stochastic", 1000)] < errs[("bf16_nearest", 1000)], errs
