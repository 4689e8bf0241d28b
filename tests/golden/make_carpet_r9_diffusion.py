"""Writes carpet_r9_diffusion.npz: binary64 reference values of the diffusion
workload on the level-9 Sierpinski carpet, computed by the CPU oracle only.

Workload: the explicit update u' = u + a * sum over member Moore neighbours of
(u_q - u_p) (the PDE application named in the paper's Introduction, in the
form fixed for this project), a = 0.1, U(0,1) start from SplitMix64 seed 2201
keyed by the expanded coordinate, carpet replicas in row order, level 9
(134,217,728 cells), 1000 steps.  The oracle advances the whole field in
binary64 through its neighbour table (8.6 GB of int64; about ten minutes on
eight cores).

Stored: the compact indices of 100,002 fixed cells (cells 0 and N-1 and
100,000 drawn uniformly with numpy's PCG64 seeded 9), their values at
t = 0, 1, 10, 100, 1000, and at each t the whole field's infinity norm, sum,
minimum and maximum.

Run from the repository root:  python tests/golden/make_carpet_r9_diffusion.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

CARPET = (3, [(0, 0), (1, 0), (2, 0), (0, 1), (2, 1), (0, 2), (1, 2), (2, 2)])
LEVEL, SEED, COEF = 9, 2201, 0.1
CHECKPOINTS = (0, 1, 10, 100, 1000)
OUT = os.path.join(HERE, "carpet_r9_diffusion.npz")


def main() -> None:
    O = oracle.Fractal(*CARPET, LEVEL)
    rng = np.random.default_rng(9)
    idx = np.concatenate([[0, O.N - 1], rng.integers(0, O.N, 100_000)]).astype(np.int64)
    t0 = time.time()
    u = O.fill_uniform_compact(SEED)
    print(f"start: {time.time() - t0:.1f} s", flush=True)
    nb = O.neighbour_table()
    print(f"neighbour table: {time.time() - t0:.1f} s", flush=True)
    vals, inf, total, lo, hi = [], [], [], [], []
    done = 0
    for t in CHECKPOINTS:
        if t > done:
            u = O.diffuse_steps(u, COEF, t - done, nb)
            done = t
        vals.append(u[idx])
        inf.append(float(np.max(np.abs(u))))
        total.append(float(np.sum(u)))
        lo.append(float(u.min()))
        hi.append(float(u.max()))
        print(f"t={t}: {time.time() - t0:.1f} s, inf-norm {inf[-1]:.17g}, sum {total[-1]:.17g}", flush=True)
    np.savez_compressed(OUT, level=LEVEL, seed=SEED, coef=COEF, steps=np.array(CHECKPOINTS), idx=idx,
                        values=np.stack(vals), inf_norm=np.array(inf), field_sum=np.array(total),
                        field_min=np.array(lo), field_max=np.array(hi))
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
