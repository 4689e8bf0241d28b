"""Seeded workload definitions (inputs only: no part of the method's arithmetic).

Replica patterns of the fractals used by the benchmarks, and the batched
workload's instance list: for instance i of a batch with master seed m, the
pattern is draw(m, 2i) mod 3 over (triangle, carpet, Vicsek) and the level is
uniform over the levels whose cell count lies in [1e4, 1e7] (triangle 9..14,
carpet 5..7, Vicsek 6..10) by draw(m, 2i+1); the instance's own seed is
draw(m, 2i + 1_000_003).  draw(m, i) is output i+1 of SplitMix64 (Steele, Lea
& Flood 2014) seeded with m.
"""
from __future__ import annotations

TRIANGLE = (2, ((0, 0), (1, 0), (0, 1)))
CARPET = (3, ((0, 0), (1, 0), (2, 0), (0, 1), (2, 1), (0, 2), (1, 2), (2, 2)))
VICSEK = (3, ((1, 0), (0, 1), (1, 1), (2, 1), (1, 2)))

PATTERNS = {"triangle": TRIANGLE, "carpet": CARPET, "vicsek": VICSEK}
LEVELS = {"triangle": range(9, 15), "carpet": range(5, 8), "vicsek": range(6, 11)}

_M64 = (1 << 64) - 1


def draw(seed: int, i: int) -> int:
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def batch_instances(count: int = 512, master_seed: int = 2201):
    """[(name, s, offsets, r, seed)] for the batched workload."""
    names = ("triangle", "carpet", "vicsek")
    out = []
    for i in range(count):
        name = names[draw(master_seed, 2 * i) % 3]
        levels = LEVELS[name]
        r = levels[draw(master_seed, 2 * i + 1) % len(levels)]
        s, offs = PATTERNS[name]
        out.append((name, s, offs, r, draw(master_seed, 2 * i + 1_000_003)))
    return out
