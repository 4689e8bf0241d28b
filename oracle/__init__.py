"""CPU oracle for the Squeeze compact-fractal stencil.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2201_00613_amd``); its arithmetic lives in
``squeeze_oracle.c`` (plain C, 64-bit integers / binary64), written from the
paper's definitions: replication of the NBB transition function, the lambda
and nu maps level by level, and the Life / diffusion rules on the expanded
grid or through the maps.

Every function here is a thin numpy <-> ctypes marshaller.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "squeeze_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A test run may point the loader at another build of the same source (the
# sanitizer build of tests/test_host_sanitizers.py).
_LIB_OVERRIDE = os.environ.get("SQZ_ORACLE_LIB")

HOLE = -1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            path = _LIB_OVERRIDE
        else:
            path = build() if not os.path.exists(_LIB_PATH) else _LIB_PATH
        L = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        f64p = ctypes.POINTER(ctypes.c_double)
        c_int, c_i64, c_u64, c_u32, c_dbl = (
            ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double)
        sig = {
            "orc_num_threads": (c_int, []),
            "orc_build_order": (None, [c_int, c_int, i32p, c_int, i32p]),
            "orc_lambda_batch": (None, [c_int, c_int, i32p, c_int, u64p, c_i64, i64p]),
            "orc_nu_batch": (None, [c_int, c_int, i32p, c_int, i64p, c_i64, i64p]),
            "orc_nu": (c_i64, [c_int, c_int, i32p, c_int, c_i64, c_i64]),
            "orc_dense_inverse": (None, [c_int, c_int, c_int, i32p, i64p]),
            "orc_splitmix64": (c_u64, [c_u64, c_u64]),
            "orc_fill_compact": (None, [c_int, c_int, i32p, c_int, c_u64, c_u32, c_u64, c_u64, u8p]),
            "orc_fill_expanded": (None, [c_int, c_int, i32p, c_int, c_u64, c_u32, u8p]),
            "orc_fill_uniform_compact": (None, [c_int, c_int, i32p, c_int, c_u64, c_u64, c_u64, f64p]),
            "orc_life_expanded": (c_i64, [c_i64, u8p, u8p, u8p]),
            "orc_life_compact": (c_i64, [c_int, c_int, i32p, c_int, u8p, c_u64, c_u64, u8p]),
            "orc_light_cone": (None, [c_int, c_int, i32p, c_int, c_u64, c_u32, i64p, c_i64, c_int, u8p]),
            "orc_diffuse_compact": (None, [c_int, c_int, i32p, c_int, c_dbl, f64p, c_u64, c_u64, f64p]),
            "orc_diffuse_cone": (None, [c_int, c_int, i32p, c_int, c_u64, c_dbl, i64p, c_i64, c_int, f64p]),
            "orc_neighbour_table": (None, [c_int, c_int, i32p, c_int, c_u64, c_u64, i64p]),
            "orc_diffuse_table": (None, [c_i64, i64p, c_dbl, c_int, f64p, f64p]),
            "orc_life_table": (None, [c_i64, i64p, c_int, u8p, u8p]),
            "orc_life_windows": (None, [c_int, c_int, i32p, c_int, c_u64, c_u32, i64p, c_i64, c_int, c_int, c_int,
                                        u8p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Fractal:
    """(s, replica offsets, level r): the descriptor of an NBB fractal."""

    def __init__(self, s: int, offsets, r: int):
        self.s = int(s)
        self.offsets = [(int(x), int(y)) for x, y in offsets]
        self.k = len(self.offsets)
        self.r = int(r)
        self.n = self.s ** self.r
        self.N = self.k ** self.r
        self._offs = np.ascontiguousarray(np.array(self.offsets, dtype=np.int32).reshape(-1))

    def _a(self):
        return (self.s, self.k, _ptr(self._offs, ctypes.c_int32), self.r)

    # -- construction and maps ------------------------------------------
    def order(self) -> np.ndarray:
        """(N, 2) int32 expanded coordinates of compact cells 0..N-1 (replication)."""
        xy = np.empty((self.N, 2), dtype=np.int32)
        lib().orc_build_order(*self._a(), _ptr(xy, ctypes.c_int32))
        return xy

    def lam(self, c) -> np.ndarray:
        """(len, 2) int64 expanded coordinates of compact indices c (level-digit formula)."""
        c = np.ascontiguousarray(np.asarray(c, dtype=np.uint64).reshape(-1))
        xy = np.empty((c.size, 2), dtype=np.int64)
        lib().orc_lambda_batch(*self._a(), _ptr(c, ctypes.c_uint64), c.size, _ptr(xy, ctypes.c_int64))
        return xy

    def nu(self, xy) -> np.ndarray:
        """int64 compact index of each (x, y), or HOLE (-1); top-down level scan."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int64).reshape(-1, 2))
        c = np.empty(xy.shape[0], dtype=np.int64)
        lib().orc_nu_batch(*self._a(), _ptr(xy, ctypes.c_int64), xy.shape[0], _ptr(c, ctypes.c_int64))
        return c

    def dense_inverse(self) -> np.ndarray:
        """(n, n) int64 array [y, x] -> compact index or HOLE, from the replication order."""
        xy = self.order()
        d = np.empty((self.n, self.n), dtype=np.int64)
        lib().orc_dense_inverse(self.s, self.k, self.r, _ptr(xy, ctypes.c_int32), _ptr(d, ctypes.c_int64))
        return d

    def member(self) -> np.ndarray:
        """(n, n) uint8 membership mask [y, x]."""
        return (self.dense_inverse() >= 0).astype(np.uint8)

    # -- inputs -----------------------------------------------------------
    def fill_compact(self, seed: int, p: float, c0: int = 0, c1: int | None = None) -> np.ndarray:
        c1 = self.N if c1 is None else c1
        out = np.empty(c1 - c0, dtype=np.uint8)
        lib().orc_fill_compact(*self._a(), seed, threshold24(p), c0, c1, _ptr(out, ctypes.c_uint8))
        return out

    def fill_expanded(self, seed: int, p: float) -> np.ndarray:
        out = np.empty((self.n, self.n), dtype=np.uint8)
        lib().orc_fill_expanded(*self._a(), seed, threshold24(p), _ptr(out, ctypes.c_uint8))
        return out

    def fill_uniform_compact(self, seed: int, c0: int = 0, c1: int | None = None) -> np.ndarray:
        c1 = self.N if c1 is None else c1
        out = np.empty(c1 - c0, dtype=np.float64)
        lib().orc_fill_uniform_compact(*self._a(), seed, c0, c1, _ptr(out, ctypes.c_double))
        return out

    # -- Life -------------------------------------------------------------
    def life_compact(self, state: np.ndarray, c0: int = 0, c1: int | None = None) -> np.ndarray:
        """One B3/S23 step through lambda/nu; returns cells [c0, c1)."""
        state = np.ascontiguousarray(state, dtype=np.uint8)
        assert state.size == self.N
        c1 = self.N if c1 is None else c1
        out = np.empty(c1 - c0, dtype=np.uint8)
        bad = lib().orc_life_compact(*self._a(), _ptr(state, ctypes.c_uint8), c0, c1,
                                     _ptr(out, ctypes.c_uint8))
        if bad:
            raise ValueError(f"{bad} states outside {{0,1}}")
        return out

    def light_cone(self, seed: int, p: float, xy, t: int) -> np.ndarray:
        """States of cells xy after t steps from fill(seed, p), one window per cell."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int64).reshape(-1, 2))
        out = np.empty(xy.shape[0], dtype=np.uint8)
        lib().orc_light_cone(*self._a(), seed, threshold24(p), _ptr(xy, ctypes.c_int64),
                             xy.shape[0], t, _ptr(out, ctypes.c_uint8))
        return out

    def life_windows(self, seed: int, p: float, corners, w: int, h: int, t: int) -> np.ndarray:
        """(count, h, w) states after t steps from fill(seed, p) of the w x h rectangles with
        the given (x0, y0) corners, indexed [q, y - y0, x - x0]; 0 on holes and outside the box."""
        corners = np.ascontiguousarray(np.asarray(corners, dtype=np.int64).reshape(-1, 2))
        out = np.empty((corners.shape[0], h, w), dtype=np.uint8)
        lib().orc_life_windows(*self._a(), seed, threshold24(p), _ptr(corners, ctypes.c_int64), corners.shape[0],
                               w, h, t, _ptr(out, ctypes.c_uint8))
        return out

    def neighbour_table(self, c0: int = 0, c1: int | None = None) -> np.ndarray:
        c1 = self.N if c1 is None else c1
        nb = np.empty((c1 - c0, 8), dtype=np.int64)
        lib().orc_neighbour_table(*self._a(), c0, c1, _ptr(nb, ctypes.c_int64))
        return nb

    def life_steps(self, state: np.ndarray, steps: int, nb: np.ndarray | None = None) -> np.ndarray:
        """`steps` B3/S23 steps via a neighbour table (built here if not given)."""
        nb = self.neighbour_table() if nb is None else nb
        u = np.array(state, dtype=np.uint8, copy=True)
        if np.any(u > 1):
            raise ValueError("states outside {0,1}")
        tmp = np.empty_like(u)
        lib().orc_life_table(self.N, _ptr(nb, ctypes.c_int64), steps, _ptr(u, ctypes.c_uint8),
                             _ptr(tmp, ctypes.c_uint8))
        return u

    # -- diffusion --------------------------------------------------------
    def diffuse_compact(self, u: np.ndarray, a: float, c0: int = 0, c1: int | None = None) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        c1 = self.N if c1 is None else c1
        out = np.empty(c1 - c0, dtype=np.float64)
        lib().orc_diffuse_compact(*self._a(), a, _ptr(u, ctypes.c_double), c0, c1,
                                  _ptr(out, ctypes.c_double))
        return out

    def diffuse_cone(self, seed: int, a: float, xy, t: int) -> np.ndarray:
        """Values of cells xy after t diffusion steps from fill_uniform(seed), one window per cell."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.int64).reshape(-1, 2))
        out = np.empty(xy.shape[0], dtype=np.float64)
        lib().orc_diffuse_cone(*self._a(), seed, a, _ptr(xy, ctypes.c_int64), xy.shape[0], t,
                               _ptr(out, ctypes.c_double))
        return out

    def diffuse_steps(self, u: np.ndarray, a: float, steps: int, nb: np.ndarray | None = None) -> np.ndarray:
        nb = self.neighbour_table() if nb is None else nb
        u = np.array(u, dtype=np.float64, copy=True)
        tmp = np.empty_like(u)
        lib().orc_diffuse_table(self.N, _ptr(nb, ctypes.c_int64), a, steps,
                                _ptr(u, ctypes.c_double), _ptr(tmp, ctypes.c_double))
        return u


def life_expanded(member: np.ndarray, state: np.ndarray) -> np.ndarray:
    """One masked B3/S23 step on an expanded (n, n) grid."""
    member = np.ascontiguousarray(member, dtype=np.uint8)
    state = np.ascontiguousarray(state, dtype=np.uint8)
    n = member.shape[0]
    out = np.empty_like(state)
    bad = lib().orc_life_expanded(n, _ptr(member, ctypes.c_uint8), _ptr(state, ctypes.c_uint8),
                                  _ptr(out, ctypes.c_uint8))
    if bad:
        raise ValueError(f"{bad} states outside {{0,1}}")
    return out


def splitmix64(seed: int, i: int) -> int:
    """Output number i+1 of SplitMix64 seeded with `seed`."""
    return int(lib().orc_splitmix64(seed, i))


def threshold24(p: float) -> int:
    """floor(p * 2^24): a cell is alive iff the top 24 bits of its hash are below this."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("p must lie in [0, 1]")
    return int(np.floor(p * 16777216.0))


def num_threads() -> int:
    return int(lib().orc_num_threads())
