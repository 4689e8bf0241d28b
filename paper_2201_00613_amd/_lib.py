"""ctypes loader for libsqueeze.so (in-tree build).  Fails loudly when missing."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsqueeze.so")

# sqz_status codes (include/squeeze.h)
OK, ERR_INVALID, ERR_RANGE, ERR_NOMEM, ERR_HIP, ERR_UNSUPPORTED = range(6)
HOLE = (1 << 64) - 1
LAYOUT_COMPACT, LAYOUT_EXPANDED = 0, 1
IMPL_AUTO, IMPL_CELL, IMPL_TILE, IMPL_XTILE, IMPL_CELL_MFMA, IMPL_BITS = 0, 1, 2, 3, 4, 5
MAP_SCALAR, MAP_MFMA = 0, 1
RUN_AUTO, RUN_LAUNCHES, RUN_RESIDENT = 0, 1, 2
F32, BF16 = 0, 1
ROUND_NEAREST_EVEN, ROUND_STOCHASTIC = 0, 1
MASS_WORK_DOUBLES = 1025


class SqueezeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class Info(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_int32), ("k", ctypes.c_int32), ("r", ctypes.c_int32),
        ("tile_level", ctypes.c_int32), ("n", ctypes.c_int64), ("cells", ctypes.c_uint64),
        ("compact_w", ctypes.c_uint64), ("compact_h", ctypes.c_uint64),
        ("has_tile", ctypes.c_int32), ("xtile_level", ctypes.c_int32),
        ("run_steps_per_launch", ctypes.c_int32), ("bits_level", ctypes.c_int32),
        ("resident_run", ctypes.c_int32),
    ]


class Diffusion(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("rounding", ctypes.c_int), ("coef", ctypes.c_float),
                ("impl", ctypes.c_int), ("seed", ctypes.c_uint64), ("steps_per_launch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes); must match include/squeeze.h
SIGNATURES = {
    "sqz_descriptor_check": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(Info)]),
    "sqz_fractal_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "sqz_fractal_destroy": (None, [ctypes.c_void_p]),
    "sqz_fractal_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "sqz_lambda_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "sqz_nu_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "sqz_lambda_omega_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sqz_microblock_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "sqz_microblock_pack": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "sqz_microblock_unpack": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sqz_microblock_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "sqz_batch_steps_per_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "sqz_batch_set_tiled_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "sqz_batch_tiled_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
    "sqz_lambda_map_impl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_nu_map_impl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_fill_bernoulli": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_fill_uniform": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_compact_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_compact_step_impl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "sqz_compact_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p]),
    "sqz_compact_run_form": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_void_p]),
    "sqz_run_form_auto": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int)]),
    "sqz_expanded_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_diffuse_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diffusion), ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_diffuse_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Diffusion), ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_mass_f64": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "sqz_mass_f64_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_double,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_bf16_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "sqz_bf16_decode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "sqz_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sqz_last_error": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """Load libsqueeze.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != OK:
        msg = lib().sqz_last_error().decode(errors="replace")
        raise SqueezeError(status, msg)


SIGNATURES.update({
    "sqz_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sqz_batch_destroy": (None, [ctypes.c_void_p]),
    "sqz_batch_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "sqz_batch_fill_bernoulli": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "sqz_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sqz_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p]),
    "sqz_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int32)]),
})
