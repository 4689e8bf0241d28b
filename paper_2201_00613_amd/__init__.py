"""Squeeze on MI355X: compact-fractal stencils through the lambda/nu space maps.

Python binding of libsqueeze (include/squeeze.h).  Every call marshals torch
device tensors to the C ABI and launches on torch's current HIP stream; all
arithmetic runs in the library's HIP kernels.  There is no CPU fallback: the
binding raises if the native library is missing or no HIP device is present.
"""
from __future__ import annotations

import contextlib
import ctypes

from ._lib import (BF16, F32, HOLE, IMPL_AUTO, IMPL_BITS, IMPL_CELL, IMPL_CELL_MFMA, IMPL_TILE, IMPL_XTILE,
                   LAYOUT_COMPACT, LAYOUT_EXPANDED, MAP_MFMA, MAP_SCALAR, MASS_WORK_DOUBLES, ROUND_NEAREST_EVEN,
                   ROUND_STOCHASTIC, RUN_AUTO, RUN_LAUNCHES, RUN_RESIDENT, Diffusion, Info, SqueezeError, check,
                   lib)

__all__ = ["Fractal", "SqueezeError", "HOLE", "descriptor_check", "IMPLS"]

IMPLS = {"auto": IMPL_AUTO, "cell": IMPL_CELL, "tile": IMPL_TILE, "xtile": IMPL_XTILE, "cell_mfma": IMPL_CELL_MFMA,
         "bits": IMPL_BITS}
MAP_IMPLS = {"scalar": MAP_SCALAR, "mfma": MAP_MFMA}
RUN_FORMS = {"auto": RUN_AUTO, "launches": RUN_LAUNCHES, "resident": RUN_RESIDENT}
DTYPES = {"f32": F32, "bf16": BF16}
ROUNDINGS = {"nearest": ROUND_NEAREST_EVEN, "stochastic": ROUND_STOCHASTIC}


def _offsets_array(offsets):
    flat = [int(v) for xy in offsets for v in xy]
    return (ctypes.c_int32 * max(1, len(flat)))(*flat), len(flat) // 2


def descriptor_check(s: int, offsets, r: int) -> dict:
    """Validate (s, offsets, r) on the host only; returns the sqz_info fields."""
    arr, k = _offsets_array(offsets)
    info = Info()
    check(lib().sqz_descriptor_check(s, k, arr, r, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in Info._fields_}


_TORCH = None
_SAME_DEVICE = contextlib.nullcontext()


def _torch():
    global _TORCH
    if _TORCH is None:
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("paper_2201_00613_amd needs a HIP device (torch.cuda.is_available() is False)")
        _TORCH = torch
    return _TORCH


def _stream(torch, device):
    """torch's current stream on `device` as a raw handle (torch's own accessor when it
    has one: the public current_stream() builds a Stream object on every call)."""
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(device.index))
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Fractal:
    """An NBB fractal (s, replica offsets, level r) resident on one HIP device.

    Compact state tensors are uint8 (Life) of length ``cells``; the expanded
    bounding-box layout is an (n, n) uint8 tensor indexed [y, x].
    """

    def __init__(self, s: int, offsets, r: int, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        arr, k = _offsets_array(offsets)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().sqz_fractal_create(s, k, arr, r, ctypes.byref(h)))
        self._h = h
        info = Info()
        check(lib().sqz_fractal_info(h, ctypes.byref(info)))
        self.s, self.k, self.r = info.s, info.k, info.r
        self.n, self.cells = info.n, info.cells
        self.compact_shape = (info.compact_h, info.compact_w)
        self.has_tile = bool(info.has_tile)
        self.tile_level = info.tile_level
        self.xtile_level = info.xtile_level
        self.run_steps_per_launch = info.run_steps_per_launch
        self.resident_run = bool(info.resident_run)
        self.bits_level = info.bits_level
        self.offsets = [tuple(map(int, xy)) for xy in offsets]

    def close(self):
        if getattr(self, "_h", None):
            lib().sqz_fractal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _ctx(self):
        """(torch, a context that makes the fractal's device current, its current stream);
        no device switch when the device is current already."""
        torch = _torch()
        dev = _SAME_DEVICE if torch.cuda.current_device() == self.device.index else torch.cuda.device(self.device)
        return torch, dev, _stream(torch, self.device)

    def _need(self, t, dtype, numel, name):
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name}: need a contiguous {dtype} tensor of {numel} elements on {self.device}")

    def empty_state(self, layout: str = "compact"):
        torch = _torch()
        numel = self.cells if layout == "compact" else self.n * self.n
        return torch.empty(numel, dtype=torch.uint8, device=self.device)

    # -- maps -----------------------------------------------------------------
    def lambda_map(self, idx, impl: str = "scalar", out=None):
        """idx: int64 tensor (read as uint64) -> (count, 2) int32 (x, y); (-1,-1) past the end.
        impl: "scalar" (look-up tables) or "mfma" (matrix-core digit sums)."""
        torch, dev, st = self._ctx()
        idx = idx.contiguous()
        self._need(idx, torch.int64, idx.numel(), "idx")
        if out is None:
            out = torch.empty((idx.numel(), 2), dtype=torch.int32, device=self.device)
        self._need(out, torch.int32, 2 * idx.numel(), "out")
        with dev:
            check(lib().sqz_lambda_map_impl(self._h, MAP_IMPLS[impl], _ptr(idx), idx.numel(), _ptr(out), st))
        return out

    def nu_map(self, xy, impl: str = "scalar", out=None):
        """xy: (count, 2) int32 -> int64 tensor of compact indices, -1 (= SQZ_HOLE) for holes.
        impl: "scalar" (look-up tables) or "mfma" (matrix-core digit sums)."""
        torch, dev, st = self._ctx()
        xy = xy.contiguous()
        count = xy.numel() // 2
        self._need(xy, torch.int32, 2 * count, "xy")
        if out is None:
            out = torch.empty(count, dtype=torch.int64, device=self.device)
        self._need(out, torch.int64, count, "out")
        with dev:
            check(lib().sqz_nu_map_impl(self._h, MAP_IMPLS[impl], _ptr(xy), count, _ptr(out), st))
        return out

    # -- starts ---------------------------------------------------------------
    def fill_bernoulli(self, seed: int, p: float, layout: str = "compact", out=None):
        torch, dev, st = self._ctx()
        out = self.empty_state(layout) if out is None else out
        numel = self.cells if layout == "compact" else self.n * self.n
        self._need(out.view(-1), torch.uint8, numel, "out")
        lay = LAYOUT_COMPACT if layout == "compact" else LAYOUT_EXPANDED
        with dev:
            check(lib().sqz_fill_bernoulli(self._h, seed, p, lay, _ptr(out), st))
        return out

    def fill_uniform(self, seed: int, out=None):
        torch, dev, st = self._ctx()
        out = torch.empty(self.cells, dtype=torch.float32, device=self.device) if out is None else out
        self._need(out, torch.float32, self.cells, "out")
        with dev:
            check(lib().sqz_fill_uniform(self._h, seed, _ptr(out), st))
        return out

    # -- Life -----------------------------------------------------------------
    def compact_step(self, src, dst, impl: str = "auto"):
        torch, dev, st = self._ctx()
        self._need(src, torch.uint8, self.cells, "src")
        self._need(dst, torch.uint8, self.cells, "dst")
        with dev:
            check(lib().sqz_compact_step_impl(self._h, IMPLS[impl], _ptr(src), _ptr(dst), st))
        return dst

    def compact_run(self, a, b, steps: int, form: str = "auto"):
        """steps Life steps ping-ponging a -> b -> a ...; returns the tensor holding the result.
        form: "auto", "launches" (one launch per group of steps) or "resident" (one launch,
        tiles held on chip for the whole run)."""
        torch, dev, st = self._ctx()
        self._need(a, torch.uint8, self.cells, "a")
        self._need(b, torch.uint8, self.cells, "b")
        with dev:
            check(lib().sqz_compact_run_form(self._h, RUN_FORMS[form], _ptr(a), _ptr(b), steps, st))
        return a if steps % 2 == 0 else b

    def auto_run_form(self, steps: int) -> str:
        """The run form compact_run(form="auto") takes for `steps` steps (sqz_run_form_auto):
        "resident" or "launches"."""
        form = ctypes.c_int(0)
        check(lib().sqz_run_form_auto(self._h, steps, ctypes.byref(form)))
        return {v: k for k, v in RUN_FORMS.items()}[form.value]

    def expanded_step(self, src, dst):
        torch, dev, st = self._ctx()
        self._need(src.view(-1), torch.uint8, self.n * self.n, "src")
        self._need(dst.view(-1), torch.uint8, self.n * self.n, "dst")
        with dev:
            check(lib().sqz_expanded_step(self._h, _ptr(src), _ptr(dst), st))
        return dst

    # -- block-level layouts ---------------------------------------------------
    def lambda_omega_step(self, src, dst, block_level: int):
        """Life on the expanded n x n array with workgroups over the compact grid of
        level-`block_level` blocks; cells outside member blocks of dst must be 0."""
        torch, dev, st = self._ctx()
        self._need(src.view(-1), torch.uint8, self.n * self.n, "src")
        self._need(dst.view(-1), torch.uint8, self.n * self.n, "dst")
        with dev:
            check(lib().sqz_lambda_omega_step(self._h, block_level, _ptr(src), _ptr(dst), st))
        return dst

    def microblock_bytes(self, block_level: int) -> int:
        v = ctypes.c_uint64()
        check(lib().sqz_microblock_bytes(self._h, block_level, ctypes.byref(v)))
        return v.value

    def microblock_pack(self, compact, block_level: int, out=None):
        torch, dev, st = self._ctx()
        self._need(compact, torch.uint8, self.cells, "compact")
        nbytes = self.microblock_bytes(block_level)
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._need(out, torch.uint8, nbytes, "out")
        with dev:
            check(lib().sqz_microblock_pack(self._h, block_level, _ptr(compact), _ptr(out), st))
        return out

    def microblock_unpack(self, blocks, block_level: int, out=None):
        torch, dev, st = self._ctx()
        self._need(blocks, torch.uint8, self.microblock_bytes(block_level), "blocks")
        if out is None:
            out = torch.empty(self.cells, dtype=torch.uint8, device=self.device)
        self._need(out, torch.uint8, self.cells, "out")
        with dev:
            check(lib().sqz_microblock_unpack(self._h, block_level, _ptr(blocks), _ptr(out), st))
        return out

    def microblock_step(self, src, dst, block_level: int):
        torch, dev, st = self._ctx()
        nbytes = self.microblock_bytes(block_level)
        self._need(src, torch.uint8, nbytes, "src")
        self._need(dst, torch.uint8, nbytes, "dst")
        with dev:
            check(lib().sqz_microblock_step(self._h, block_level, _ptr(src), _ptr(dst), st))
        return dst

    # -- diffusion ------------------------------------------------------------
    def _diffusion(self, dtype, coef, rounding, impl, seed, steps_per_launch=0):
        return Diffusion(DTYPES[dtype], ROUNDINGS[rounding], coef, IMPLS[impl], seed, steps_per_launch, 0)

    def _field_dtype(self, dtype):
        torch = _torch()
        return torch.float32 if dtype == "f32" else torch.uint16

    def diffuse_step(self, src, dst, coef: float, dtype: str = "f32", step: int = 0, rounding: str = "nearest",
                     impl: str = "auto", seed: int = 0):
        torch, dev, st = self._ctx()
        td = self._field_dtype(dtype)
        self._need(src, td, self.cells, "src")
        self._need(dst, td, self.cells, "dst")
        d = self._diffusion(dtype, coef, rounding, impl, seed)
        with dev:
            check(lib().sqz_diffuse_step(self._h, ctypes.byref(d), step, _ptr(src), _ptr(dst), st))
        return dst

    def diffuse_run(self, a, b, steps: int, coef: float, dtype: str = "f32", first_step: int = 0,
                    rounding: str = "nearest", impl: str = "auto", seed: int = 0, steps_per_launch: int = 0):
        """steps diffusion steps ping-ponging a -> b -> ...; returns the tensor holding the result.
        steps_per_launch 2..3 selects multi-step expanded tiles (same results)."""
        torch, dev, st = self._ctx()
        td = self._field_dtype(dtype)
        self._need(a, td, self.cells, "a")
        self._need(b, td, self.cells, "b")
        d = self._diffusion(dtype, coef, rounding, impl, seed, steps_per_launch)
        with dev:
            check(lib().sqz_diffuse_run(self._h, ctypes.byref(d), first_step, steps, _ptr(a), _ptr(b), st))
        return a if steps % 2 == 0 else b

    def mass_f64(self, u, dtype: str = "f32", offset: float = 0.0, work=None):
        """Binary64 sum of offset + u on the device; returns a 0-d float64 device tensor
        (element 0 of `work`, a float64 tensor of MASS_WORK_DOUBLES elements, allocated here
        if not given)."""
        torch, dev, st = self._ctx()
        self._need(u, self._field_dtype(dtype), self.cells, "u")
        work = torch.empty(MASS_WORK_DOUBLES, dtype=torch.float64, device=self.device) if work is None else work
        self._need(work, torch.float64, MASS_WORK_DOUBLES, "work")
        with dev:
            check(lib().sqz_mass_f64(self._h, DTYPES[dtype], _ptr(u), offset, _ptr(work), st))
        return work[0]

    def mass_f64_noalloc(self, u, out, dtype: str = "f32", offset: float = 0.0):
        """mass_f64 with the partial sums in the library's static scratch (sqz_mass_f64_noalloc);
        `out`: a one-element float64 device tensor, receives the sum."""
        torch, dev, st = self._ctx()
        self._need(u, self._field_dtype(dtype), self.cells, "u")
        self._need(out, torch.float64, 1, "out")
        with dev:
            check(lib().sqz_mass_f64_noalloc(self._h, DTYPES[dtype], _ptr(u), offset, _ptr(out), st))
        return out[0]

    def bf16_encode(self, u, offset: float, out=None):
        torch, dev, st = self._ctx()
        self._need(u, torch.float32, self.cells, "u")
        out = torch.empty(self.cells, dtype=torch.uint16, device=self.device) if out is None else out
        self._need(out, torch.uint16, self.cells, "out")
        with dev:
            check(lib().sqz_bf16_encode(self._h, _ptr(u), offset, _ptr(out), st))
        return out

    def bf16_decode(self, b, offset: float, out=None):
        torch, dev, st = self._ctx()
        self._need(b, torch.uint16, self.cells, "b")
        out = torch.empty(self.cells, dtype=torch.float32, device=self.device) if out is None else out
        self._need(out, torch.float32, self.cells, "out")
        with dev:
            check(lib().sqz_bf16_decode(self._h, _ptr(b), offset, _ptr(out), st))
        return out


class Batch:
    """Many fractals advanced together: one persistent launch per step (sqz_batch_*).

    The state is one uint8 tensor of ``total_bytes``; instance i's cells are the
    slice ``[offsets[i], offsets[i] + fractals[i].cells)`` (see ``instance``).
    """

    def __init__(self, fractals):
        torch = _torch()
        self.fractals = list(fractals)
        n = len(self.fractals)
        arr = (ctypes.c_void_p * n)(*[f._h.value for f in self.fractals])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.fractals[0].device):
            check(lib().sqz_batch_create(n, arr, ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_uint64 * (n + 1))()
        total = ctypes.c_uint64()
        check(lib().sqz_batch_layout(h, offs, ctypes.byref(total)))
        self.offsets = [int(v) for v in offs]
        self.total_bytes = self.offsets[-1]
        self.total_cells = int(total.value)
        self.device = self.fractals[0].device
        k = ctypes.c_int32()
        check(lib().sqz_batch_steps_per_launch(h, ctypes.byref(k)))
        self.steps_per_launch = int(k.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().sqz_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ctx(self):
        """(torch, a context that makes the batch's device current, its current stream);
        no device switch when the device is current already."""
        torch = _torch()
        dev = _SAME_DEVICE if torch.cuda.current_device() == self.device.index else torch.cuda.device(self.device)
        return torch, dev, _stream(torch, self.device)

    def _need(self, t, name):
        torch = _torch()
        if t.device != self.device or t.dtype != torch.uint8 or not t.is_contiguous() or t.numel() != self.total_bytes:
            raise ValueError(f"{name}: need a contiguous uint8 tensor of {self.total_bytes} bytes on {self.device}")

    def empty_state(self):
        torch = _torch()
        return torch.zeros(self.total_bytes, dtype=torch.uint8, device=self.device)

    def instance(self, state, i: int):
        return state[self.offsets[i]:self.offsets[i] + self.fractals[i].cells]

    def fill_bernoulli(self, seeds, p: float, out=None):
        torch, dev, st = self._ctx()
        out = self.empty_state() if out is None else out
        self._need(out, "out")
        arr = (ctypes.c_uint64 * len(self.fractals))(*[int(s) for s in seeds])
        with dev:
            check(lib().sqz_batch_fill_bernoulli(self._h, arr, p, _ptr(out), st))
        return out

    def step(self, src, dst):
        torch, dev, st = self._ctx()
        self._need(src, "src")
        self._need(dst, "dst")
        with dev:
            check(lib().sqz_batch_step(self._h, _ptr(src), _ptr(dst), st))
        return dst

    def run(self, a, b, steps: int):
        """steps steps ping-ponging a -> b -> ... (hipGraph replay for steps >= 2)."""
        torch, dev, st = self._ctx()
        self._need(a, "a")
        self._need(b, "b")
        with dev:
            check(lib().sqz_batch_run(self._h, _ptr(a), _ptr(b), steps, st))
        return a if steps % 2 == 0 else b

    def autotune(self, a, b) -> int:
        torch, dev, st = self._ctx()
        self._need(a, "a")
        self._need(b, "b")
        w = ctypes.c_int32()
        with dev:
            check(lib().sqz_batch_autotune(self._h, _ptr(a), _ptr(b), st, ctypes.byref(w)))
        self._refresh_steps()
        return int(w.value)

    TILED_FORMS = {"groups": 0, "persistent": 1, "per_tile": 2}

    def set_tiled_launch(self, form, steps_per_launch: int = 0, wg_per_cu: int = 0):
        """Launch form of the instances with a tiled kernel (sqz_batch_set_tiled_launch):
        "groups" (or False, 0) one launch per pattern group; "persistent" (or True, 1) one
        persistent launch over all of them; "per_tile" (2) one launch over all of them with a
        workgroup per tile."""
        code = self.TILED_FORMS[form] if isinstance(form, str) else int(form)
        check(lib().sqz_batch_set_tiled_launch(self._h, code, steps_per_launch, wg_per_cu))
        self._refresh_steps()

    @property
    def tiled_launch(self) -> dict:
        """The launch form in use for the tiled instances (sqz_batch_tiled_launch):
        {"form": "groups" | "persistent" | "per_tile" | None, "steps_per_launch", "wg_per_cu"}."""
        f, k, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().sqz_batch_tiled_launch(self._h, ctypes.byref(f), ctypes.byref(k), ctypes.byref(w)))
        names = {v: n for n, v in self.TILED_FORMS.items()}
        return {"form": names.get(f.value), "steps_per_launch": k.value, "wg_per_cu": w.value}

    def _refresh_steps(self):
        k = ctypes.c_int32()
        check(lib().sqz_batch_steps_per_launch(self._h, ctypes.byref(k)))
        self.steps_per_launch = int(k.value)
