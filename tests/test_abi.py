"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and validates descriptors without touching a device."""
import ctypes
import os
import re

import pytest

import fractals as FR

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "squeeze.h")


@pytest.fixture(scope="module")
def sqz():
    import paper_2201_00613_amd as m

    m._lib.lib()
    return m


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SQZ_API\s+[\w\s\*]*?\b(sqz_\w+)\s*\(", text)))


def test_header_declares_the_interface():
    names = declared_symbols()
    for want in ("sqz_fractal_create", "sqz_fractal_destroy", "sqz_lambda_map", "sqz_nu_map",
                 "sqz_compact_step", "sqz_compact_run", "sqz_expanded_step", "sqz_fill_bernoulli",
                 "sqz_last_error", "sqz_status_string", "sqz_descriptor_check"):
        assert want in names


def test_library_exports_every_declared_symbol(sqz):
    L = ctypes.CDLL(sqz._lib.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(declared_symbols()) == set(sqz._lib.SIGNATURES), "binding and header disagree"


def test_status_strings(sqz):
    L = sqz._lib.lib()
    assert L.sqz_status_string(0) == b"ok"
    assert L.sqz_status_string(2) == b"size out of range"
    assert L.sqz_status_string(99) == b"unknown status"


@pytest.mark.parametrize("name", sorted(FR.ALL))
def test_valid_descriptors(sqz, name):
    s, offs = FR.ALL[name]
    for r in (0, 1, 5):
        info = sqz.descriptor_check(s, offs, r)
        assert info["cells"] == len(offs) ** r and info["n"] == s ** r
        assert info["compact_w"] * info["compact_h"] == info["cells"]
        assert info["compact_w"] == len(offs) ** ((r + 1) // 2)


def test_level_limits(sqz):
    s, offs = FR.TRIANGLE
    assert sqz.descriptor_check(s, offs, 30)["n"] == 2 ** 30
    with pytest.raises(sqz.SqueezeError) as e:
        sqz.descriptor_check(s, offs, 31)  # n = 2^31 does not fit
    assert e.value.status == 2
    s, offs = FR.CARPET
    assert sqz.descriptor_check(s, offs, 19)["cells"] == 8 ** 19
    with pytest.raises(sqz.SqueezeError) as e:
        sqz.descriptor_check(s, offs, 21)  # 8^21 = 2^63
    assert e.value.status == 2


@pytest.mark.parametrize("s,offs,r,why", [
    (1, [(0, 0)], 2, "s < 2"),
    (17, [(0, 0)], 2, "s > 16"),
    (2, [], 2, "k = 0"),
    (2, [(0, 0), (1, 0), (0, 1), (1, 1), (0, 0)], 2, "k > s*s"),
    (2, [(0, 0), (0, 0)], 2, "duplicate offset"),
    (2, [(0, 0), (2, 0)], 2, "offset outside [0,s)"),
    (3, [(0, -1)], 2, "negative offset"),
    (2, [(0, 0), (1, 0)], -1, "negative level"),
])
def test_invalid_descriptors(sqz, s, offs, r, why):
    with pytest.raises(sqz.SqueezeError) as e:
        sqz.descriptor_check(s, offs, r)
    assert e.value.status == 1, why
    assert sqz._lib.lib().sqz_last_error()


def test_null_arguments_rejected_without_device(sqz):
    L = sqz._lib.lib()
    assert L.sqz_descriptor_check(2, 3, None, 4, None) == 1
    assert L.sqz_fractal_create(2, 3, None, 4, None) == 1
    assert L.sqz_fractal_info(None, None) == 1
    L.sqz_fractal_destroy(None)  # allowed


def test_binding_refuses_cpu_only(sqz):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    with pytest.raises(RuntimeError):
        sqz.Fractal(2, FR.TRIANGLE[1], 3)
