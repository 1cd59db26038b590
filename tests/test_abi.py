"""The C ABI library loads on the host, exports every symbol include/bessel.h
declares, and rejects bad arguments before any GPU work (these calls return
from host-side checks, so they run without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2108_11560_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(bessel_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libbessel.so is not built (python -m paper_2108_11560_amd.build)")
    return _lib.load()


def test_header_declares_the_paths():
    names = declared_functions()
    for required in ["bessel_logk", "bessel_logk_dv_dx", "bessel_range", "bessel_logk_backward",
                     "bessel_logk_hess", "bessel_hess_vjp", "bessel_last_error"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding knows every declared function
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_version_string(lib):
    assert b"gfx950" in lib.bessel_version()


FAKE_A = ctypes.c_void_p(0x10000)
FAKE_B = ctypes.c_void_p(0x20000)
FAKE_C = ctypes.c_void_p(0x30000)
NULL = ctypes.c_void_p(0)


def err(lib):
    return lib.bessel_last_error().decode()


def test_bad_dtype(lib):
    assert lib.bessel_logk(7, 4, FAKE_A, FAKE_B, FAKE_C, 128, 0, NULL, NULL) == -2
    assert "dtype" in err(lib)


def test_negative_n(lib):
    assert lib.bessel_logk(1, -1, FAKE_A, FAKE_B, FAKE_C, 128, 0, NULL, NULL) == -1


def test_null_inputs(lib):
    assert lib.bessel_logk(1, 4, NULL, FAKE_B, FAKE_C, 128, 0, NULL, NULL) == -1
    assert lib.bessel_logk(1, 4, FAKE_A, FAKE_B, NULL, 128, 0, NULL, NULL) == -1
    assert lib.bessel_logk_dv_dx(1, 4, FAKE_A, FAKE_B, NULL, NULL, NULL, FAKE_C, 128, 0, NULL, NULL) == -1
    assert lib.bessel_range(1, 4, FAKE_A, FAKE_B, NULL, FAKE_C, NULL, NULL, 0, NULL, NULL, NULL) == -1


@pytest.mark.parametrize("nbins", [-5, 0, 1, 4097, 1 << 20])
def test_nbins_range(lib, nbins):
    assert lib.bessel_logk(1, 4, FAKE_A, FAKE_B, FAKE_C, nbins, 0, NULL, NULL) == -3


def test_range_mode(lib):
    assert lib.bessel_logk(1, 4, FAKE_A, FAKE_B, FAKE_C, 128, 9, NULL, NULL) == -4
    # the learned range (per element or tabulated) needs a predictor handle
    assert lib.bessel_logk(0, 4, FAKE_A, FAKE_B, FAKE_C, 128, 1, NULL, NULL) == -4
    assert lib.bessel_logk(0, 4, FAKE_A, FAKE_B, FAKE_C, 128, 2, NULL, NULL) == -4
    # ... and is provided for F32 only
    assert lib.bessel_logk(1, 4, FAKE_A, FAKE_B, FAKE_C, 128, 2, FAKE_A, NULL) == -7
    assert lib.bessel_range(1, 4, FAKE_A, FAKE_B, FAKE_C, NULL, NULL, NULL, 2, FAKE_A, NULL, NULL) == -7


def test_zero_length_is_noop(lib):
    assert lib.bessel_logk(1, 0, NULL, NULL, NULL, 128, 0, NULL, NULL) == 0
    assert lib.bessel_logk_dv_dx(0, 0, NULL, NULL, NULL, NULL, NULL, NULL, 64, 0, NULL, NULL) == 0
    assert lib.bessel_range(0, 0, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL, NULL) == 0
    assert lib.bessel_logk_backward(1, 0, NULL, NULL, NULL, NULL, NULL, NULL) == 0


def test_alias_detection(lib):
    # 4 doubles = 32 bytes; FAKE_A+16 overlaps FAKE_A's range
    inside = ctypes.c_void_p(0x10000 + 16)
    assert lib.bessel_logk(1, 4, FAKE_A, FAKE_B, inside, 128, 0, NULL, NULL) == -6
    assert lib.bessel_logk_dv_dx(1, 4, FAKE_A, FAKE_B, NULL, NULL, FAKE_C, FAKE_C, 128, 0, NULL, NULL) == -6
    assert lib.bessel_range(1, 4, FAKE_A, FAKE_B, FAKE_C, FAKE_C, NULL, NULL, 0, NULL, NULL, NULL) == -6
    assert lib.bessel_logk_backward(1, 4, FAKE_A, FAKE_B, FAKE_C, FAKE_A, NULL, NULL) == -6
    assert "overlap" in err(lib)


def test_error_status_names():
    assert _lib.STATUS[-3] == "BESSEL_ERR_NBINS"
    with pytest.raises(_lib.BesselError):
        _lib.check(-3, "x")


def test_gh_argument_errors(lib):
    args = [FAKE_A, FAKE_A, FAKE_A, FAKE_A, 4, FAKE_B, NULL, FAKE_C, NULL, NULL, NULL, NULL]
    assert lib.bessel_gh_logk_sum(4, *args, 128, 1, NULL, NULL) == -7  # per-element network: not here
    assert lib.bessel_gh_logk_sum(4, *args, 128, 2, NULL, NULL) == -4  # the table needs a predictor
    assert lib.bessel_gh_logk_sum(4, *args, 128, 3, NULL, NULL) == -4
    assert lib.bessel_gh_logk_sum(4, *args, 1, 0, NULL, NULL) == -3
    assert lib.bessel_gh_logk_sum(-1, *args, 128, 0, NULL, NULL) == -1
    assert lib.bessel_gh_logk_sum(0, *args, 128, 0, NULL, NULL) == 0
    bad = [FAKE_A, FAKE_A, FAKE_A, FAKE_A, 4, FAKE_B, NULL, FAKE_A, NULL, NULL, NULL, NULL]
    assert lib.bessel_gh_logk_sum(4, *bad, 128, 0, NULL, NULL) == -6
    # the allocation-free variant runs the same checks first
    for fn in (lib.bessel_gh_logk_sum, lib.bessel_gh_logk_sum_noalloc):
        assert fn(4, *args, 128, 1, NULL, NULL) == -7
        assert fn(4, *args, 128, 2, NULL, NULL) == -4
        assert fn(4, *args, 1, 0, NULL, NULL) == -3
        assert fn(4, *bad, 128, 0, NULL, NULL) == -6
        assert fn(0, *args, 128, 0, NULL, NULL) == 0


def test_gh_noalloc_rejects_beyond_its_static_partials(lib):
    # 1025 sets x 256 chunks of 256 samples: one set more than the static array
    # holds; the host check returns before any GPU call
    sets = [ctypes.c_void_p(0x1000000 * (k + 1)) for k in range(4)]
    y, out = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x20000000)
    rc = lib.bessel_gh_logk_sum_noalloc(1025, *sets, 65536, y, NULL, out, NULL, NULL, NULL, NULL, 128, 0, NULL, NULL)
    assert rc == -1
    assert "static partials" in err(lib)


def test_mlp_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.bessel_mlp_create(FAKE_A, 7, ctypes.byref(h)) == -1  # wrong parameter count
    assert lib.bessel_mlp_create(NULL, 4490, NULL) == -1
    assert lib.bessel_mlp_destroy(NULL) == 0


def test_hess_argument_errors(lib):
    outs = [FAKE_C, NULL, NULL, NULL, NULL, NULL]
    assert lib.bessel_logk_hess(7, 4, FAKE_A, FAKE_B, *outs, 128, NULL) == -2
    assert lib.bessel_logk_hess(1, -1, FAKE_A, FAKE_B, *outs, 128, NULL) == -1
    assert lib.bessel_logk_hess(1, 4, FAKE_A, FAKE_B, *outs, 1, NULL) == -3
    assert lib.bessel_logk_hess(1, 4, FAKE_A, FAKE_B, *([NULL] * 6), 128, NULL) == -1
    assert lib.bessel_logk_hess(1, 4, FAKE_A, FAKE_B, FAKE_A, *([NULL] * 5), 128, NULL) == -6
    assert lib.bessel_logk_hess(1, 4, FAKE_A, FAKE_B, FAKE_C, FAKE_C, *([NULL] * 4), 128, NULL) == -6
    assert lib.bessel_logk_hess(1, 0, NULL, NULL, *([NULL] * 6), 128, NULL) == 0


def test_hess_vjp_argument_errors(lib):
    assert lib.bessel_hess_vjp(1, 4, NULL, NULL, FAKE_A, FAKE_A, FAKE_A, FAKE_B, NULL, NULL) == -1
    assert lib.bessel_hess_vjp(1, 4, FAKE_A, NULL, FAKE_B, NULL, NULL, FAKE_C, NULL, NULL) == -1
    assert lib.bessel_hess_vjp(1, 4, FAKE_A, NULL, FAKE_B, NULL, FAKE_B, FAKE_A, NULL, NULL) == -6
    assert lib.bessel_hess_vjp(3, 4, FAKE_A, NULL, FAKE_B, NULL, FAKE_B, FAKE_C, NULL, NULL) == -2
    assert lib.bessel_hess_vjp(1, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL) == 0


def test_split_threshold_setter(lib):
    prev = ctypes.c_int64()
    assert lib.bessel_set_split_threshold(-1, ctypes.byref(prev)) == -1
    assert lib.bessel_set_split_threshold((1 << 26) + 1, NULL) == -1
    assert lib.bessel_set_split_threshold(77, ctypes.byref(prev)) == 0
    old = prev.value
    assert lib.bessel_set_split_threshold(old, ctypes.byref(prev)) == 0
    assert prev.value == 77


def test_logdk_argument_errors(lib):
    # dtype, n, v, x, order_v, order_x, logdk, sign, nbins, stream
    assert lib.bessel_logdk(5, 4, FAKE_A, FAKE_B, 1, 0, FAKE_C, NULL, 128, NULL) == -2
    assert lib.bessel_logdk(1, -1, FAKE_A, FAKE_B, 1, 0, FAKE_C, NULL, 128, NULL) == -1
    assert lib.bessel_logdk(1, 4, NULL, FAKE_B, 1, 0, FAKE_C, NULL, 128, NULL) == -1
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 9, 0, FAKE_C, NULL, 128, NULL) == -8
    assert "orders" in err(lib)
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 0, -1, FAKE_C, NULL, 128, NULL) == -8
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 1, 0, FAKE_C, NULL, 1, NULL) == -3
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 1, 0, NULL, NULL, 128, NULL) == -1
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 1, 0, FAKE_A, NULL, 128, NULL) == -6
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 1, 0, FAKE_C, FAKE_B, 128, NULL) == -6
    assert lib.bessel_logdk(1, 4, FAKE_A, FAKE_B, 1, 0, FAKE_C, FAKE_C, 128, NULL) == -6
    assert lib.bessel_logdk(1, 0, NULL, NULL, 8, 8, NULL, NULL, 128, NULL) == 0
    assert _lib.STATUS[-8] == "BESSEL_ERR_ORDER"
