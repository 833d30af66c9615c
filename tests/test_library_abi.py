"""librr.so loads and exports every symbol that include/rr.h declares (CPU only: no compute)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rr.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2501_07642_amd import _lib
    if not os.path.exists(_lib.lib_path()):
        pytest.fail("librr.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(_lib.lib_path())


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["rr_prepare", "rr_draw_balance", "rr_draw_exact", "rr_regenerate", "rr_balance_keys",
              "rr_rand_test", "rr_draw_balance_batched", "rr_free", "rr_last_error"]:
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_binding_covers_every_symbol():
    from paper_2501_07642_amd import _lib
    assert sorted(name for name, _, _ in _lib.SIGNATURES) == declared_symbols()


def test_binding_loads_and_errors_without_device(lib):
    import paper_2501_07642_amd as rr
    L = rr.load()
    assert isinstance(L.rr_last_error(), bytes)
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    st = L.rr_prepare(None, 0, 10, 3, 3, 5, 0.0, None, ctypes.byref(h))
    assert rr._lib.STATUS[st] == "RR_E_ARG"
    assert b"invalid" in L.rr_last_error()


def test_shape_limits_rejected_before_device_use(lib):
    """n above RR_MAX_N and d above RR_MAX_D are refused before any device call (the pointer is
    never dereferenced)."""
    import paper_2501_07642_amd as rr
    L = rr.load()
    text = open(HEADER).read()
    max_n = int(re.search(r"#define RR_MAX_N (\d+)", text).group(1))
    max_d = eval(re.search(r"#define RR_MAX_D (\(1 << \d+\))", text).group(1))
    fake = ctypes.c_void_p(256)
    h = ctypes.c_void_p()
    st = L.rr_prepare(fake, 0, max_n + 1, 3, 3, 5, 0.0, None, ctypes.byref(h))
    assert rr._lib.STATUS[st] == "RR_E_UNSUPPORTED" and b"RR_MAX_N" in L.rr_last_error()
    st = L.rr_prepare(fake, 0, 10, max_d + 1, max_d + 1, 5, 0.0, None, ctypes.byref(h))
    assert rr._lib.STATUS[st] == "RR_E_UNSUPPORTED" and b"RR_MAX_D" in L.rr_last_error()
    assert not h.value
