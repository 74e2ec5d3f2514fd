"""The C-ABI library loads and exports every entry point include/sps.h declares
(no compute calls: this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_19919_amd", "libsps.so")
HDR = os.path.join(ROOT, "include", "sps.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sps_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("sps_weights", "sps_phot_exact", "sps_phot_approx", "sps_loglike_grad", "sps_hmc_run",
              "sps_create", "sps_destroy", "sps_last_error", "sps_build_ztable"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsps.so not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsps.so not built")
def test_binding_lists_every_declared_symbol():
    import paper_2506_19919_amd as sps
    assert set(declared()) == set(sps.ABI_FUNCTIONS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsps.so not built")
def test_create_rejects_null_arguments_without_touching_the_device():
    lib = C.CDLL(LIB)
    lib.sps_last_error.restype = C.c_char_p
    h = C.c_void_p(123)
    rc = lib.sps_create(C.byref(h), 0, None, None, None, 0, 10)
    assert rc == 1 and h.value is None
    assert b"null" in lib.sps_last_error()
    assert lib.sps_create(None, 0, None, None, None, 0, 10) == 1
