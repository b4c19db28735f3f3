"""CPU-side checks of the C-ABI library: it loads, exports every declared entry point, and
the binding's signatures cover the header.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "vbarms.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vbarms_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def built():
    from paper_1508_02219_amd import build, vbarms
    if not os.path.exists(vbarms.LIB_PATH):
        build.build()
    return vbarms


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("vbarms_create", "vbarms_destroy", "vbarms_compress", "vbarms_factor", "vbarms_apply",
                     "vbarms_solve", "vbarms_spmv", "vbarms_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(built):
    lib = ctypes.CDLL(built.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header(built):
    assert sorted(built.SIGNATURES) == _declared()


def test_binding_loads_library(built):
    lib = built.lib()
    for name in _declared():
        assert getattr(lib, name).restype is not None or name == "vbarms_destroy"


def test_create_without_device_fails_cleanly(built):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = built.lib().vbarms_create(ctypes.byref(h), None)
    assert rc == built.ERR_HIP and not h.value


def test_null_handle_is_rejected(built):
    lib = built.lib()
    assert lib.vbarms_factor(None, None) == built.ERR_ARG
    assert lib.vbarms_destroy(None) == built.ERR_ARG
    assert lib.vbarms_last_error(None) == b"invalid handle"
