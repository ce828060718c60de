"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side argument validation works without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sgn_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def sg():
    import paper_0704_3486_amd as sg
    return sg


def test_header_declares_the_hot_path():
    names = declared_functions()
    for f in ("sgn_create", "sgn_deflate_import", "sgn_apply", "sgn_destroy", "sgn_matvec"):
        assert f in names


def test_every_declared_symbol_is_exported(sg):
    lib = C.CDLL(sg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_covers_all_statuses(sg):
    for st in range(0, -8, -1):
        assert sg.sgn_strerror(st) != "unknown status"
    assert sg.sgn_strerror(-99) == "unknown status"


def test_create_rejects_bad_arguments_on_host(sg):
    lib = sg.lib
    dims = (C.c_int * 4)(4, 4, 1, 4)
    buf = (C.c_double * 8)()
    assert lib.sgn_create(buf, dims, 0.0, -1.6) is None
    assert "extent" in sg.sgn_create_error()
    dims = (C.c_int * 4)(4, 4, 4, 4)
    assert lib.sgn_create(buf, dims, 0.0, -4.0) is None
    assert "m_w" in sg.sgn_create_error()
    assert lib.sgn_create(None, dims, 0.0, -1.6) is None


def test_null_context_is_a_state_error(sg):
    lib = sg.lib
    assert lib.sgn_apply(None, None, None, 1e-8, 10) == sg.SGN_ESTATE
    assert lib.sgn_apply_fixed(None, None, None, 10) == sg.SGN_ESTATE
    assert lib.sgn_deflate_import(None, 0, None, None) == sg.SGN_ESTATE
    assert lib.sgn_matvec(None, None, None) == sg.SGN_ESTATE
    assert lib.sgn_deflation_size(None) == sg.SGN_ESTATE
    assert lib.sgn_footprint_bytes(None, 10, 1) == 0
    lib.sgn_destroy(None)


def test_binding_refuses_host_tensors(sg):
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        sg._dptr(torch.zeros(4, dtype=torch.complex128))
