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


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3), (90, 4)])
def test_host_eigensolver_matches_lapack(sg, n, seed):
    # the small eigensolver of the deflation setup runs on the host: check it
    # against LAPACK (numpy.linalg.eig) without a GPU
    import numpy as np

    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Af = np.asfortranarray(A)
    w = np.zeros(n, complex)
    V = np.zeros((n, n), complex, order="F")
    st = sg.lib.sgn_host_eig(n, Af.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                              V.ctypes.data_as(C.c_void_p))
    assert st == 0
    ref = np.linalg.eigvals(A)
    d = np.abs(w[:, None] - ref[None, :])
    assert d.min(axis=1).max() < 1e-10 * max(1, np.abs(ref).max())
    assert np.linalg.norm(A @ V - V * w[None, :]) < 1e-10 * np.linalg.norm(A)
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)


def test_host_eigensolver_on_hessenberg_and_triangular(sg):
    import numpy as np

    rng = np.random.default_rng(9)
    n = 30
    for A in (np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1),
              np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))),
              np.diag(np.arange(1, n + 1) * (1 + 0.5j))):
        Af = np.asfortranarray(A)
        w = np.zeros(n, complex)
        V = np.zeros((n, n), complex, order="F")
        assert sg.lib.sgn_host_eig(n, Af.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                                   V.ctypes.data_as(C.c_void_p)) == 0
        assert np.linalg.norm(A @ V - V * w[None, :]) < 1e-10 * np.linalg.norm(A)


def test_binding_covers_every_declared_function(sg):
    # the Python binding names every entry point of the header (same names)
    src = open(os.path.join(ROOT, "paper_0704_3486_amd", "__init__.py")).read()
    missing = [n for n in declared_functions() if f'"{n}"' not in src]
    assert not missing, missing
