"""Host-only checks of the C ABI: the library loads and exports every entry point that
include/bie.h declares; argument errors come back as error codes without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bie.h")
LIB = os.path.join(ROOT, "paper_1707_06551_amd", "libbie.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bie_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["bie_build_spheres", "bie_apply_bio", "bie_solve_resistance", "bie_solve_mobility",
                     "bie_free", "bie_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbie.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(L, name), name
    from paper_1707_06551_amd import bie
    assert sorted(bie.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbie.so not built")
def test_null_arguments_are_rejected_without_a_device():
    L = ctypes.CDLL(LIB)
    L.bie_apply_bio.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.bie_apply_bio.restype = ctypes.c_int
    L.bie_last_error.restype = ctypes.c_char_p
    assert L.bie_apply_bio(None, 3, 0, None, None) == -1
    assert b"null" in L.bie_last_error()
    L.bie_build_spheres.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.bie_build_spheres.restype = ctypes.c_int
    assert L.bie_build_spheres(None, 0, None, None) == -1


def test_options_struct_matches_the_header():
    # field order and types of bie_opts in include/bie.h against the binding's mirror
    from paper_1707_06551_amd import bie
    body = re.search(r"typedef struct \{(.*?)\} bie_opts;", open(HEADER).read(), re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(int|double|void\*)\s+(\w+);", body)
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double, "void*": ctypes.c_void_p}
    assert [(n, ctype[t]) for t, n in fields] == list(bie.Opts._fields_)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbie.so not built")
@pytest.mark.parametrize("bad", [dict(p=0), dict(p=21), dict(n_phi=7), dict(n_phi=6), dict(near_method=2),
                                 dict(legendre_mfma=2), dict(n_spheres=0), dict(n_spheres=65537),
                                 dict(near_gap=float("inf")), dict(near_gap=float("nan")),
                                 dict(near_gap=0.0, near_tol=float("nan")), dict(near_gap=0.0, near_tol=2.0)])
def test_invalid_options_are_rejected_before_any_device_call(bad):
    import numpy as np
    from paper_1707_06551_amd import bie
    L = ctypes.CDLL(LIB)
    L.bie_build_spheres.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.bie_build_spheres.restype = ctypes.c_int
    L.bie_last_error.restype = ctypes.c_char_p
    kw = dict(p=4, n_phi=0, near_method=0, legendre_mfma=0, n_spheres=2, near_gap=1.0, near_tol=0.0)
    kw.update(bad)
    o = bie.Opts(kw["p"], kw["n_phi"], kw["near_gap"], 0, None, kw["near_method"], kw["legendre_mfma"], kw["near_tol"])
    centres = np.arange(3 * max(kw["n_spheres"], 1), dtype=np.float64) * 3.0
    h = ctypes.c_void_p()
    rc = L.bie_build_spheres(centres.ctypes.data, kw["n_spheres"], ctypes.byref(o), ctypes.byref(h))
    assert rc == -1 and h.value is None, (rc, L.bie_last_error())
    assert L.bie_last_error()
