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


def header_struct(name):
    """(field, ctypes type) of a typedef struct of include/bie.h, in order."""
    body = re.search(r"typedef struct \{([^{}]*?)\} " + name + ";", open(HEADER).read(), re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double, "void*": ctypes.c_void_p, "long long": ctypes.c_longlong,
             "const double*": ctypes.c_void_p, "double*": ctypes.c_void_p}
    out = []
    for t, n, k in re.findall(r"((?:const\s+)?(?:long long|int|double|void)\s*\*?)\s*(\w+)(?:\[(\d+)\])?;", body):
        ct = ctype[re.sub(r"\s+\*", "*", t.strip())]
        out.append((n, ct * int(k) if k else ct))
    return out


@pytest.mark.parametrize("name,cls", [("bie_opts", "Opts"), ("bie_solve_opts", "SolveOpts"),
                                      ("bie_solve_info", "SolveInfo")])
def test_structs_match_the_header(name, cls):
    # field order, types and the resulting size of each option / result struct of
    # include/bie.h against the binding's mirror
    from paper_1707_06551_amd import bie
    fields = header_struct(name)
    mirror = getattr(bie, cls)
    assert [n for n, _ in fields] == [n for n, _ in mirror._fields_]
    for (n, t), (_, u) in zip(fields, mirror._fields_):
        assert ctypes.sizeof(t) == ctypes.sizeof(u) and getattr(t, "_length_", 0) == getattr(u, "_length_", 0), n

    class Ref(ctypes.Structure):
        _fields_ = fields
    assert ctypes.sizeof(Ref) == ctypes.sizeof(mirror)
    for n, _ in fields:
        assert getattr(Ref, n).offset == getattr(mirror, n).offset, n


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
