"""Thin ctypes binding of libbie.so (C ABI in include/bie.h).

Argument marshalling only: every step of the method runs in the HIP library.  Device
arrays are torch tensors on a HIP device (float64, contiguous); their data pointers and
the current torch stream are handed to the library.  Loading fails loudly when the
library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbie.so")

OP_S, OP_D, OP_SD_BIE, OP_DN_BIE, OP_MOBILITY = 1, 2, 3, 4, 5
STAGE_SELF, STAGE_NEAR, STAGE_FAR = 0x100, 0x200, 0x400
FP64, MIXED = 0, 1
PC_NONE, PC_M0, PC_MLP = 0, 1, 2
OK, ENOCONV, EINVAL, EOVERLAP, EDEVICE, ENOMEM = 0, 1, -1, -2, -3, -4

EXPORTED = [
    "bie_build_spheres", "bie_free", "bie_sizes", "bie_get_nodes", "bie_near_pairs", "bie_apply_bio",
    "bie_vsh_forward", "bie_vsh_inverse", "bie_solve_resistance", "bie_solve_mobility", "bie_last_error",
]


class Opts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("n_phi", ctypes.c_int), ("near_gap", ctypes.c_double),
                ("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_steps", ctypes.c_int), ("matvecs_fp64", ctypes.c_int),
                ("matvecs_mixed", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libbie.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1707_06551_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.bie_build_spheres.argtypes = [VP, I64, P(Opts), P(VP)]
    L.bie_build_spheres.restype = I
    L.bie_free.argtypes = [VP]
    L.bie_free.restype = None
    L.bie_sizes.argtypes = [VP, P(I64), P(I64), P(I64), P(I64)]
    L.bie_sizes.restype = I
    L.bie_get_nodes.argtypes = [VP, VP, VP]
    L.bie_get_nodes.restype = I
    L.bie_near_pairs.argtypes = [VP, P(I64), VP]
    L.bie_near_pairs.restype = I
    L.bie_apply_bio.argtypes = [VP, I, I, VP, VP]
    L.bie_apply_bio.restype = I
    L.bie_vsh_forward.argtypes = [VP, I, VP, VP]
    L.bie_vsh_forward.restype = I
    L.bie_vsh_inverse.argtypes = [VP, I, VP, VP]
    L.bie_vsh_inverse.restype = I
    L.bie_solve_resistance.argtypes = [VP, VP, VP, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_resistance.restype = I
    L.bie_solve_mobility.argtypes = [VP, VP, VP, VP, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_mobility.restype = I
    L.bie_last_error.argtypes = []
    L.bie_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


class BieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bie error {code}: {msg}")
        self.code = code


def _check(rc, allow_noconv=False):
    if rc == OK or (allow_noconv and rc == ENOCONV):
        return rc
    raise BieError(rc, lib().bie_last_error().decode())


def _hptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "expected a contiguous float64 device tensor"
    return ctypes.c_void_p(t.data_ptr())


class Spheres:
    """A context for n_b unit spheres (bie_build_spheres)."""

    def __init__(self, centres, p, n_phi=0, near_gap=1.0, device=0, stream=None):
        import torch
        L = lib()
        c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        o = Opts(p, n_phi, near_gap, device, ctypes.c_void_p(stream.cuda_stream))
        h = ctypes.c_void_p()
        _check(L.bie_build_spheres(_hptr(c), c.shape[0], ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        n, nb, P, mm = (ctypes.c_int64() for _ in range(4))
        _check(L.bie_sizes(h, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(P), ctypes.byref(mm)))
        self.N, self.nb, self.P, self.mmax, self.p = n.value, nb.value, P.value, mm.value, p
        self.ncoef = sum(p + 1 - m for m in range(self.mmax + 1))

    def close(self):
        if getattr(self, "_h", None):
            lib().bie_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self):
        xyz = np.empty((self.N, 3))
        w = np.empty(self.N)
        _check(lib().bie_get_nodes(self._h, _hptr(xyz), _hptr(w)))
        return xyz, w

    def near_pairs(self):
        cnt = ctypes.c_int64()
        _check(lib().bie_near_pairs(self._h, ctypes.byref(cnt), None))
        pairs = np.empty((2, cnt.value), dtype=np.int64)
        _check(lib().bie_near_pairs(self._h, ctypes.byref(cnt), _hptr(pairs)))
        return pairs

    def dof(self, op):
        return 3 * self.N + (6 * self.nb if (op & 0xff) == OP_MOBILITY else 0)

    def apply(self, op, mu, u=None, precision=FP64):
        import torch
        if u is None:
            u = torch.empty(self.dof(op), dtype=torch.float64, device=mu.device)
        _check(lib().bie_apply_bio(self._h, op, precision, _dptr(mu), _dptr(u)))
        return u

    def vsh_forward(self, mu, precision=FP64):
        import torch
        coef = torch.empty(self.nb * 3 * self.ncoef * 2, dtype=torch.float64, device=mu.device)
        _check(lib().bie_vsh_forward(self._h, precision, _dptr(mu), _dptr(coef)))
        return coef

    def vsh_inverse(self, coef, precision=FP64):
        import torch
        u = torch.empty(3 * self.N, dtype=torch.float64, device=coef.device)
        _check(lib().bie_vsh_inverse(self._h, precision, _dptr(coef), _dptr(u)))
        return u

    @staticmethod
    def _sopts(tol, restart, max_iter, precision, precond, inner_tol):
        return SolveOpts(tol, restart, max_iter, precision, precond, inner_tol)

    def solve_resistance(self, v, omega, tol=1e-8, restart=100, max_iter=1000, precision=FP64, precond=PC_NONE,
                         inner_tol=1e-4, want_psi=False):
        import torch
        v = np.ascontiguousarray(v, dtype=np.float64)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        F = np.empty((self.nb, 3))
        T = np.empty((self.nb, 3))
        psi = torch.empty(3 * self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_psi else None
        info = SolveInfo()
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol)
        rc = lib().bie_solve_resistance(self._h, _hptr(v), _hptr(om), ctypes.byref(so), _hptr(F), _hptr(T),
                                        _dptr(psi) if psi is not None else None, ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return F, T, psi, dict(info.as_dict(), converged=(rc == OK))

    def solve_mobility(self, F, T, slip=None, tol=1e-8, restart=100, max_iter=1000, precision=FP64,
                       precond=PC_NONE, inner_tol=1e-4, want_mu=False):
        import torch
        F = np.ascontiguousarray(F, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        v = np.empty((self.nb, 3))
        om = np.empty((self.nb, 3))
        mu = torch.empty(3 * self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_mu else None
        info = SolveInfo()
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol)
        rc = lib().bie_solve_mobility(self._h, _hptr(F), _hptr(T), _dptr(slip) if slip is not None else None,
                                      ctypes.byref(so), _hptr(v), _hptr(om),
                                      _dptr(mu) if mu is not None else None, ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return v, om, mu, dict(info.as_dict(), converged=(rc == OK))
