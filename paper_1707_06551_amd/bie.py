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
OP_K, OP_KL_BIE = 6, 7   # single-layer traction; 1/2 I + K + L of the traction mobility form
STAGE_SELF, STAGE_NEAR, STAGE_FAR = 0x100, 0x200, 0x400
FP64, MIXED = 0, 1
PC_NONE, PC_M0, PC_MLP = 0, 1, 2
PC_RIGID = 0x10   # flag: global rigid-mode coarse correction (resistance form)
PC_LOCAL = 0x20   # flag: learned correction on the base preconditioner's local residual
OK, ENOCONV, EINVAL, EOVERLAP, EDEVICE, ENOMEM = 0, 1, -1, -2, -3, -4

EXPORTED = [
    "bie_build_spheres", "bie_free", "bie_sizes", "bie_get_nodes", "bie_near_pairs", "bie_apply_bio",
    "bie_vsh_forward", "bie_vsh_inverse", "bie_solve_resistance", "bie_solve_mobility", "bie_last_error",
    "bie_solve", "bie_apply_precond", "bie_lowmodes", "bie_lowmodes_synth", "bie_pair_geometry",
    "bie_mlp_n_weights", "bie_precond_load", "bie_mlp_eval", "bie_mlp_train", "bie_eval_field",
    "bie_apply_laplace", "bie_solve_magnetic", "bie_solve_mobility_traction", "bie_build_spheres_radii",
    "bie_num_nodes", "bie_near_gap", "bie_near_gap_for", "bie_apply_bio_noalloc", "bie_precond_sample",
]
NLOW = 25
NFEAT = 8
NFRAME = 34


class MlpData(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("n_spheres", ctypes.c_int64), ("n_configs", ctypes.c_int64),
                ("n_rhs", ctypes.c_int32), ("feats", ctypes.c_void_p), ("frames", ctypes.c_void_p),
                ("pair_i", ctypes.c_void_p), ("pair_j", ctypes.c_void_p), ("sph_ptr", ctypes.c_void_p),
                ("cfg_sph", ctypes.c_void_p), ("cfg_pair", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("target", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("n_phi", ctypes.c_int), ("near_gap", ctypes.c_double),
                ("device", ctypes.c_int), ("hip_stream", ctypes.c_void_p), ("near_method", ctypes.c_int),
                ("legendre_mfma", ctypes.c_int), ("near_tol", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("x0", ctypes.c_void_p), ("res_hist", ctypes.c_void_p), ("res_hist_cap", ctypes.c_int)]


T_TRANSFORM, T_NEAR, T_FAR, T_PRECOND, T_KRYLOV, T_OTHER = range(6)
STAGE_NAMES = ("transform", "near", "far", "precond", "krylov", "other")


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_steps", ctypes.c_int), ("matvecs_fp64", ctypes.c_int),
                ("matvecs_mixed", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("t_stage_s", ctypes.c_double * 8), ("pairs_evaluated", ctypes.c_longlong),
                ("near_evals", ctypes.c_longlong), ("res_hist_len", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "t_stage_s"}
        d["t_stage_s"] = {n: self.t_stage_s[i] for i, n in enumerate(STAGE_NAMES)}
        return d


_lib = None


def lib():
    """Load libbie.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_1707_06551_amd.build`")
    # torch ships its own HIP runtime under the same soname as the system one that the
    # library links: importing torch first makes the library bind to torch's copy, so the
    # process holds one runtime (device pointers and streams cross between the two).
    # Loaded the other way round the process would hold two, and torch's finds no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, VP = ctypes.POINTER, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    L.bie_build_spheres.argtypes = [VP, I64, P(Opts), P(VP)]
    L.bie_build_spheres.restype = I
    L.bie_build_spheres_radii.argtypes = [VP, VP, I64, P(Opts), P(VP)]
    L.bie_build_spheres_radii.restype = I
    L.bie_free.argtypes = [VP]
    L.bie_free.restype = None
    L.bie_sizes.argtypes = [VP, P(I64), P(I64), P(I64), P(I64)]
    L.bie_sizes.restype = I
    L.bie_num_nodes.argtypes = [VP, P(I64)]
    L.bie_num_nodes.restype = I
    L.bie_near_gap.argtypes = [VP, P(D), P(D)]
    L.bie_near_gap.restype = I
    L.bie_near_gap_for.argtypes = [I, I, D, P(D)]
    L.bie_near_gap_for.restype = I
    L.bie_get_nodes.argtypes = [VP, VP, VP]
    L.bie_get_nodes.restype = I
    L.bie_near_pairs.argtypes = [VP, P(I64), VP]
    L.bie_near_pairs.restype = I
    L.bie_apply_bio.argtypes = [VP, I, I, VP, VP]
    L.bie_apply_bio.restype = I
    L.bie_apply_bio_noalloc.argtypes = [VP, I, I, VP, VP]
    L.bie_apply_bio_noalloc.restype = I
    L.bie_vsh_forward.argtypes = [VP, I, VP, VP]
    L.bie_vsh_forward.restype = I
    L.bie_vsh_inverse.argtypes = [VP, I, VP, VP]
    L.bie_vsh_inverse.restype = I
    L.bie_solve_resistance.argtypes = [VP, VP, VP, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_resistance.restype = I
    L.bie_solve_mobility.argtypes = [VP, VP, VP, VP, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_mobility.restype = I
    L.bie_solve_mobility_traction.argtypes = [VP, VP, VP, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_mobility_traction.restype = I
    L.bie_last_error.argtypes = []
    L.bie_last_error.restype = ctypes.c_char_p
    L.bie_solve.argtypes = [VP, I, VP, VP, P(SolveOpts), P(SolveInfo)]
    L.bie_solve.restype = I
    L.bie_apply_precond.argtypes = [VP, I, I, I, VP, VP]
    L.bie_apply_precond.restype = I
    L.bie_eval_field.argtypes = [VP, I, VP, I64, VP, VP]
    L.bie_eval_field.restype = I
    L.bie_apply_laplace.argtypes = [VP, I, D, VP, VP]
    L.bie_apply_laplace.restype = I
    L.bie_solve_magnetic.argtypes = [VP, VP, D, P(SolveOpts), VP, VP, VP, P(SolveInfo)]
    L.bie_solve_magnetic.restype = I
    L.bie_lowmodes.argtypes = [VP, VP, VP]
    L.bie_lowmodes.restype = I
    L.bie_lowmodes_synth.argtypes = [VP, VP, VP]
    L.bie_lowmodes_synth.restype = I
    L.bie_pair_geometry.argtypes = [VP, P(I64), VP, VP, VP, VP]
    L.bie_pair_geometry.restype = I
    L.bie_precond_sample.argtypes = [VP, I, I, VP, VP, VP, VP]
    L.bie_precond_sample.restype = I
    L.bie_mlp_n_weights.argtypes = []
    L.bie_mlp_n_weights.restype = I64
    L.bie_precond_load.argtypes = [VP, VP, I64]
    L.bie_precond_load.restype = I
    L.bie_mlp_eval.argtypes = [P(MlpData), VP, P(D), VP]
    L.bie_mlp_eval.restype = I
    L.bie_mlp_train.argtypes = [P(MlpData), VP, I, I, D, VP]
    L.bie_mlp_train.restype = I
    _lib = L
    return L


def mlp_n_weights():
    return int(lib().bie_mlp_n_weights())


def near_gap_for(p, tol, n_phi=0):
    """d* of Eq. 4.5 for grid order p and precision tol (bie_near_gap_for; host only)."""
    d = ctypes.c_double()
    _check(lib().bie_near_gap_for(p, n_phi, tol, ctypes.byref(d)))
    return d.value


class TrainingSet:
    """Host-side packing of MLP training data (see bie_mlp_data in include/bie.h)."""

    def __init__(self, n_rhs):
        self.n_rhs = n_rhs
        self.feats, self.frames, self.pi, self.pj, self.xi, self.t = [], [], [], [], [], []
        self.cfg_sph, self.cfg_pair = [0], [0]
        self.sph_ptr = [0]

    def add(self, pair_i, pair_j, feats, frames, xi, target):
        """One configuration: pairs grouped by target sphere; xi, target (nb, n_rhs, 25)."""
        s0, p0 = self.cfg_sph[-1], self.cfg_pair[-1]
        nb = xi.shape[0]
        counts = np.bincount(pair_i, minlength=nb)
        self.pi.append(pair_i.astype(np.int32) + s0)
        self.pj.append(pair_j.astype(np.int32) + s0)
        self.feats.append(np.asarray(feats, np.float32))
        self.frames.append(np.asarray(frames, np.float32))
        self.xi.append(np.asarray(xi, np.float32))
        self.t.append(np.asarray(target, np.float32))
        self.sph_ptr.extend((p0 + np.cumsum(counts)).tolist())
        self.cfg_sph.append(s0 + nb)
        self.cfg_pair.append(p0 + len(pair_i))

    def pack(self):
        cat = lambda xs, dt, w: np.ascontiguousarray(np.concatenate(xs).astype(dt)) if xs else np.zeros((0, w), dt)
        self._arrs = dict(
            feats=cat(self.feats, np.float32, NFEAT), frames=cat(self.frames, np.float32, NFRAME),
            pi=cat(self.pi, np.int32, 1), pj=cat(self.pj, np.int32, 1),
            sph=np.ascontiguousarray(np.array(self.sph_ptr, np.int32)),
            cs=np.ascontiguousarray(np.array(self.cfg_sph, np.int32)),
            cp=np.ascontiguousarray(np.array(self.cfg_pair, np.int32)),
            xi=cat(self.xi, np.float32, 1), t=cat(self.t, np.float32, 1))
        a = self._arrs
        d = MlpData(a["pi"].size, a["cs"][-1], len(self.cfg_sph) - 1, self.n_rhs, _hptr(a["feats"]),
                    _hptr(a["frames"]), _hptr(a["pi"]), _hptr(a["pj"]), _hptr(a["sph"]), _hptr(a["cs"]),
                    _hptr(a["cp"]), _hptr(a["xi"]), _hptr(a["t"]))
        self._data = d
        return d

    def eval(self, weights):
        d = self.pack()
        w = np.ascontiguousarray(weights, np.float32)
        g = np.empty_like(w)
        loss = ctypes.c_double()
        _check(lib().bie_mlp_eval(ctypes.byref(d), _hptr(w), ctypes.byref(loss), _hptr(g)))
        return loss.value, g

    def train(self, weights, epochs, cfg_per_batch=8, lr=1e-3):
        d = self.pack()
        w = np.ascontiguousarray(weights, np.float32).copy()
        hist = np.zeros(max(1, epochs))
        _check(lib().bie_mlp_train(ctypes.byref(d), _hptr(w), epochs, cfg_per_batch, lr, _hptr(hist)))
        return w, hist[:epochs]


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
    """A context for n_b spheres (bie_build_spheres; bie_build_spheres_radii when radii
    are given: polydisperse suspensions, a subset of the operators).  legendre_mfma = 1
    runs the transforms' Legendre stages on the matrix cores (bie_opts.legendre_mfma).
    near_gap = None (or <= 0) measures d* of Eq. 4.5 for the precision near_tol
    (None: the library's default, 1e-8); a positive near_gap is taken as given."""

    def __init__(self, centres, p, n_phi=0, near_gap=None, device=0, stream=None, near_method=0, radii=None,
                 legendre_mfma=0, near_tol=None):
        import torch
        L = lib()
        c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        o = Opts(p, n_phi, 0.0 if near_gap is None else near_gap, device, ctypes.c_void_p(stream.cuda_stream),
                 near_method, legendre_mfma, 0.0 if near_tol is None else near_tol)
        h = ctypes.c_void_p()
        if radii is None:
            _check(L.bie_build_spheres(_hptr(c), c.shape[0], ctypes.byref(o), ctypes.byref(h)))
        else:
            rad = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
            if rad.size != c.shape[0]:
                raise ValueError("one radius per sphere")
            _check(L.bie_build_spheres_radii(_hptr(c), _hptr(rad), c.shape[0], ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        n, nb, P, mm = (ctypes.c_int64() for _ in range(4))
        _check(L.bie_sizes(h, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(P), ctypes.byref(mm)))
        self.N, self.nb, self.P, self.mmax, self.p = n.value, nb.value, P.value, mm.value, p
        self.ncoef = sum(p + 1 - m for m in range(self.mmax + 1))
        d, t = ctypes.c_double(), ctypes.c_double()
        _check(L.bie_near_gap(h, ctypes.byref(d), ctypes.byref(t)))
        self.near_gap, self.near_tol = d.value, t.value
        cnt = ctypes.c_int64()
        _check(L.bie_near_pairs(h, ctypes.byref(cnt), None))
        self.n_near = cnt.value
        # node pairs of one far-field pass: all ordered pairs of distinct, well-separated spheres
        self.far_node_pairs = (self.nb * (self.nb - 1) - self.n_near) * self.P * self.P

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

    def apply_noalloc(self, op, mu, u, precision=FP64):
        """bie_apply_bio_noalloc: as apply(), with the work buffers in the library's
        static device array (no device allocation); u must be given."""
        _check(lib().bie_apply_bio_noalloc(self._h, op, precision, _dptr(mu), _dptr(u)))
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

    def solve(self, op, b, tol=1e-8, restart=100, max_iter=1000, precision=FP64, precond=PC_NONE, inner_tol=1e-4,
              x0=None, history=0):
        """Generic solve A x = b (device tensors) for OP_DN_BIE, OP_MOBILITY, OP_SD_BIE or OP_KL_BIE."""
        import torch
        x = torch.empty_like(b)
        info = SolveInfo()
        hist = np.zeros(history) if history else None
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol, x0, hist)
        rc = lib().bie_solve(self._h, op, _dptr(b), _dptr(x), ctypes.byref(so), ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return x, self._info(info, rc, hist)

    def apply_precond(self, op, r, precond=PC_M0, precision=FP64):
        import torch
        z = torch.empty_like(r)
        _check(lib().bie_apply_precond(self._h, op, precision, precond, _dptr(r), _dptr(z)))
        return z

    def apply_laplace(self, kind, q, eta=0.0, out=None):
        """kind 0: (1/2 I + eta K^L)[q] (N); kind 1: exterior gradient of S^L[q] (3N)."""
        import torch
        if out is None:
            out = torch.empty(self.N * (1 if kind == 0 else 3), dtype=torch.float64, device=q.device)
        _check(lib().bie_apply_laplace(self._h, kind, eta, _dptr(q), _dptr(out)))
        return out

    def solve_magnetic(self, H0, eta, tol=1e-10, restart=100, max_iter=1000, precond=PC_M0, want_q=False, x0=None,
                       history=0):
        """Problem 3: magnetic forces and torques (nb, 3) on the spheres in the field H0."""
        import torch
        h = np.ascontiguousarray(H0, dtype=np.float64).reshape(3)
        F = np.empty((self.nb, 3))
        T = np.empty((self.nb, 3))
        q = torch.empty(self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_q else None
        info = SolveInfo()
        hist = np.zeros(history) if history else None
        so = self._sopts(tol, restart, max_iter, FP64, precond, 1e-4, x0, hist)
        rc = lib().bie_solve_magnetic(self._h, _hptr(h), eta, ctypes.byref(so), _dptr(q) if q is not None else None,
                                      _hptr(F), _hptr(T), ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return F, T, q, self._info(info, rc, hist)

    def eval_field(self, op, mu, targets, u=None):
        """Layer potential of op (OP_S, OP_D, OP_SD_BIE, OP_DN_BIE) of the node density mu
        (device, 3N) at fluid points targets ((M, 3) host array or device tensor) ->
        device tensor (3M)."""
        import torch
        if torch.is_tensor(targets):
            t = targets.contiguous()
        else:
            t = torch.from_numpy(np.ascontiguousarray(targets, dtype=np.float64).reshape(-1, 3)).to(mu.device)
        m = t.numel() // 3
        if u is None:
            u = torch.empty(3 * m, dtype=torch.float64, device=mu.device)
        _check(lib().bie_eval_field(self._h, op, _dptr(mu), m, _dptr(t) if m else None, _dptr(u) if m else None))
        return u

    def lowmodes(self, f):
        import torch
        rho = torch.empty(self.nb * NLOW, dtype=torch.float64, device=f.device)
        _check(lib().bie_lowmodes(self._h, _dptr(f), _dptr(rho)))
        return rho

    def lowmodes_synth(self, rho):
        import torch
        f = torch.empty(3 * self.N, dtype=torch.float64, device=rho.device)
        _check(lib().bie_lowmodes_synth(self._h, _dptr(rho), _dptr(f)))
        return f

    def pair_geometry(self):
        cnt = ctypes.c_int64()
        _check(lib().bie_pair_geometry(self._h, ctypes.byref(cnt), None, None, None, None))
        n = cnt.value
        pi = np.empty(n, np.int32)
        pj = np.empty(n, np.int32)
        feats = np.empty((n, NFEAT), np.float32)
        frames = np.empty((n, NFRAME), np.float64)
        _check(lib().bie_pair_geometry(self._h, ctypes.byref(cnt), _hptr(pi), _hptr(pj), _hptr(feats), _hptr(frames)))
        return pi, pj, feats, frames

    def precond_sample(self, op, precond, b, x):
        """bie_precond_sample: (xi, target), device tensors n_b x 25."""
        import torch
        xi = torch.empty(self.nb * NLOW, dtype=torch.float64, device=b.device)
        t = torch.empty_like(xi)
        _check(lib().bie_precond_sample(self._h, op, precond, _dptr(b), _dptr(x), _dptr(xi), _dptr(t)))
        return xi, t

    def load_precond(self, weights):
        w = np.ascontiguousarray(weights, np.float32)
        _check(lib().bie_precond_load(self._h, _hptr(w), w.size))

    @staticmethod
    def _sopts(tol, restart, max_iter, precision, precond, inner_tol, x0=None, hist=None):
        return SolveOpts(tol, restart, max_iter, precision, precond, inner_tol,
                         _dptr(x0) if x0 is not None else None, _hptr(hist) if hist is not None else None,
                         0 if hist is None else hist.size)

    @staticmethod
    def _info(info, rc, hist):
        d = dict(info.as_dict(), converged=(rc == OK))
        if hist is not None:
            d["res_hist"] = hist[:info.res_hist_len].copy()
        return d

    def solve_resistance(self, v, omega, tol=1e-8, restart=100, max_iter=1000, precision=FP64, precond=PC_NONE,
                         inner_tol=1e-4, want_psi=False, x0=None, history=0):
        import torch
        v = np.ascontiguousarray(v, dtype=np.float64)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        F = np.empty((self.nb, 3))
        T = np.empty((self.nb, 3))
        psi = torch.empty(3 * self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_psi else None
        info = SolveInfo()
        hist = np.zeros(history) if history else None
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol, x0, hist)
        rc = lib().bie_solve_resistance(self._h, _hptr(v), _hptr(om), ctypes.byref(so), _hptr(F), _hptr(T),
                                        _dptr(psi) if psi is not None else None, ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return F, T, psi, self._info(info, rc, hist)

    def solve_mobility_traction(self, F, T, tol=1e-8, restart=100, max_iter=1000, precision=FP64,
                                precond=PC_M0, inner_tol=1e-4, want_mu=False, x0=None, history=0):
        """Problem 2 in the paper's form (Eqs. 5.7-5.8): (v, omega, mu or None, info)."""
        import torch
        F = np.ascontiguousarray(F, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        v = np.empty((self.nb, 3))
        om = np.empty((self.nb, 3))
        mu = torch.empty(3 * self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_mu else None
        info = SolveInfo()
        hist = np.zeros(history) if history else None
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol, x0, hist)
        rc = lib().bie_solve_mobility_traction(self._h, _hptr(F), _hptr(T), ctypes.byref(so), _hptr(v), _hptr(om),
                                               _dptr(mu) if mu is not None else None, ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return v, om, mu, self._info(info, rc, hist)

    def solve_mobility(self, F, T, slip=None, tol=1e-8, restart=100, max_iter=1000, precision=FP64,
                       precond=PC_NONE, inner_tol=1e-4, want_mu=False, x0=None, history=0):
        import torch
        F = np.ascontiguousarray(F, dtype=np.float64)
        T = np.ascontiguousarray(T, dtype=np.float64)
        v = np.empty((self.nb, 3))
        om = np.empty((self.nb, 3))
        mu = torch.empty(3 * self.N, dtype=torch.float64, device=f"cuda:{self.device}") if want_mu else None
        info = SolveInfo()
        hist = np.zeros(history) if history else None
        so = self._sopts(tol, restart, max_iter, precision, precond, inner_tol, x0, hist)
        rc = lib().bie_solve_mobility(self._h, _hptr(F), _hptr(T), _dptr(slip) if slip is not None else None,
                                      ctypes.byref(so), _hptr(v), _hptr(om),
                                      _dptr(mu) if mu is not None else None, ctypes.byref(info))
        _check(rc, allow_noconv=True)
        return v, om, mu, self._info(info, rc, hist)
