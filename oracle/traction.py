"""Traction of the Stokes single layer (Eq. 2.22, Section 3.3) and the paper's own
formulation of the mobility problem (Problem 2, Eqs. 5.7-5.8).

Test infrastructure only (see ``oracle/__init__.py``).

The operator
  K[sigma](x) = int T(x, y) n(x) sigma(y) dGamma(y),   T_ijk = -3/(4 pi) r_i r_j r_k / |r|^5,
  r = x - y (Eq. 2.20 as printed), is the traction, at x with unit normal n(x), of the
flow S[sigma]: stress (grad u + grad u^T - p I) with -grad p + lap u = 0 (viscosity 1),
the convention of Eq. 3.18 and of the jump A.6 ([[T[S[sigma]]]] = -sigma).

On n_b unit spheres, at a node x of sphere t, the contribution of sphere s is
* self (s = t): the principal value K_pv = (K_+ + K_-)/2 of Table 3.12, applied
  spectrally like the other self terms (Section 4.1);
* near (gap test of Eq. 4.5): the traction of the exterior series of S_s (Eqs. 3.6-3.8,
  Eq. 3.17) at x with the TARGET sphere's normal, which has tangential components in
  the source frame (the general case of Eq. 3.18).  The paper maps the nine terms of
  Eq. 3.18 to vector harmonics with precomputed matrices (Fig. 1); here the same
  traction is evaluated at the node directly, from the flow written through decaying
  harmonic potentials (below);
* far: the smooth quadrature of Eq. 4.4 with the kernel above.

Harmonic form of the exterior single layer.  With Phi_nm = r^{-n-1} Y_n^m:
  grad Phi_nm = r^{-n-2} V_n^m,   x cross grad Phi_nm = r^{-n-1} X_n^m,
  r^{-n} V_n^m = r^2 grad Phi_nm,  r^{-n} W_n^m = r^2 grad Phi_nm + (2n+1) x Phi_nm
(from the definitions of V, W, X in Eqs. 2.4-2.6).  The exterior branches of Eqs. 3.6-3.8
then read
  u = grad Psi_A + r^2 grad Psi_B + x Psi_C + x cross grad Psi_X,
  Psi_A = sum (s_V sigV + s_WV sigW) Phi,   Psi_B = sum (s_W - s_WV) sigW Phi,
  Psi_C = sum (2n+1) s_W sigW Phi,          Psi_X = sum s_X sigX Phi,
with s_V = n/((2n+1)(2n+3)), s_W = (n+1)/((2n+1)(2n-1)), s_WV = n/(2(2n+1)),
s_X = 1/(2n+1) the coefficients of Eqs. 3.6-3.8.  lap(r^2 grad Phi) = -2(2n+1) grad Phi
and lap(x Phi) = 2 grad Phi give lap u = grad Psi_P with the pressure
  p = Psi_P = sum n sigW Phi
(decaying, so no constant).  The velocity gradient needs Psi, grad Psi and the Hessian
of the potentials; the Hessian is the gradient of the derivative potentials:
d_i Phi_nm is harmonic, decaying, homogeneous of degree -n-2, so
r^{n+2} d_i Phi_nm = e_i . V_n^m is a combination of degree n+1 harmonics, found here by
quadrature projection (exact: the integrand is a polynomial the grid integrates).

Problem 2 in the paper's form (Eqs. 5.7-5.8): u = sum_k S_k[mu + rho] with
  rho_k(x) = F_k / (4 pi) + 3/(8 pi) T_k x (x - c_k)
(int rho = F_k, int (x - c_k) x rho = T_k on a unit sphere: force and torque the particle
exerts on the fluid, the library's convention), and
  (1/2 I + sum_k (K_k + L_k)) mu = -(1/2 I + sum_k K_k) rho,
  L_k[mu](x) = int_k mu + (int_k (y - c_k) x mu) x (x - c_k)   for x on sphere k.
Reading: L_k acts on the targets of its own sphere only (the centroid in its definition
is that of the target's sphere); it lifts the 6-dimensional rigid null space of
1/2 I + K on each sphere and forces zero net force and torque of mu.  The rigid motion
is read off u on each sphere: v_k = (1/4 pi) int_k u, omega_k = 3/(8 pi) int_k (x - c_k) x u.

Parity: pinned by tests/test_oracle_traction.py: the harmonic form reproduces the
exterior series of Eqs. 3.6-3.8; the gradient and Hessian match central differences; the
traction matches brute-force quadrature of the kernel on an upsampled source grid for
arbitrary target normals; with n = e_r it reproduces the exterior branches of
Eqs. 3.19-3.21 and, at r -> 1, the K_+ row of Table 3.12; the traction on a closed sphere
outside the source carries no net force or torque; the pressure matches quadrature of
the Stokeslet pressure; an isolated sphere moves with F/(6 pi), T/(8 pi); the solved
mu has zero force and torque; the velocities agree with the bordered formulation.
"""
import math

import numpy as np

from . import spectra
from .grid import sphere_grid
from .harmonics import mode_list, vsh_at
from .operators import Operators
from .solvers import gmres

C_K = 3.0 / (4.0 * math.pi)


# ---- kernels (Eqs. 2.19-2.22) -----------------------------------------------------------
def traction_sum(x, nx, y, q, chunk=2048):
    """K at points x (T, 3) with normals nx (T, 3) of sources at y (S, 3) with strengths
    q = w * sigma (S, 3): -3/(4 pi) sum r (r . q)(r . n_x) / |r|^5, r = x - y."""
    out = np.zeros((x.shape[0], 3))
    for s0 in range(0, y.shape[0], chunk):
        r = x[:, None, :] - y[None, s0:s0 + chunk, :]
        r2 = np.einsum("tsi,tsi->ts", r, r)
        rq = np.einsum("tsi,si->ts", r, q[s0:s0 + chunk])
        rn = np.einsum("tsi,ti->ts", r, nx)
        out += -C_K * np.einsum("tsi,ts->ti", r, rq * rn / (r2 * r2 * np.sqrt(r2)))
    return out


def pressure_sum(x, y, q):
    """Pressure of S[sigma]: 1/(4 pi) sum (r . q) / |r|^3, r = x - y (Stokeslet pressure)."""
    r = x[:, None, :] - y[None, :, :]
    r2 = np.einsum("tsi,tsi->ts", r, r)
    rq = np.einsum("tsi,si->ts", r, q)
    return (rq / (r2 * np.sqrt(r2))).sum(axis=1) / (4.0 * math.pi)


# ---- spectra (Table 3.12) -----------------------------------------------------------------
def eig_Kplus(n):
    """Table 3.12, row K_+ (exterior limit): (V, W, X)."""
    v = -2.0 * n * (n + 2) / ((2 * n + 1) * (2 * n + 3))
    w = -(2.0 * n * n + 1) / ((2 * n + 1) * (2 * n - 1)) if n >= 1 else 0.0
    x = -(n + 2.0) / (2 * n + 1) if n >= 1 else 0.0
    return v, w, x


def eig_Kminus(n):
    """Table 3.12, row K_- (interior limit): (V, W, X)."""
    v = (2.0 * n * n + 4 * n + 3) / ((2 * n + 1) * (2 * n + 3))
    w = 2.0 * (n - 1) * (n + 1) / ((2 * n + 1) * (2 * n - 1)) if n >= 1 else 0.0
    x = (n - 1.0) / (2 * n + 1) if n >= 1 else 0.0
    return v, w, x


def eig_Kpv(n):
    """Principal value on the surface: the mean of the two one-sided limits (their
    difference is the jump -I of A.6)."""
    return tuple(0.5 * (a + b) for a, b in zip(eig_Kplus(n), eig_Kminus(n)))


def exterior_K_er(n, r):
    """Eqs. 3.19-3.21, exterior branches (r > 1), target normal e_r: the traction of
    S[V] is kVV V, of S[W] is kWW W + kWV V, of S[X] is kXX X."""
    kvv = -2.0 * n * (n + 2) / ((2 * n + 1) * (2 * n + 3)) * r ** (-n - 3)
    if n == 0:
        return kvv, 0.0, 0.0, 0.0
    kww = -(2.0 * n * n + 1) / ((2 * n + 1) * (2 * n - 1)) * r ** (-n - 1)
    kwv = n * (n + 2.0) / (2 * n + 1) * (r ** (-n - 1) - r ** (-n - 3))
    kxx = -(n + 2.0) / (2 * n + 1) * r ** (-n - 2)
    return kvv, kww, kwv, kxx


# ---- harmonic potentials ------------------------------------------------------------------
_ladder_cache = {}


def ladder(p, mmax):
    """Matrices L_i (i = x, y, z) with e_i . V_n^m = sum_{n'm'} L_i[n'm', nm] Y_{n'}^{m'}
    for the modes (n <= p, |m| <= min(n, mmax)) on the left, all modes of degree <= p+1
    on the right (only n' = n+1 is nonzero).  By quadrature projection on a grid that
    integrates the products exactly."""
    key = (p, mmax)
    if key not in _ladder_cache:
        g = sphere_grid(p + 2, 2 * p + 6)
        _m_in, _Yi, Vi, _Wi, _Xi = vsh_at(g["xhat"], p, mmax)
        _m_out, Yo, _Vo, _Wo, _Xo = vsh_at(g["xhat"], p + 1, p + 1)
        wq = g["wnode"]
        L = np.einsum("ok,mki,k->iom", np.conj(Yo), Vi, wq)    # (3, M_out, M_in)
        _ladder_cache[key] = L
    return _ladder_cache[key]


def potential_derivs(c, p, mmax, d):
    """Psi = sum c_nm Phi_nm over modes (n <= p, |m| <= min(n, mmax)) at points d
    (K, 3) relative to the source centre (|d| > 0).  c (M, B) complex.
    Returns value (K, B), gradient (K, 3, B), Hessian (K, 3, 3, B), complex."""
    r = np.linalg.norm(d, axis=1)
    xh = d / r[:, None]
    modes_in = mode_list(p, mmax)
    modes_out = mode_list(p + 1, p + 1)
    _mi, Y, V, _W, _X = vsh_at(xh, p, mmax)
    _mo, _Yo, Vo, _Wo, _Xo = vsh_at(xh, p + 1, p + 1)
    n_in = np.array([n for n, _ in modes_in])
    n_out = np.array([n for n, _ in modes_out])
    f0 = r[None, :] ** (-n_in[:, None] - 1.0)                    # (M, K)
    f1 = r[None, :] ** (-n_in[:, None] - 2.0)
    val = np.einsum("mk,mb->kb", Y * f0, c)
    grad = np.einsum("mki,mk,mb->kib", V, f1, c)
    L = ladder(p, mmax)
    cd = np.einsum("iom,mb->iob", L, c)                          # derivative potentials
    fo = r[None, :] ** (-n_out[:, None] - 2.0)
    hess = np.einsum("okj,ok,iob->kijb", Vo, fo, cd)
    return val, grad, hess


def single_layer_flow_complex(coef, p, mmax, d):
    """Exterior flow of S applied to sum coef Z (V, W, X families, coef (3, M, B)) on
    the unit sphere, at points d (K, 3) relative to its centre, through the harmonic
    potentials of the module header.  Returns (u (K, 3, B), grad u (K, 3, 3, B) with
    G[k, i, j] = d_j u_i, p (K, B)), complex (the flow of each complex mode)."""
    modes = mode_list(p, mmax)
    n = np.array([nn for nn, _ in modes], dtype=np.float64)
    sV = n / ((2 * n + 1) * (2 * n + 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        sW = np.where(n >= 1, (n + 1) / ((2 * n + 1) * (2 * n - 1)), 0.0)
    sWV = n / (2 * (2 * n + 1))
    sX = np.where(n >= 1, 1.0 / (2 * n + 1), 0.0)
    cV, cW, cX = coef[0], coef[1], coef[2]
    A = sV[:, None] * cV + sWV[:, None] * cW
    Bc = (sW - sWV)[:, None] * cW
    C = ((2 * n + 1) * sW)[:, None] * cW
    Xc = sX[:, None] * cX
    Pc = n[:, None] * cW
    _a, gA, hA = potential_derivs(A, p, mmax, d)
    _b, gB, hB = potential_derivs(Bc, p, mmax, d)
    vC, gC, _c = potential_derivs(C, p, mmax, d)
    _x, gX, hX = potential_derivs(Xc, p, mmax, d)
    vP, _gp, _hp = potential_derivs(Pc, p, mmax, d)
    r2 = np.einsum("ki,ki->k", d, d)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    u = gA + r2[:, None, None] * gB + d[:, :, None] * vC[:, None, :]
    u = u + np.einsum("ikl,xk,xlb->xib", eps, d, gX)
    G = hA + r2[:, None, None, None] * hB
    G = G + 2.0 * np.einsum("xj,xib->xijb", d, gB)
    G = G + np.eye(3)[None, :, :, None] * vC[:, None, None, :]
    G = G + np.einsum("xi,xjb->xijb", d, gC)
    G = G + np.einsum("ijl,xlb->xijb", eps, gX)
    G = G + np.einsum("ikl,xk,xljb->xijb", eps, d, hX)
    return u, G, vP


def single_layer_flow(coef, p, mmax, d):
    """single_layer_flow_complex for the coefficients of a real density: real parts."""
    u, G, pr = single_layer_flow_complex(coef, p, mmax, d)
    return u.real, G.real, pr.real


def single_layer_traction(coef, p, mmax, d, nrm):
    """Traction (grad u + grad u^T - p I) n of the exterior flow of S[sigma] at points d
    (relative to the source centre) with unit normals nrm (K, 3).  Returns (K, 3, B)."""
    _u, G, pr = single_layer_flow(coef, p, mmax, d)
    t = np.einsum("xijb,xj->xib", G, nrm) + np.einsum("xjib,xj->xib", G, nrm)
    return t - nrm[:, :, None] * pr[:, None, :]


# ---- the operators on n_b spheres ---------------------------------------------------------
class TractionOps:
    """K and the second-kind operator of Eq. 5.8 on the discretisation of `geom`."""

    def __init__(self, geom):
        self.g = geom
        self.ops = Operators(geom)

    def eigen_Kpv(self):
        lam = np.zeros((3, len(self.ops.vsh.modes)))
        for i, (n, _m) in enumerate(self.ops.vsh.modes):
            lam[:, i] = eig_Kpv(n)
        return lam

    def self_part(self, mu):
        mu = np.asarray(mu, dtype=np.float64).reshape(self.g.N, 3)
        lam = self.eigen_Kpv()
        out = np.zeros_like(mu)
        for k in range(self.g.nb):
            sl = self.g.sphere_nodes(k)
            out[sl] = self.ops.vsh.inverse(lam * self.ops.vsh.forward(mu[sl]))
        return out

    def near_part(self, mu):
        g = self.g
        mu = np.asarray(mu, dtype=np.float64).reshape(g.N, 3)
        out = np.zeros((g.N, 3))
        for t in range(g.nb):
            rows = g.sphere_nodes(t)
            for s in np.nonzero(g.near[t])[0]:
                coef = self.ops.vsh.forward(mu[g.sphere_nodes(s)])[..., None]
                # traction is scale invariant: evaluate in units of the source radius
                d = (g.nodes[rows] - g.centres[s][None, :]) / g.radii[s]
                out[rows] += single_layer_traction(coef, g.p, g.mmax, d, g.xhat[rows])[..., 0]
        return out

    def far_part(self, mu):
        g = self.g
        mu = np.asarray(mu, dtype=np.float64).reshape(g.N, 3)
        q = mu * g.w[:, None]
        out = np.zeros((g.N, 3))
        for t in range(g.nb):
            rows = g.sphere_nodes(t)
            src = [s for s in range(g.nb) if s != t and not g.near[t, s]]
            if not src:
                continue
            idx = np.concatenate([np.arange(s * g.P, (s + 1) * g.P) for s in src])
            out[rows] = traction_sum(g.nodes[rows], g.xhat[rows], g.nodes[idx], q[idx])
        return out

    def apply_K(self, mu):
        """sum_k K_k[mu] at every node (principal value on the own sphere)."""
        return self.self_part(mu) + self.near_part(mu) + self.far_part(mu)

    def L_part(self, mu):
        """L_k[mu] on the nodes of sphere k: int_k mu + (int_k (y - c_k) x mu) x (x - c_k)."""
        g = self.g
        mu = np.asarray(mu, dtype=np.float64).reshape(g.N, 3)
        F, T = self.ops.moments(mu)
        F, T = F[..., 0], T[..., 0]
        k = g.sphere_of
        return F[k] + np.cross(T[k], g.nodes - g.centres[k])

    def apply_KL_BIE(self, mu):
        """(1/2 I + sum_k (K_k + L_k))[mu], the left side of Eq. 5.8."""
        mu = np.asarray(mu, dtype=np.float64).reshape(self.g.N, 3)
        return 0.5 * mu + self.apply_K(mu) + self.L_part(mu)


def force_density(geom, F, T):
    """rho of Eq. 5.7 on every node: F_k/(4 pi a^2) + 3/(8 pi a^4) T_k x (x - c_k) on a
    sphere of radius a (area 4 pi a^2, int (x-c) x (T x (x-c)) = 8 pi a^4 / 3 T)."""
    k = geom.sphere_of
    a = geom.radii[k][:, None]
    return (np.asarray(F, float)[k] / (4.0 * math.pi * a ** 2)
            + 3.0 / (8.0 * math.pi * a ** 4) * np.cross(np.asarray(T, float)[k], geom.nodes - geom.centres[k]))


def rigid_motion(geom, u):
    """(v_k, omega_k) from the velocity u on the nodes: (1/(4 pi a^2)) int u and
    3/(8 pi a^4) int (x - c) x u (the rigid motion of u on a sphere of radius a)."""
    wu = u * geom.w[:, None]
    a = geom.radii[:, None]
    v = wu.reshape(geom.nb, geom.P, 3).sum(axis=1) / (4.0 * math.pi * a ** 2)
    om = np.cross(geom.nodes - geom.centres[geom.sphere_of], wu).reshape(geom.nb, geom.P, 3).sum(axis=1)
    return v, om * 3.0 / (8.0 * math.pi * a ** 4)


def solve_mobility_traction(geom, F, T, tol=1e-11, restart=100, max_iter=1000):
    """Problem 2 by Eqs. 5.7-5.8.  Returns (v, omega, mu, info)."""
    to = TractionOps(geom)
    rho = force_density(geom, F, T)
    b = -(0.5 * rho + to.apply_K(rho)).reshape(-1)
    mu, info = gmres(lambda z: to.apply_KL_BIE(z).reshape(-1), b, tol=tol, restart=restart, max_iter=max_iter)
    mu = mu.reshape(geom.N, 3)
    u = to.ops.apply("S", mu + rho)
    v, om = rigid_motion(geom, u)
    return v, om, mu, info
