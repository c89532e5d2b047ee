"""Laplace layer potentials on spheres (Section 3.1, Theorem 1) and the magnetostatic
problem of Problem 3 (Eqs. 5.9-5.13): the definitions the HIP path must reproduce.

Test infrastructure only (see ``oracle/__init__.py``).

* Scalar transform: c_nm = sum_g w_g f(x_g) conj(Y_n^m(x_g)) (orthonormal Y of Eq. 2.1,
  Eq. 4.4 weights), n <= p, |m| <= mmax.
* Single layer S^L[q](x) = int q(y) / (4 pi |x - y|) dS_y, evaluated sphere by sphere as
  the Stokes operators are (Eq. 4.5 separation test):
  - own sphere, exterior limit at the surface: S^L[Y_n^m] = Y_n^m / (2n+1) (Theorem 1);
    its gradient sum c (grad_s Y - (n+1) Y e_r) / (2n+1) = sum c V_n^m / (2n+1)
    (Eq. 3.3 differentiated at r = 1+);
  - near spheres: Eq. 3.3 exterior, c Y r^{-n-1} / (2n+1), and its gradient
    f'(r) Y e_r + (f(r)/r) grad_s Y with f = r^{-n-1} / (2n+1);
  - other spheres: smooth quadrature, kernels 1 / (4 pi r) and -r / (4 pi r^3).
* K^L = normal derivative of S^L at the target: on the own surface its principal value
  -1 / (2(2n+1)) (the exterior derivative of Eq. 3.3 is -(n+1)/(2n+1) = -1/2 + K_pv).
* Problem 3: phi = -H0 . x + S^L[q] (Eq. 5.12); (1/2 I + eta K^L)[q] = eta H0 . n
  (Eq. 5.13), eta = (mu - mu0) / (mu + mu0); H = -grad phi = H0 - grad S^L[q] on the
  fluid side; traction of the Maxwell stress (mu0 = 1) t = (H . n) H - |H|^2 n / 2; the
  force and torque on sphere k are int t and int (x - c_k) x t (Eq. 4.4 quadrature).
  The fluid couples to the field only through these (Section 5), which the mobility
  problem then takes as applied loads.
* Spheres of radius a (geometry with radii: nodes c + a x, weights a^2 w): S^L of a
  sphere of radius a is a times the unit-sphere layer at (x - c)/a (kernel of degree -1
  in length, area element of degree 2), so the own-sphere value carries a, the series
  is evaluated at (x - c)/a with its value times a, and the gradient and K^L are
  scale-free; the quadrature uses the actual nodes and weights; the torque arm is
  x - c = a n.

Parity: pinned by tests/test_oracle_laplace.py (Theorem 1 by brute-force quadrature;
the textbook magnetisable sphere in a uniform field; the gradient against finite
differences of the series; zero net force on an isolated sphere; the far-field
dipole-dipole force between two spheres).
"""
import math

import numpy as np

from .harmonics import mode_list, pbar, pbar_dtheta, pbar_over_sin, spherical_frame


def ylm_at(xhat, p, mmax):
    """modes, Y (M, K), dY/dtheta (M, K), (1/sin) dY/dphi (M, K) at unit directions."""
    t, phi, er, eth, eph = spherical_frame(np.asarray(xhat, dtype=np.float64))
    modes = mode_list(p, mmax)
    Y = np.zeros((len(modes), len(t)), dtype=np.complex128)
    Dt = np.zeros_like(Y)
    Dp = np.zeros_like(Y)
    for i, (n, m) in enumerate(modes):
        e = np.exp(1j * m * phi)
        Y[i] = pbar(n, m, t) * e
        Dt[i] = pbar_dtheta(n, m, t) * e
        Dp[i] = 1j * m * pbar_over_sin(n, m, t) * e
    return modes, Y, Dt, Dp, er, eth, eph


class Laplace:
    def __init__(self, geom):
        self.g = geom
        xh = geom.grid["xhat"]
        self.modes, self.Y, self.Dt, self.Dp, self.er, self.eth, self.eph = ylm_at(xh, geom.p, geom.mmax)
        self.n = np.array([n for (n, _m) in self.modes])

    def coef(self, f_sphere):
        """Scalar transform of one sphere's node values (P,) -> (M,) complex."""
        return np.conj(self.Y) @ (self.g.grid["wnode"] * f_sphere)

    def synth(self, c):
        return (c @ self.Y).real

    # ---- values / gradients at arbitrary exterior points of one source sphere -------
    def series(self, c, centre, x, radius=1.0):
        """S^L of the density with coefficients c on the sphere of the given radius at
        centre: value (K,) and gradient (K, 3) at points x (K, 3) outside it (Eq. 3.3,
        in units of the radius)."""
        d = (x - centre[None, :]) / radius
        r = np.linalg.norm(d, axis=1)
        modes, Y, Dt, Dp, er, eth, eph = ylm_at(d / r[:, None], self.g.p, self.g.mmax)
        n = np.array([nn for (nn, _m) in modes])[:, None]
        f = r[None, :] ** (-n - 1) / (2 * n + 1)
        fp = -(n + 1) * r[None, :] ** (-n - 2) / (2 * n + 1)
        val = (c[:, None] * f * Y).sum(0).real
        gr = (c[:, None] * fp * Y).sum(0).real
        gt = (c[:, None] * (f / r[None, :]) * Dt).sum(0).real
        gp = (c[:, None] * (f / r[None, :]) * Dp).sum(0).real
        grad = gr[:, None] * er + gt[:, None] * eth + gp[:, None] * eph
        return radius * val, grad

    def direct(self, q_sphere, centre, x, radius=1.0):
        """Smooth quadrature of S^L and its gradient from one sphere's nodes (Eq. 4.4 on
        the sphere of the given radius: nodes c + a x, weights a^2 w)."""
        y = centre[None, :] + radius * self.g.grid["xhat"]
        qw = q_sphere * radius ** 2 * self.g.grid["wnode"]
        r = x[:, None, :] - y[None, :, :]
        d = np.linalg.norm(r, axis=2)
        val = (qw[None, :] / d).sum(1) / (4 * math.pi)
        grad = -(qw[None, :, None] * r / d[..., None] ** 3).sum(1) / (4 * math.pi)
        return val, grad

    # ---- operators on the node values of all spheres --------------------------------
    def potential_and_gradient(self, q, self_term=True):
        """S^L[q] and its exterior gradient at every node (self: Theorem 1 and its
        exterior derivative, on the band-limited projection; near: Eq. 3.3; far:
        quadrature).  self_term=False leaves out the own sphere."""
        g = self.g
        q = np.asarray(q, dtype=np.float64).reshape(g.N)
        val = np.zeros(g.N)
        grad = np.zeros((g.N, 3))
        coefs = [self.coef(q[g.sphere_nodes(k)]) for k in range(g.nb)]
        n = self.n
        for t in range(g.nb):
            sl = g.sphere_nodes(t)
            c = coefs[t] if self_term else 0.0 * coefs[t]
            val[sl] = g.radii[t] * self.synth(c / (2 * n + 1))
            # sum c / (2n+1) (grad_s Y - (n+1) Y e_r)
            a = c[:, None] / (2 * n + 1)[:, None]
            gt = (a * self.Dt).sum(0).real
            gp = (a * self.Dp).sum(0).real
            gr = (-(n + 1)[:, None] * a * self.Y).sum(0).real
            grad[sl] = gr[:, None] * self.er + gt[:, None] * self.eth + gp[:, None] * self.eph
            x = g.nodes[sl]
            for s in range(g.nb):
                if s == t:
                    continue
                if g.near[t, s]:
                    v, gd = self.series(coefs[s], g.centres[s], x, g.radii[s])
                else:
                    v, gd = self.direct(q[g.sphere_nodes(s)], g.centres[s], x, g.radii[s])
                val[sl] += v
                grad[sl] += gd
        return val, grad

    def k_operator(self, q):
        """K^L[q] at every node: the normal derivative of S^L, on the own surface its
        principal value -1 / (2(2n+1)) on the band-limited projection (the identity of
        the second-kind equation acts on the grid values, as for the Stokes forms)."""
        g = self.g
        q = np.asarray(q, dtype=np.float64).reshape(g.N)
        _v, grad = self.potential_and_gradient(q, self_term=False)
        out = np.einsum("gi,gi->g", grad, g.xhat)
        for t in range(g.nb):
            sl = g.sphere_nodes(t)
            out[sl] += self.synth(self.coef(q[sl]) * (-0.5 / (2 * self.n + 1)))
        return out

    def magnetic_bie(self, q, eta):
        """(1/2 I + eta K^L)[q] (Eq. 5.13)."""
        return 0.5 * np.asarray(q).reshape(-1) + eta * self.k_operator(q)


def solve_magnetic(geom, H0, eta):
    """Problem 3: q from Eq. 5.13 (dense LU), then the Maxwell-stress force and torque on
    every sphere.  Returns q (N,), F (nb, 3), T (nb, 3), H at the nodes (N, 3)."""
    lap = Laplace(geom)
    H0 = np.asarray(H0, dtype=np.float64)
    N = geom.N
    A = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        A[:, j] = lap.magnetic_bie(e, eta)
    q = np.linalg.solve(A, eta * geom.xhat @ H0)
    _v, grad = lap.potential_and_gradient(q)
    H = H0[None, :] - grad
    nrm = geom.xhat
    Hn = np.einsum("gi,gi->g", H, nrm)
    t = Hn[:, None] * H - 0.5 * np.einsum("gi,gi->g", H, H)[:, None] * nrm
    wt = geom.w[:, None] * t
    F = wt.reshape(geom.nb, geom.P, 3).sum(1)
    arm = geom.nodes - np.repeat(geom.centres, geom.P, axis=0)     # x - c = a n
    T = np.cross(arm, wt).reshape(geom.nb, geom.P, 3).sum(1)
    return q, F, T, H
