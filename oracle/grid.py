"""Quadrature grid on a unit sphere (Section 4, Eqs. 4.2-4.4).

Test infrastructure only (see ``oracle/__init__.py``).

Parity: pinned by tests/test_oracle_grid.py (total area 4 pi, exact integration of
low-degree polynomials, nodes on the unit sphere).
"""
import math

import numpy as np


def default_nphi(p):
    """Azimuthal node count.  Eq. 4.2 prints 2p+2, the unknown count of Section 6
    (N = 6p(p+1) n_b) implies 2p; the default here is 2p."""
    return 2 * p


def mmax_for(p, n_phi):
    """Largest azimuthal order resolved without aliasing on an n_phi-point uniform grid:
    modes e^{i m phi} with |m| < n_phi / 2 are distinct and integrate exactly."""
    return min(p, n_phi // 2 - 1)


def sphere_grid(p, n_phi=None):
    """Gauss-Legendre x uniform grid of Eq. 4.2 on the unit sphere.

    Returns a dict with
      t      (p+1,)  GL nodes t_j = cos(theta_j), sorted descending (theta ascending)
      lam    (p+1,)  GL weights lambda_j
      theta  (p+1,)
      phi    (n_phi,) phi_l = 2 pi l / n_phi
      w      (p+1,)  smooth-quadrature weight per node of latitude j, Eq. 4.4 with the
                     unit-sphere area element: w_j = 2 pi lambda_j / n_phi
      xhat   (P, 3)  unit position (= outward normal) of node g = j * n_phi + l
      wnode  (P,)    weight of node g
    """
    if n_phi is None:
        n_phi = default_nphi(p)
    t, lam = np.polynomial.legendre.leggauss(p + 1)
    order = np.argsort(-t)
    t = t[order]
    lam = lam[order]
    theta = np.arccos(t)
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    w = 2.0 * math.pi * lam / n_phi
    st = np.sqrt(1.0 - t * t)
    xhat = np.empty((p + 1, n_phi, 3))
    xhat[:, :, 0] = st[:, None] * np.cos(phi)[None, :]
    xhat[:, :, 1] = st[:, None] * np.sin(phi)[None, :]
    xhat[:, :, 2] = t[:, None] * np.ones(n_phi)[None, :]
    wnode = np.repeat(w, n_phi)
    return dict(p=p, n_phi=n_phi, t=t, lam=lam, theta=theta, phi=phi, w=w,
                xhat=xhat.reshape(-1, 3), wnode=wnode)


class Geometry:
    """n_b spheres with the grid of Eq. 4.2 on each (unit radius unless ``radii`` given).

    Node order: g = k * P + j * n_phi + l (sphere k, latitude j, longitude l).
    ``near_gap`` is the separation threshold d* of Eq. 4.5 written as a surface gap:
    spheres s != t are "near" when |c_t - c_s| - 2 < d*.  With radii a_k (polydisperse
    suspensions, Section 6), node x = c_k + a_k xhat, weight a_k^2 w, and the gap is
    measured in units of the source radius: near[t, s] when
    |c_t - c_s| - a_t - a_s < d* a_s (the far quadrature of sphere s resolves distances
    on the scale of its own node spacing, a_s / p).
    """

    def __init__(self, centres, p, n_phi=None, near_gap=1.0, radii=None):
        self.centres = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        self.nb = self.centres.shape[0]
        self.grid = sphere_grid(p, n_phi)
        self.p = p
        self.n_phi = self.grid["n_phi"]
        self.mmax = mmax_for(p, self.n_phi)
        self.P = (p + 1) * self.n_phi
        self.N = self.nb * self.P
        self.near_gap = float(near_gap)
        self.radii = np.ones(self.nb) if radii is None else np.asarray(radii, dtype=np.float64).reshape(-1)
        self.unit = bool(np.all(self.radii == 1.0))
        a = self.radii
        xh = self.grid["xhat"]
        self.xhat = np.tile(xh, (self.nb, 1))                     # outward normals
        self.nodes = (self.centres[:, None, :] + a[:, None, None] * xh[None, :, :]).reshape(-1, 3)
        self.w = (a[:, None] ** 2 * self.grid["wnode"][None, :]).reshape(-1)
        self.sphere_of = np.repeat(np.arange(self.nb), self.P)
        d = np.linalg.norm(self.centres[:, None, :] - self.centres[None, :, :], axis=-1)
        self.centre_dist = d
        near = (d - a[:, None] - a[None, :] < self.near_gap * a[None, :])
        np.fill_diagonal(near, False)
        self.near = near                                          # near[t, s]

    def sphere_nodes(self, k):
        return slice(k * self.P, (k + 1) * self.P)
