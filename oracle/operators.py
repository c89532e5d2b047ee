"""The discretised boundary integral operators on n_b unit spheres (Sections 4.1, 4.3, 5).

Test infrastructure only (see ``oracle/__init__.py``).

For a combination a_S S + a_D D of the Stokes layer potentials, the value at a node x on
sphere t is the sum of three parts (Section 4.3):

* self (s = t): singular integral, applied spectrally (Section 4.1, "singular and
  near-singular integrands", Eqs. 4.6-4.7): project the density of sphere t onto V, W, X,
  multiply by the eigenvalues of Theorem 2 (D taken as the principal value
  D_pv = D_+ - 1/2), synthesise on the grid;
* near (s != t, surface gap |c_t - c_s| - 2 < d*, the separation test of Eq. 4.5):
  project the density of sphere s and evaluate the exterior formulas 3.6-3.11 at x;
* far (all other s): the smooth quadrature of Eq. 4.4, i.e. the direct sum of the kernel
  times w * density over the nodes of s.

Second-kind equations (Section 5):
  SD_BIE  1/2 mu + sum_k (S_k + D_k)[mu]                 (Eqs. 5.4, 5.17)
  DN_BIE  1/2 psi + sum_k (D_k + N_k)[psi]               (Eq. 5.19)
  MOBILITY the bordered form of Eq. 5.17 with Eq. 5.15's force and torque rows set to
           the applied (F_k, T_k): unknowns (mu, v_k, omega_k).
The identity term acts on the grid values; N_k is the Stokeslet-plus-rotlet completion
flow at the centre with strength int psi and torque int (y - c_k) x psi.

Parity: the pieces are pinned individually (tests/test_oracle_*.py); a multi-sphere
matvec as a whole has no closed form beyond the one- and two-sphere pins (drag, far
field asymptotics, exterior-solution reproduction), see tests/test_oracle_solve.py.
"""
import math

import numpy as np

from . import kernels, spectra
from .harmonics import DenseVSH, vsh_at

OPS = {
    # name: (a_S, a_D, identity coefficient, completion flow)
    "S": (1.0, 0.0, 0.0, False),
    "D": (0.0, 1.0, 0.0, False),
    "SD_BIE": (1.0, 1.0, 0.5, False),
    "DN_BIE": (0.0, 1.0, 0.5, True),
}


class Operators:
    def __init__(self, geom):
        self.g = geom
        self.vsh = DenseVSH(geom.grid, geom.p, geom.mmax)

    # ---- helpers -------------------------------------------------------------------
    def _as_batch(self, mu):
        mu = np.asarray(mu, dtype=np.float64)
        if mu.ndim == 2:
            return mu[..., None], False
        return mu, True

    def eigen_scale(self, a_s, a_d):
        """(3, M) multipliers a_S lambda_S + a_D lambda_Dpv per family and mode."""
        lam = np.zeros((3, len(self.vsh.modes)))
        for i, (n, _m) in enumerate(self.vsh.modes):
            s = spectra.eig_S(n)
            d = spectra.eig_Dpv(n)
            for f in range(3):
                lam[f, i] = a_s * s[f] + a_d * d[f]
        return lam

    def coefficients(self, mu, k):
        """VSH coefficients (3, M, B) of the density on sphere k."""
        return self.vsh.forward(mu[self.g.sphere_nodes(k)])

    # ---- the three parts -----------------------------------------------------------
    def self_part(self, mu, a_s, a_d, spheres=None):
        """Self term on every sphere (or only on `spheres`; other entries stay 0).  On a
        sphere of radius a the single layer scales with a (its kernel is homogeneous of
        degree -1 and the area element of degree 2), the double layer not at all."""
        mu, batch = self._as_batch(mu)
        out = np.zeros_like(mu)
        for k in (range(self.g.nb) if spheres is None else spheres):
            lam = self.eigen_scale(a_s * self.g.radii[k], a_d)[..., None]
            sl = self.g.sphere_nodes(k)
            out[sl] = self.vsh.inverse(lam * self.vsh.forward(mu[sl]))
        return out if batch else out[..., 0]

    def _targets(self, targets):
        if targets is None:
            return np.arange(self.g.N)
        return np.asarray(targets, dtype=np.int64)

    def far_part(self, mu, a_s, a_d, targets=None):
        mu, batch = self._as_batch(mu)
        g = self.g
        tg = self._targets(targets)
        q = mu * g.w[:, None, None]
        out = np.zeros((tg.size, 3, mu.shape[2]))
        tsph = g.sphere_of[tg]
        for t in np.unique(tsph):
            rows = np.nonzero(tsph == t)[0]
            allowed = np.array([s for s in range(g.nb) if s != t and not g.near[t, s]], dtype=np.int64)
            if allowed.size == 0:
                continue
            src = (allowed[:, None] * g.P + np.arange(g.P)[None, :]).ravel()
            out[rows] = kernels.direct_sum(g.nodes[tg[rows]], g.nodes[src], g.xhat[src], q[src], a_s, a_d)
        return out if batch else out[..., 0]

    def near_field_from(self, coef, centre, x, a_s, a_d, radius=1.0):
        """Exterior series (Eqs. 3.6-3.11) of the layer potential a_S S + a_D D of a
        density with VSH coefficients coef (3, M, B) on the sphere of radius `radius`
        at `centre`, evaluated at points x (K, 3) outside it (in units of the radius,
        the single layer scaled by it)."""
        a_s = a_s * radius
        d = (x - centre[None, :]) / radius
        r = np.linalg.norm(d, axis=1)
        modes, _Y, V, W, X = vsh_at(d / r[:, None], self.g.p, self.g.mmax)
        out = np.zeros((x.shape[0], 3, coef.shape[2]), dtype=np.complex128)
        for i, (n, _m) in enumerate(modes):
            fs = spectra.exterior_S(n, r)
            fd = spectra.exterior_D(n, r)
            fvv, fww, fwv, fxx = [np.broadcast_to(a_s * np.asarray(a) + a_d * np.asarray(b), r.shape)
                                  for a, b in zip(fs, fd)]
            cv, cw, cx = coef[0, i], coef[1, i], coef[2, i]              # (B,)
            out += V[i][:, :, None] * (np.asarray(fvv)[:, None, None] * cv[None, None, :]
                                       + np.asarray(fwv)[:, None, None] * cw[None, None, :])
            out += W[i][:, :, None] * (np.asarray(fww)[:, None, None] * cw[None, None, :])
            out += X[i][:, :, None] * (np.asarray(fxx)[:, None, None] * cx[None, None, :])
        return out.real

    def near_part(self, mu, a_s, a_d, targets=None):
        mu, batch = self._as_batch(mu)
        g = self.g
        tg = self._targets(targets)
        out = np.zeros((tg.size, 3, mu.shape[2]))
        tsph = g.sphere_of[tg]
        cache = {}
        for t in np.unique(tsph):
            rows = np.nonzero(tsph == t)[0]
            for s in np.nonzero(g.near[t])[0]:
                if s not in cache:
                    cache[s] = self.coefficients(mu, s)
                out[rows] += self.near_field_from(cache[s], g.centres[s], g.nodes[tg[rows]], a_s, a_d, g.radii[s])
        return out if batch else out[..., 0]

    def moments(self, mu):
        """Per sphere: F_k = sum w mu, T_k = sum w (y - c_k) x mu  (quadrature, Eq. 4.4,
        with the actual nodes and weights, so a sphere of radius a carries a^2 and a^3).
        Returns (nb, 3, B), (nb, 3, B)."""
        mu, _ = self._as_batch(mu)
        g = self.g
        wm = mu * g.w[:, None, None]
        F = wm.reshape(g.nb, g.P, 3, -1).sum(axis=1)
        o = (g.nodes - g.centres[g.sphere_of])[:, :, None]
        Tq = np.stack([o[:, 1] * wm[:, 2] - o[:, 2] * wm[:, 1],
                       o[:, 2] * wm[:, 0] - o[:, 0] * wm[:, 2],
                       o[:, 0] * wm[:, 1] - o[:, 1] * wm[:, 0]], axis=1)
        T = Tq.reshape(g.nb, g.P, 3, -1).sum(axis=1)
        return F, T

    def completion_part(self, psi, targets=None):
        """sum_k N_k[psi](x): Stokeslet of strength F_k plus rotlet of torque T_k at c_k."""
        psi, batch = self._as_batch(psi)
        g = self.g
        tg = self._targets(targets)
        F, T = self.moments(psi)
        out = np.zeros((tg.size, 3, psi.shape[2]))
        x = g.nodes[tg]
        for k in range(g.nb):
            out += kernels.stokeslet_rotlet(x, g.centres[k], F[k], T[k])
        return out if batch else out[..., 0]

    # ---- full operators ------------------------------------------------------------
    def apply(self, op, mu, targets=None):
        """Apply the operator `op` (see OPS) to node values mu (N, 3[, B]); returns the
        values at `targets` (default: all nodes)."""
        a_s, a_d, c_i, compl = OPS[op]
        mu_b, batch = self._as_batch(mu)
        tg = self._targets(targets)
        out = self.self_part(mu_b, a_s, a_d, np.unique(self.g.sphere_of[tg]))[tg]
        out = out + c_i * mu_b[tg]
        out += self.near_part(mu_b, a_s, a_d, tg)
        out += self.far_part(mu_b, a_s, a_d, tg)
        if compl:
            out += self.completion_part(mu_b, tg)
        return out if batch else out[..., 0]

    # ---- bordered mobility system (Eqs. 5.14-5.17 with 5.15 set to (F, T)) -----------
    def mobility_size(self):
        return 3 * self.g.N + 6 * self.g.nb

    def apply_mobility(self, xvec):
        """xvec = [mu (N*3); v (nb*3); omega (nb*3)] (flattened, [, B]) ->
        [1/2 mu + sum (S+D) mu - v_i - omega_i x (x - c_i);
         (1/4pi) sum_k w mu;  (3/8pi) sum_k w (y - c_k) x mu]."""
        g = self.g
        xvec = np.asarray(xvec, dtype=np.float64)
        batch = xvec.ndim == 2
        if not batch:
            xvec = xvec[:, None]
        B = xvec.shape[1]
        mu = xvec[:3 * g.N].reshape(g.N, 3, B)
        v = xvec[3 * g.N:3 * g.N + 3 * g.nb].reshape(g.nb, 3, B)
        om = xvec[3 * g.N + 3 * g.nb:].reshape(g.nb, 3, B)
        u = self.apply("SD_BIE", mu)
        k = g.sphere_of
        o = (g.nodes - g.centres[k])[:, :, None]                  # x - c_k
        w_ = om[k]
        rot = np.stack([w_[:, 1] * o[:, 2] - w_[:, 2] * o[:, 1],
                        w_[:, 2] * o[:, 0] - w_[:, 0] * o[:, 2],
                        w_[:, 0] * o[:, 1] - w_[:, 1] * o[:, 0]], axis=1)
        u = u - v[k] - rot
        F, T = self.moments(mu)
        out = np.concatenate([u.reshape(3 * g.N, B), (F / (4 * math.pi)).reshape(3 * g.nb, B),
                              (3.0 * T / (8 * math.pi)).reshape(3 * g.nb, B)], axis=0)
        return out if batch else out[:, 0]
