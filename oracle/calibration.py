"""Separation threshold of Eq. 4.5 chosen from a requested precision.

Test infrastructure only (see ``oracle/__init__.py``).

Eq. 4.5 treats two spheres as well separated, so that the smooth quadrature of Eq. 4.4 is
used between them, when their distance is at least eta times the larger diameter, and
leaves eta to be fixed from the precision the user asks for.  For unit spheres that is a
surface-gap test g >= d* with d* = 2 eta.  This module measures, with the test of
Section 6 (Fig. 5: a random density on a unit sphere, targets on spherical shells at
given distances from the surface, smooth quadrature against the exact exterior
potentials of Section 3.2), how far from the surface the quadrature reaches a tolerance,
and turns that into d*.

The measurement, for grid order p on n_phi longitudes:

1. densities sigma = sum f V_n^m + g W_n^m + h X_n^m with every coefficient of degree
   n <= p and order |m| <= mmax drawn uniformly from [-1, 1] (real and imaginary parts;
   m = 0 real, W_0 = X_0 = 0; negative orders by conjugate symmetry, so sigma is real):
   the band limit of the discretisation, with a flat spectrum as the hardest case of it;
   the draws are a counter-based SplitMix64 stream (``uniform``);
2. K target directions on the golden-angle spiral, at radius 1 + g;
3. exact values of S[sigma] and D[sigma] there from the exterior branches of
   Eqs. 3.6-3.11;
4. the smooth quadrature sum_nodes w K(x, y) sigma(y) of Eq. 4.4 (the oracle's direct sum);
5. error e(g) = max over the densities, both operators, targets and components of
   |quadrature - exact|, divided by the largest |sigma| over the nodes.

Reading: the error is measured against the density's size rather than the potential's
value on the shell.  In a second-kind matvec the quadrature error of every far pair adds
to 1/2 mu plus the layer potentials, so an operator accurate to tol relative to the
density needs each far pair accurate to that; the potential of a high-degree mode decays
like r^-n-2 and would make a pointwise relative measure demand arbitrarily large gaps.

Gaps are taken from the grid g_k = 2^(k/8) / 64, k = 0 .. 104 (1/64 .. 128).  The search:
a coarse pass down the grid in steps of 8 from the top while e <= tol / 10, then a fine
pass in steps of 1 below the last coarse gap that passed, again while e <= tol / 10.
d* is the last gap that passed; if the top of the grid already fails, d* is infinite
(every pair of spheres is near).

Parity: pinned by tests/test_oracle_calibration.py: at a gap of 100 the error is at
rounding level (exact formulas and quadrature agree), at gaps of 0.3-1 the exact values
equal a brute-force quadrature on a fine grid (so the formulas, not the quadrature under
test, are the reference), the error decays at the rate the quadrature's exactness
predicts, and d* grows as the tolerance shrinks and falls as p grows.
"""
import math

import numpy as np

from . import spectra
from .grid import mmax_for, sphere_grid
from .harmonics import DenseVSH, vsh_at
from .kernels import direct_sum

N_DIRECTIONS = 256
N_DENSITIES = 2
GAP_STEPS = 104          # g_k = 2^(k/8) / 64, k = 0 .. GAP_STEPS
MASK64 = (1 << 64) - 1


def gap_grid(k):
    return 2.0 ** (k / 8.0) / 64.0


def splitmix64(i):
    """Output number i (i >= 0) of SplitMix64 (Steele, Lea and Flood, 2014) started from
    state 0: the state after i + 1 increments of the golden-ratio constant, then the
    generator's two xor-shift-multiply rounds and a final xor-shift."""
    z = ((i + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform(i):
    """Counter-based uniform on [-1, 1): top 53 bits of splitmix64(i)."""
    return (splitmix64(i) >> 11) * (2.0 ** -53) * 2.0 - 1.0


def slots(p, mmax):
    """Coefficient slots (m, n), m = 0..mmax, n = m..p (the order of Fig. 1)."""
    return [(m, n) for m in range(mmax + 1) for n in range(m, p + 1)]


def density_coefficients(p, mmax, d):
    """Coefficients of density d as a dict (family, n, m) -> complex for m >= 0.  Draw
    number ((d * 3 + f) * ncoef + slot) * 2 + {0: real, 1: imaginary}."""
    sl = slots(p, mmax)
    nc = len(sl)
    out = {}
    for f in range(3):
        for i, (m, n) in enumerate(sl):
            base = ((d * 3 + f) * nc + i) * 2
            re, im = uniform(base), uniform(base + 1)
            if m == 0:
                im = 0.0
            if n == 0 and f > 0:
                re = im = 0.0
            out[(f, n, m)] = complex(re, im)
    return out


def directions(K=N_DIRECTIONS):
    """Golden-angle spiral: z_i = 1 - (2i + 1)/K, phi_i = i pi (3 - sqrt 5)."""
    i = np.arange(K, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / K
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


class ShellTest:
    """The densities of one grid and their exact / quadrature potentials on shells."""

    def __init__(self, p, n_phi=None, n_dens=N_DENSITIES, K=N_DIRECTIONS):
        self.grid = sphere_grid(p, n_phi)
        self.p = p
        self.mmax = mmax_for(p, self.grid["n_phi"])
        self.vsh = DenseVSH(self.grid, p, self.mmax)
        self.dirs = directions(K)
        modes = self.vsh.modes
        self.coef = np.zeros((n_dens, 3, len(modes)), dtype=np.complex128)
        for d in range(n_dens):
            c = density_coefficients(p, self.mmax, d)
            for i, (n, m) in enumerate(modes):
                for f in range(3):
                    v = c.get((f, n, abs(m)), 0.0)
                    self.coef[d, f, i] = v if m >= 0 else np.conj(v)
        self.sigma = np.stack([self.vsh.inverse(self.coef[d]) for d in range(n_dens)], axis=-1)  # (P, 3, B)
        self.sigma_max = np.abs(self.sigma).max()
        self._modes, _Y, self._V, self._W, self._X = vsh_at(self.dirs, p, self.mmax)

    def exact(self, R, op):
        """Exterior formulas (Eqs. 3.6-3.11) of op in {'S', 'D'} at radius R: (K, 3, B)."""
        ext = spectra.exterior_S if op == "S" else spectra.exterior_D
        out = np.zeros((self.dirs.shape[0], 3, self.coef.shape[0]), dtype=np.complex128)
        for i, (n, _m) in enumerate(self._modes):
            fvv, fww, fwv, fxx = ext(n, R)
            cv, cw, cx = self.coef[:, 0, i], self.coef[:, 1, i], self.coef[:, 2, i]
            out += ((fvv * cv + fwv * cw)[None, None, :] * self._V[i][:, :, None]
                    + (fww * cw)[None, None, :] * self._W[i][:, :, None]
                    + (fxx * cx)[None, None, :] * self._X[i][:, :, None])
        return out.real

    def quadrature(self, R, op):
        """Smooth quadrature of Eq. 4.4 at radius R: (K, 3, B)."""
        q = self.sigma * self.grid["wnode"][:, None, None]
        a_s, a_d = (1.0, 0.0) if op == "S" else (0.0, 1.0)
        xh = self.grid["xhat"]
        return direct_sum(R * self.dirs, xh, xh, q, a_s, a_d)

    def error(self, gap):
        R = 1.0 + gap
        e = 0.0
        for op in ("S", "D"):
            e = max(e, float(np.abs(self.quadrature(R, op) - self.exact(R, op)).max()))
        return e / self.sigma_max


def calibrated_gap(p, tol, n_phi=None):
    """d*(p, tol): see the module docstring for the density, the error and the search.
    Returns math.inf when even the largest gap of the grid misses tol / 10."""
    st = ShellTest(p, n_phi)
    target = tol / 10.0
    k = GAP_STEPS
    if st.error(gap_grid(k)) > target:
        return math.inf
    while k - 8 >= 0 and st.error(gap_grid(k - 8)) <= target:
        k -= 8
    while k - 1 >= 0 and st.error(gap_grid(k - 1)) <= target:
        k -= 1
    return gap_grid(k)
