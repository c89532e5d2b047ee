"""Scalar and vector spherical harmonics, written from their definitions (Section 2.1).

Test infrastructure only (see ``oracle/__init__.py``).

* Y_n^m of Definition 2.1 / Eq. 2.1: orthonormal, no Condon-Shortley phase,
  Y_n^{-m} = conj(Y_n^m).
* V, W, X of Definition 2.2 / Eqs. 2.4-2.6, evaluated as Cartesian vectors.
* The dense vector transform: forward = quadrature projection onto V, W, X with the
  grid of Eq. 4.4 (the coefficients of Eq. 2.12 / 2.13-2.14); inverse = synthesis.

Parity: pinned by tests/test_oracle_harmonics.py (against scipy's associated Legendre
functions up to the (-1)^m phase, discrete orthonormality, Cartesian identities of the
degree-one harmonics, round trip on band-limited fields).
"""
import math

import numpy as np
from numpy.polynomial import legendre as npleg


def norm_const(n, m):
    """sqrt((2n+1)/(4 pi) * (n-|m|)!/(n+|m|)!) of Eq. 2.1."""
    m = abs(m)
    return math.sqrt((2 * n + 1) / (4.0 * math.pi) * (math.factorial(n - m) / math.factorial(n + m)))


def _dm_legendre(n, m, t):
    """d^m/dt^m P_n(t) through the Legendre-series derivative (numpy.polynomial)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    if m > 0:
        c = npleg.legder(c, m)
    return npleg.legval(t, c)


def pbar(n, m, t):
    """Normalised P_n^|m|(t) = N_nm (1-t^2)^{m/2} d^m P_n/dt^m (no (-1)^m factor)."""
    m = abs(m)
    t = np.asarray(t, dtype=np.float64)
    if m > n:
        return np.zeros_like(t)
    return norm_const(n, m) * (1.0 - t * t) ** (m / 2.0) * _dm_legendre(n, m, t)


def pbar_dtheta(n, m, t):
    """d/dtheta of pbar(n, m, cos theta), from the product rule on the definition:
    N [ m t (1-t^2)^{(m-1)/2} P^{(m)} - (1-t^2)^{(m+1)/2} P^{(m+1)} ]  (finite at the poles)."""
    m = abs(m)
    t = np.asarray(t, dtype=np.float64)
    if m > n:
        return np.zeros_like(t)
    s2 = 1.0 - t * t
    out = -(s2 ** ((m + 1) / 2.0)) * _dm_legendre(n, m + 1, t)
    if m > 0:
        out = out + m * t * s2 ** ((m - 1) / 2.0) * _dm_legendre(n, m, t)
    return norm_const(n, m) * out


def pbar_over_sin(n, m, t):
    """pbar(n, m, t) / sin(theta) for m >= 1: N (1-t^2)^{(m-1)/2} P^{(m)}  (finite at poles).
    Returns 0 for m = 0 (it is only ever multiplied by m)."""
    m = abs(m)
    t = np.asarray(t, dtype=np.float64)
    if m == 0 or m > n:
        return np.zeros_like(t)
    return norm_const(n, m) * (1.0 - t * t) ** ((m - 1) / 2.0) * _dm_legendre(n, m, t)


def spherical_frame(xhat):
    """Unit vectors e_r, e_theta, e_phi at unit directions xhat (..., 3), with
    theta = acos(z) and phi = atan2(y, x) (phi = 0 on the axis)."""
    x, y, z = xhat[..., 0], xhat[..., 1], xhat[..., 2]
    z = np.clip(z, -1.0, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.arctan2(y, x)
    cp, sp = np.cos(phi), np.sin(phi)
    er = np.stack([st * cp, st * sp, z], axis=-1)
    eth = np.stack([z * cp, z * sp, -st], axis=-1)
    eph = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    return z, phi, er, eth, eph


def mode_list(p, mmax):
    """(n, m) pairs with 0 <= n <= p and |m| <= min(n, mmax)."""
    return [(n, m) for n in range(p + 1) for m in range(-min(n, mmax), min(n, mmax) + 1)]


def vsh_at(xhat, p, mmax):
    """Evaluate Y, V, W, X (Eqs. 2.1, 2.4-2.6) at unit directions xhat (K, 3).

    Returns (modes, Y, V, W, X): Y (M, K) complex, V/W/X (M, K, 3) complex Cartesian,
    where M = len(modes).  grad_gamma Y = dY/dtheta e_theta + (1/sin theta) dY/dphi e_phi.
    """
    t, phi, er, eth, eph = spherical_frame(np.asarray(xhat, dtype=np.float64))
    modes = mode_list(p, mmax)
    K = t.shape[0]
    M = len(modes)
    Y = np.zeros((M, K), dtype=np.complex128)
    V = np.zeros((M, K, 3), dtype=np.complex128)
    W = np.zeros((M, K, 3), dtype=np.complex128)
    X = np.zeros((M, K, 3), dtype=np.complex128)
    for i, (n, m) in enumerate(modes):
        e = np.exp(1j * m * phi)
        y = pbar(n, m, t) * e
        dth = pbar_dtheta(n, m, t) * e
        dph_over_sin = 1j * m * pbar_over_sin(n, m, t) * e
        grad = dth[:, None] * eth + dph_over_sin[:, None] * eph
        Y[i] = y
        V[i] = grad - (n + 1) * y[:, None] * er
        W[i] = grad + n * y[:, None] * er
        X[i] = np.cross(er, grad)
    return modes, Y, V, W, X


def vsh_norms(n):
    """Squared L2 norms of V_n^m, W_n^m, X_n^m on the unit sphere:
    (n+1)(2n+1), n(2n+1), n(n+1)  (|grad Y|^2 integrates to n(n+1), |Y|^2 to 1)."""
    return (n + 1) * (2 * n + 1), n * (2 * n + 1), n * (n + 1)


class DenseVSH:
    """Dense forward/inverse vector transform on one sphere's grid (Section 2.1).

    Forward: coefficient of Z_n^m = sum_nodes w mu . conj(Z_n^m) / ||Z_n^m||^2.
    Inverse: mu = sum coef_Z Z_n^m (real part for real fields).
    Coefficient arrays have shape (3, M, ...) for families (V, W, X); W and X entries at
    n = 0 are identically zero.
    """

    def __init__(self, grid, p, mmax):
        self.p = p
        self.mmax = mmax
        self.modes, self.Y, self.V, self.W, self.X = vsh_at(grid["xhat"], p, mmax)
        self.w = grid["wnode"]
        M = len(self.modes)
        nrm = np.zeros((3, M))
        for i, (n, _m) in enumerate(self.modes):
            nrm[:, i] = vsh_norms(n)
        self.norms = nrm
        self.Z = np.stack([self.V, self.W, self.X])            # (3, M, P, 3)

    def forward(self, mu):
        """mu (P, 3[, B]) real -> coefficients (3, M[, B]) complex."""
        mu = np.asarray(mu, dtype=np.float64)
        batch = mu.ndim == 3
        if not batch:
            mu = mu[..., None]
        proj = np.einsum("fmpc,pcb->fmb", np.conj(self.Z), mu * self.w[:, None, None])
        with np.errstate(divide="ignore", invalid="ignore"):
            coef = np.where(self.norms[..., None] > 0, proj / np.where(self.norms > 0, self.norms, 1.0)[..., None], 0.0)
        return coef if batch else coef[..., 0]

    def inverse(self, coef):
        """coefficients (3, M[, B]) -> real field (P, 3[, B])."""
        coef = np.asarray(coef)
        batch = coef.ndim == 3
        if not batch:
            coef = coef[..., None]
        out = np.einsum("fmpc,fmb->pcb", self.Z, coef).real
        return out if batch else out[..., 0]
