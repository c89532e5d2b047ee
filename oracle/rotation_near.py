"""Near-pair evaluation through pole rotation (Section 4.2, Fig. 2): the definitions the
HIP path must reproduce.

Test infrastructure only (see ``oracle/__init__.py``).

For a directed near pair (source s, target t), with d = c_t - c_s:

0. the source density's V, W, X coefficients (forward transform on its grid);
1. density rotation: rotate the frame so that its pole points at c_t.  Q is the rotation
   with Q d = |d| z (Q = R_y(-beta) R_z(-alpha), alpha, beta the azimuth and polar
   angle of d); the rotated field f^R(x) = Q f(Q^T x) has, per degree n and family,
   the coefficients D^n(Q) c with Y_n^m(Q^T x) = sum_m' D^n_m'm Y_n^m'(x) (the vector
   harmonics are built from Y_n^m by rotation-covariant operations, Eqs. 2.4-2.6, so one
   matrix per degree serves the three families);
2. evaluation at the translated grid: the target's grid in the rotated frame sits at
   (0, 0, |d|) + x_jl, so its nodes have fixed (r, theta) per latitude and equispaced
   phi; the exterior series (Eqs. 3.6-3.11) is evaluated there;
3. the samples are transformed forward on the target grid (rotated frame), the
   coefficients rotated back with D^n(Q^T), and (delayed evaluation) summed over all
   near sources of the target before one inverse transform on its own grid.

The result is the projection of the near field onto the band-limited space of the
target sphere (degree <= p, |m| <= mmax), not its pointwise values; the direct method
(operators.near_part) evaluates the series at the nodes themselves.  D^n is computed
here by its definition, a quadrature projection exact for degree n.

Spheres of radii a_s (source) and a_t (target): the steps run in units of the source
radius, where the source is a unit sphere again: the target grid sits at
(0, 0, |d| / a_s) + (a_t / a_s) x_jl (each latitude still at fixed (r, theta)), and the
single layer's series carries the factor a_s (its kernel is homogeneous of degree -1 in
length, the area element of degree 2; the double layer is scale-free).  The angular
steps (rotations, projection on the target grid) do not see the radii.

Parity: pinned by tests/test_oracle_rotation.py (D^n is unitary, D^n(R_z(a)) is the
phase e^{-i m a}, rotated coefficients resynthesise the rotated field; a pair already on
the pole reduces to the projection of the direct series, also for spheres of two radii;
for smooth densities the result converges to the direct series as p grows, also with
radii; scaling a configuration by lam scales the single layer's result by lam and
leaves the double layer's unchanged).
"""
import math

import numpy as np

from . import spectra
from .grid import sphere_grid
from .harmonics import DenseVSH, mode_list, pbar, vsh_at


def rotation_to_pole(d):
    """Q = R_y(-beta) R_z(-alpha) with Q d = |d| z."""
    d = np.asarray(d, dtype=np.float64)
    r = np.linalg.norm(d)
    alpha = math.atan2(d[1], d[0])
    beta = math.acos(max(-1.0, min(1.0, d[2] / r)))
    ca, sa, cb, sb = math.cos(alpha), math.sin(alpha), math.cos(beta), math.sin(beta)
    Rz = np.array([[ca, sa, 0.0], [-sa, ca, 0.0], [0.0, 0.0, 1.0]])      # R_z(-alpha)
    Ry = np.array([[cb, 0.0, -sb], [0.0, 1.0, 0.0], [sb, 0.0, cb]])      # R_y(-beta)
    return Ry @ Rz


def _ylm(n, xhat):
    """Y_n^m(x) for m = -n..n, (2n+1, K) complex (no Condon-Shortley phase)."""
    t = np.clip(xhat[:, 2], -1.0, 1.0)
    phi = np.arctan2(xhat[:, 1], xhat[:, 0])
    out = np.empty((2 * n + 1, xhat.shape[0]), dtype=np.complex128)
    for m in range(-n, n + 1):
        out[m + n] = pbar(n, abs(m), t) * np.exp(1j * m * phi)
    return out


def wigner(n, Q):
    """D^n(Q): Y_n^m(Q^T x) = sum_m' D[m' + n, m + n] Y_n^m'(x), by projection on a grid
    that integrates products of degree-n harmonics exactly."""
    g = sphere_grid(n, 2 * n + 2)
    x = g["xhat"]
    w = g["wnode"]
    Y = _ylm(n, x)                           # (2n+1, K)
    YQ = _ylm(n, x @ Q)                      # Y(Q^T x): rows of x times Q = (Q^T x^T)^T
    return np.conj(Y) @ (w[:, None] * YQ.T)


def full_modes(p):
    return mode_list(p, p)


def expand(coef, p, mmax):
    """Coefficients on mode_list(p, mmax) -> mode_list(p, p) (zeros where |m| > mmax)."""
    src = {nm: i for i, nm in enumerate(mode_list(p, mmax))}
    out = np.zeros((3, len(full_modes(p))), dtype=np.complex128)
    for j, nm in enumerate(full_modes(p)):
        if nm in src:
            out[:, j] = coef[:, src[nm]]
    return out


def truncate(coef_full, p, mmax):
    dst = {nm: i for i, nm in enumerate(full_modes(p))}
    return np.stack([coef_full[:, dst[nm]] for nm in mode_list(p, mmax)], axis=1)


def rotate(coef_full, p, Q):
    """Coefficients (3, full modes) of f -> those of f^R(x) = Q f(Q^T x)."""
    out = np.zeros_like(coef_full)
    for n in range(p + 1):
        sl = slice(n * n, (n + 1) * (n + 1))      # full_modes(p) is ordered n, then m = -n..n
        out[:, sl] = coef_full[:, sl] @ wigner(n, Q).T
    return out


def series_at(coef_full, p, x, a_s, a_d):
    """Exterior series (Eqs. 3.6-3.11) of a_S S + a_D D for coefficients on the full mode
    list of a unit sphere at the origin, at points x (K, 3) outside it."""
    r = np.linalg.norm(x, axis=1)
    modes, _Y, V, W, X = vsh_at(x / r[:, None], p, p)
    out = np.zeros((x.shape[0], 3), dtype=np.complex128)
    for i, (n, _m) in enumerate(modes):
        fs = spectra.exterior_S(n, r)
        fd = spectra.exterior_D(n, r)
        fvv, fww, fwv, fxx = [np.broadcast_to(a_s * np.asarray(a) + a_d * np.asarray(b), r.shape) for a, b in zip(fs, fd)]
        cv, cw, cx = coef_full[0, i], coef_full[1, i], coef_full[2, i]
        out += V[i] * (fvv * cv + fwv * cw)[:, None] + W[i] * (fww * cw)[:, None] + X[i] * (fxx * cx)[:, None]
    return out.real


def pair_coefficients(geom, coef_s, d, a_s, a_d, vsh=None, rad_s=1.0, rad_t=1.0):
    """Stages 1-3 for one directed pair: the target's coefficients (mode_list(p, mmax))
    of the near field of the source density with coefficients coef_s (3, M); rad_s and
    rad_t the radii of the source and target spheres."""
    p, mmax = geom.p, geom.mmax
    vsh = vsh or DenseVSH(geom.grid, p, mmax)
    Q = rotation_to_pole(d)
    cR = rotate(expand(coef_s, p, mmax), p, Q)
    x = np.array([0.0, 0.0, np.linalg.norm(d) / rad_s])[None, :] + (rad_t / rad_s) * geom.grid["xhat"]
    uR = series_at(cR, p, x, a_s * rad_s, a_d)
    uhatR = vsh.forward(uR)
    return truncate(rotate(expand(uhatR, p, mmax), p, Q.T), p, mmax)


def near_part(geom, mu, a_s, a_d):
    """Near correction of every target sphere by pole rotation and delayed evaluation."""
    g = geom
    vsh = DenseVSH(g.grid, g.p, g.mmax)
    mu = np.asarray(mu, dtype=np.float64).reshape(g.N, 3)
    coefs = {}
    out = np.zeros((g.N, 3))
    for t in range(g.nb):
        srcs = np.nonzero(g.near[t])[0]
        if srcs.size == 0:
            continue
        acc = np.zeros((3, len(vsh.modes)), dtype=np.complex128)
        for s in srcs:
            if s not in coefs:
                coefs[s] = vsh.forward(mu[g.sphere_nodes(s)])
            acc += pair_coefficients(g, coefs[s], g.centres[t] - g.centres[s], a_s, a_d, vsh, g.radii[s], g.radii[t])
        out[g.sphere_nodes(t)] = vsh.inverse(acc)
    return out
