"""Pins for oracle/harmonics.py (Definition 2.1-2.2, Eqs. 2.1, 2.4-2.6): scipy's
associated Legendre functions, finite differences, discrete orthogonality and the
Cartesian form of the degree-0/1 harmonics."""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle.grid import mmax_for, sphere_grid
from oracle.harmonics import DenseVSH, pbar, pbar_dtheta, pbar_over_sin, vsh_at


def _real_coeffs(vsh, rng):
    """Random coefficients of a real band-limited field (c_{n,-m} = conj c_{n,m})."""
    M = len(vsh.modes)
    c = rng.standard_normal((3, M)) + 1j * rng.standard_normal((3, M))
    idx = {nm: i for i, nm in enumerate(vsh.modes)}
    for (n, m), i in idx.items():
        if m < 0:
            c[:, i] = np.conj(c[:, idx[(n, -m)]])
        elif m == 0:
            c[:, i] = c[:, i].real
        if n == 0:
            c[1:, i] = 0.0
    return c


@pytest.mark.parametrize("n,m", [(0, 0), (1, 0), (1, 1), (3, 2), (7, 5), (12, 11), (16, 3)])
def test_pbar_matches_scipy(n, m):
    t = np.linspace(-0.99, 0.99, 37)
    N = math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - m) / math.factorial(n + m))
    ref = (-1) ** m * N * sp.lpmv(m, n, t)        # scipy includes the Condon-Shortley phase
    assert np.allclose(pbar(n, m, t), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n,m", [(2, 1), (5, 3), (9, 0)])
def test_y_matches_scipy_sph_harm(n, m):
    th = np.linspace(0.1, 3.0, 11)
    ph = np.linspace(0.2, 6.0, 11)
    xh = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    modes, Y, *_ = vsh_at(xh, n, n)
    i = modes.index((n, m))
    ref = sp.sph_harm_y(n, m, th, ph) * (-1) ** m
    assert np.allclose(Y[i], ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n,m", [(1, 0), (2, 1), (6, 4), (10, 10), (13, 2)])
def test_dtheta_and_over_sin(n, m):
    th = np.linspace(0.05, math.pi - 0.05, 29)
    h = 1e-5
    fd = (pbar(n, m, np.cos(th + h)) - pbar(n, m, np.cos(th - h))) / (2 * h)
    assert np.allclose(pbar_dtheta(n, m, np.cos(th)), fd, rtol=1e-7, atol=1e-7)
    if m > 0:
        assert np.allclose(pbar_over_sin(n, m, np.cos(th)) * np.sin(th), pbar(n, m, np.cos(th)), atol=1e-13)


@pytest.mark.parametrize("p,n_phi", [(4, 8), (8, 16), (8, 18), (12, 24)])
def test_discrete_gram_is_diagonal(p, n_phi):
    g = sphere_grid(p, n_phi)
    v = DenseVSH(g, p, mmax_for(p, n_phi))
    G = np.einsum("fmpc,gkpc,p->fmgk", np.conj(v.Z), v.Z, v.w)
    D = np.zeros_like(G)
    for f in range(3):
        for i in range(len(v.modes)):
            D[f, i, f, i] = v.norms[f, i]
    assert np.abs(G - D).max() < 1e-11


@pytest.mark.parametrize("p,n_phi", [(4, 8), (8, 16), (12, 24), (8, 18)])
def test_round_trip_and_idempotence(p, n_phi):
    g = sphere_grid(p, n_phi)
    v = DenseVSH(g, p, mmax_for(p, n_phi))
    rng = np.random.default_rng(1)
    c = _real_coeffs(v, rng)
    f = v.inverse(c)
    assert np.abs(v.forward(f) - c).max() < 1e-12
    # grid -> coefficients -> grid is a projection
    mu = rng.standard_normal((g["xhat"].shape[0], 3))
    f1 = v.inverse(v.forward(mu))
    assert np.abs(v.inverse(v.forward(f1)) - f1).max() < 1e-12


def test_degree_one_cartesian_identities():
    p = 6
    g = sphere_grid(p)
    v = DenseVSH(g, p, mmax_for(p, g["n_phi"]))
    xh = g["xhat"]
    i10 = v.modes.index((1, 0))
    i00 = v.modes.index((0, 0))
    # constant e_z = sqrt(4pi/3) W_1^0
    c = v.forward(np.tile([0.0, 0.0, 1.0], (xh.shape[0], 1)))
    expect = np.zeros_like(c)
    expect[1, i10] = math.sqrt(4 * math.pi / 3)
    assert np.abs(c - expect).max() < 1e-13
    # rigid rotation e_z x xhat = -sqrt(4pi/3) X_1^0
    c = v.forward(np.cross([0.0, 0.0, 1.0], xh))
    expect = np.zeros_like(c)
    expect[2, i10] = -math.sqrt(4 * math.pi / 3)
    assert np.abs(c - expect).max() < 1e-13
    # radial xhat = -sqrt(4pi) V_0^0
    c = v.forward(xh)
    expect = np.zeros_like(c)
    expect[0, i00] = -math.sqrt(4 * math.pi)
    assert np.abs(c - expect).max() < 1e-13
    # V_1[a] = a - 3 (a.x) x is a pure V_1 field (zero W, X coefficients)
    a = np.array([0.3, -1.2, 0.7])
    c = v.forward(a[None, :] - 3 * (xh @ a)[:, None] * xh)
    mask = np.array([n == 1 for (n, m) in v.modes])
    assert np.abs(c[1:]).max() < 1e-13 and np.abs(c[0][~mask]).max() < 1e-13


def test_pole_values_are_consistent():
    # the harmonics are continuous vector fields: at the north pole the value does not
    # depend on the azimuth used to build the frame
    xh = np.array([[0.0, 0.0, 1.0]])
    modes, Y, V, W, X = vsh_at(xh, 5, 5)
    eps = 1e-7
    xe = np.array([[eps * math.cos(0.7), eps * math.sin(0.7), math.sqrt(1 - eps * eps)]])
    _, _, V2, W2, X2 = vsh_at(xe, 5, 5)
    assert np.abs(V - V2).max() < 1e-5 and np.abs(W - W2).max() < 1e-5 and np.abs(X - X2).max() < 1e-5
