"""Pins of the Laplace / magnetostatic oracle (oracle/laplace.py)."""
import math

import numpy as np
import pytest

from oracle import laplace
from oracle.grid import Geometry


def _dirs(rng, k):
    d = rng.standard_normal((k, 3))
    return d / np.linalg.norm(d, axis=1)[:, None]


@pytest.mark.parametrize("n,m", [(0, 0), (1, 1), (2, -1), (3, 2), (5, 0)])
def test_theorem1_single_layer_by_quadrature(n, m):
    # S^L[Y_n^m] at exterior points from a fine-grid quadrature vs Eq. 3.3
    g = Geometry(np.zeros((1, 3)), 30, near_gap=1.0)
    lap = laplace.Laplace(g)
    modes, Y, *_ = laplace.ylm_at(g.grid["xhat"], 30, 29)
    q = Y[modes.index((n, m))]
    x = 2.5 * _dirs(np.random.default_rng(n), 4)
    y = g.grid["xhat"]
    d = np.linalg.norm(x[:, None] - y[None], axis=2)
    brute = (g.grid["wnode"] * q)[None, :] / d
    brute = brute.sum(1) / (4 * math.pi)
    _m, Yx, *_ = laplace.ylm_at(x / 2.5, n, n)
    ref = Yx[_m.index((n, m))] * 2.5 ** (-n - 1) / (2 * n + 1)
    assert np.abs(brute - ref).max() < 1e-12


def test_magnetisable_sphere_in_a_uniform_field():
    # textbook: exterior potential -H0.x + (mu - mu0)/(mu + 2 mu0) (H0.x)/r^3
    mu = 4.0
    eta = (mu - 1.0) / (mu + 1.0)
    H0 = np.array([0.3, -1.0, 0.6])
    g = Geometry(np.zeros((1, 3)), 6, near_gap=1.0)
    q, F, T, H = laplace.solve_magnetic(g, H0, eta)
    lap = laplace.Laplace(g)
    x = np.array([1.3, 2.0, 4.0])[:, None] * _dirs(np.random.default_rng(1), 3)
    val, grad = lap.series(lap.coef(q), np.zeros(3), x)
    beta = (mu - 1.0) / (mu + 2.0)
    r = np.linalg.norm(x, axis=1)
    assert np.abs(val - beta * (x @ H0) / r ** 3).max() < 1e-12
    # surface field: H = H0 - grad S^L[q] equals -grad of the textbook potential
    xs = g.nodes
    ref_grad = beta * (H0[None, :] / 1.0 - 3 * (xs @ H0)[:, None] * xs)   # grad of beta H0.x / r^3 at r = 1
    assert np.abs(H - (H0[None, :] - ref_grad)).max() < 1e-12
    # no net force or torque on an isolated sphere
    assert np.abs(F).max() < 1e-12 and np.abs(T).max() < 1e-12


def test_gradient_against_finite_differences():
    g = Geometry(np.zeros((1, 3)), 6, near_gap=1.0)
    lap = laplace.Laplace(g)
    rng = np.random.default_rng(2)
    c = lap.coef(rng.standard_normal(g.N))
    x = np.array([1.2, 1.7, 3.0])[:, None] * _dirs(rng, 3)
    _v, grad = lap.series(c, np.zeros(3), x)
    h = 1e-5
    fd = np.zeros_like(grad)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd[:, i] = (lap.series(c, np.zeros(3), x + e)[0] - lap.series(c, np.zeros(3), x - e)[0]) / (2 * h)
    assert np.abs(grad - fd).max() < 1e-8 * np.abs(grad).max()


def test_series_matches_quadrature_far_away():
    g = Geometry(np.zeros((1, 3)), 14, near_gap=1.0)
    lap = laplace.Laplace(g)
    rng = np.random.default_rng(3)
    q = lap.synth(np.where(lap.n <= 3, lap.coef(rng.standard_normal(g.N)), 0))
    x = 5.0 * _dirs(rng, 4)
    a = lap.series(lap.coef(q), np.zeros(3), x)
    b = lap.direct(q, np.zeros(3), x)
    assert np.abs(a[0] - b[0]).max() < 1e-13 and np.abs(a[1] - b[1]).max() < 1e-13


def test_two_spheres_attract_as_induced_dipoles():
    # along the field, far apart: the force tends to the dipole-dipole value
    # 3 m^2 / (2 pi d^4) (attractive), m = 4 pi beta H0 the induced moment
    mu = 3.0
    eta, beta = (mu - 1) / (mu + 1), (mu - 1) / (mu + 2)
    H0 = np.array([0.0, 0.0, 1.0])
    errs = []
    for d in (6.0, 12.0):
        g = Geometry(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, d]]), 6, near_gap=1.0)
        _q, F, T, _H = laplace.solve_magnetic(g, H0, eta)
        m = 4 * math.pi * beta
        Fd = 3 * m * m / (2 * math.pi * d ** 4)
        assert F[0, 2] > 0 and F[1, 2] < 0                 # attraction along the axis
        assert abs(F[0, 2] + F[1, 2]) < 1e-10 * abs(F[0, 2])
        errs.append(abs(F[0, 2] - Fd) / Fd)
    assert errs[1] < errs[0] and errs[1] < 0.02, errs


def test_series_matches_quadrature_on_a_sphere_of_radius_a():
    # Eq. 3.3 in units of the radius (value times a, gradient scale-free) against the
    # quadrature with the sphere's own nodes c + a x and weights a^2 w, far away
    for a in (0.4, 2.2):
        g = Geometry(np.array([[0.3, -0.2, 0.1]]), 14, near_gap=1.0, radii=[a])
        lap = laplace.Laplace(g)
        rng = np.random.default_rng(4)
        q = lap.synth(np.where(lap.n <= 3, lap.coef(rng.standard_normal(g.N)), 0))
        x = g.centres[0] + 5.0 * a * _dirs(rng, 4)
        s = lap.series(lap.coef(q), g.centres[0], x, a)
        d = lap.direct(q, g.centres[0], x, a)
        assert np.abs(s[0] - d[0]).max() < 1e-13 * a and np.abs(s[1] - d[1]).max() < 1e-13


@pytest.mark.parametrize("a", [0.35, 1.8])
def test_magnetisable_sphere_of_radius_a(a):
    # textbook: exterior potential -H0.x + beta a^3 (H0.x) / r^3, beta = (mu - mu0)/(mu + 2 mu0);
    # the surface density and field do not depend on a; no net force or torque
    mu = 4.0
    eta, beta = (mu - 1.0) / (mu + 1.0), (mu - 1.0) / (mu + 2.0)
    H0 = np.array([0.3, -1.0, 0.6])
    g = Geometry(np.zeros((1, 3)), 6, near_gap=1.0, radii=[a])
    q, F, T, H = laplace.solve_magnetic(g, H0, eta)
    lap = laplace.Laplace(g)
    assert np.abs(q - 6 * eta / (3 - eta) * (g.xhat @ H0)).max() < 1e-12
    x = a * np.array([1.3, 2.0, 4.0])[:, None] * _dirs(np.random.default_rng(5), 3)
    val, _grad = lap.series(lap.coef(q), np.zeros(3), x, a)
    r = np.linalg.norm(x, axis=1)
    assert np.abs(val - beta * a ** 3 * (x @ H0) / r ** 3).max() < 1e-12 * a
    n = g.xhat
    assert np.abs(H - (H0[None, :] - beta * (H0[None, :] - 3 * (n @ H0)[:, None] * n))).max() < 1e-12
    assert np.abs(F).max() < 1e-12 * a ** 2 and np.abs(T).max() < 1e-12 * a ** 3


def test_two_spheres_of_different_radii_attract_as_induced_dipoles():
    # moments m_i = 4 pi beta a_i^3 H0; along the field the force tends to 3 m1 m2 / (2 pi d^4)
    mu = 3.0
    eta, beta = (mu - 1) / (mu + 1), (mu - 1) / (mu + 2)
    H0 = np.array([0.0, 0.0, 1.0])
    rad = np.array([0.6, 1.3])
    errs = []
    for d in (6.0, 12.0):
        g = Geometry(np.array([[0.0, 0.0, 0.0], [0.0, 0.0, d]]), 6, near_gap=1.0, radii=rad)
        _q, F, _T, _H = laplace.solve_magnetic(g, H0, eta)
        m1, m2 = 4 * math.pi * beta * rad ** 3
        Fd = 3 * m1 * m2 / (2 * math.pi * d ** 4)
        assert F[0, 2] > 0 and F[1, 2] < 0
        # equal and opposite up to the discretisation error, which differs between two
        # spheres of different size at one p (measured 5e-7 at d = 6; exact only for the
        # symmetric pair of equal spheres)
        assert abs(F[0, 2] + F[1, 2]) < 1e-5 * abs(F[0, 2])
        errs.append(abs(F[0, 2] - Fd) / Fd)
    assert errs[1] < errs[0] and errs[1] < 0.02, errs


def test_magnetic_loads_scale_with_the_configuration():
    # centres and radii times lam: the density and surface field are unchanged, the
    # force scales by lam^2 and the torque by lam^3 (Maxwell traction times area, arm)
    c = np.array([[0.0, 0.0, 0.0], [1.9, 0.5, -0.3], [-0.6, 1.6, 0.8]])
    rad = np.array([0.8, 0.7, 0.55])
    lam = 1.6
    H0 = np.array([0.4, 0.2, 1.0])
    q1, F1, T1, H1 = laplace.solve_magnetic(Geometry(c, 5, near_gap=1.0, radii=rad), H0, 0.4)
    q2, F2, T2, H2 = laplace.solve_magnetic(Geometry(lam * c, 5, near_gap=1.0, radii=lam * rad), H0, 0.4)
    assert np.abs(q2 - q1).max() < 1e-12 and np.abs(H2 - H1).max() < 1e-12
    assert np.abs(F2 - lam ** 2 * F1).max() < 1e-11 * np.abs(F2).max()
    assert np.abs(T2 - lam ** 3 * T1).max() < 1e-11 * np.abs(T2).max()
