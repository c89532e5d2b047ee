"""Pins of the fluid-point evaluation and the porous-media problem (oracle/field.py):
textbook flows past one sphere, the jump relation at the surface, and agreement of the
exterior series with the smooth quadrature where both converge."""
import numpy as np
import pytest

from oracle import field
from oracle.grid import Geometry
from oracle.operators import Operators
from oracle.solvers import assemble
from oracle.harmonics import DenseVSH


def _points(rng, radii, c):
    d = rng.standard_normal((len(radii), 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return c[None, :] + np.asarray(radii)[:, None] * d


def fixed_sphere_flow(x, c, U):
    """Stokes flow past a fixed unit sphere at c in the uniform stream U (textbook)."""
    r = x - c[None, :]
    d = np.linalg.norm(r, axis=1)[:, None]
    rU = (r @ U)[:, None]
    return U[None, :] - 0.75 * (U[None, :] / d + rU * r / d ** 3) - 0.25 * (U[None, :] / d ** 3 - 3 * rU * r / d ** 5)


def test_flow_past_a_fixed_sphere():
    c = np.array([0.3, -0.2, 0.5])
    g = Geometry(c[None, :], 12, near_gap=1.0)
    ops = Operators(g)
    U = np.array([0.4, -1.1, 0.7])
    A = assemble(lambda m: ops.apply("SD_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    mu = np.linalg.solve(A, -np.tile(U, g.N)).reshape(g.N, 3)
    x = _points(np.random.default_rng(1), [1.02, 1.3, 1.9, 2.2, 3.5, 8.0], c)
    err = np.abs(U[None, :] + field.evaluate(g, mu, x, "SD_BIE", ops) - fixed_sphere_flow(x, c, U)).max(axis=1)
    # within d* of the surface: exterior series, exact for this degree-one density
    assert err[:3].max() < 1e-12, err
    # beyond: smooth quadrature of Eq. 4.4 (p = 12), its error at 1.2 from the surface
    assert err[3:].max() < 2e-8, err


def test_resistance_field_of_a_translating_rotating_sphere():
    # completed double layer: psi of an isolated sphere (closed form) -> exterior flow =
    # translating sphere (Stokeslet + source doublet) + rotating sphere (rotlet)
    g = Geometry(np.zeros((1, 3)), 12, near_gap=1.0)
    ops = Operators(g)
    v = np.array([1.0, 0.5, -0.3])
    om = np.array([-0.2, 0.8, 0.4])
    xh = g.grid["xhat"]
    A = assemble(lambda m: ops.apply("DN_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    psi = np.linalg.solve(A, (v[None, :] + np.cross(om[None, :], xh)).reshape(-1)).reshape(g.N, 3)
    x = _points(np.random.default_rng(2), [1.05, 1.6, 2.5, 6.0], np.zeros(3))
    u = field.evaluate(g, psi, x, "DN_BIE", ops)
    d = np.linalg.norm(x, axis=1)[:, None]
    rv = (x @ v)[:, None]
    ref = 0.75 * (v / d + rv * x / d ** 3) + 0.25 * (v / d ** 3 - 3 * rv * x / d ** 5) + np.cross(om, x) / d ** 3
    err = np.abs(u - ref).max(axis=1)
    assert err[:2].max() < 1e-12, err      # exterior series
    assert err[2:].max() < 1e-7, err       # smooth quadrature, p = 12


def test_exterior_limit_is_the_second_kind_operator():
    # jump relation (Eq. A.7): (S + D)[mu](x) -> 1/2 mu + S mu + D_pv mu as x -> surface
    g = Geometry(np.zeros((1, 3)), 6, near_gap=1.0)
    ops = Operators(g)
    vsh = DenseVSH(g.grid, g.p, g.mmax)
    rng = np.random.default_rng(3)
    mu = vsh.inverse(vsh.forward(rng.standard_normal((g.N, 3))))        # band-limited
    k = [0, 17, 40, 63]
    eps = 1e-8
    x = g.nodes[k] * (1.0 + eps)
    u = field.evaluate(g, mu, x, "SD_BIE", ops)
    ref = ops.apply("SD_BIE", mu)[k]
    assert np.abs(u - ref).max() < 1e-6 * np.abs(ref).max()


def test_series_and_quadrature_agree_at_moderate_distance():
    # a smooth density (degree <= 3) far enough from the points that the p = 14
    # quadrature is exact to rounding: the exterior series must give the same values
    c = np.array([[0.0, 0.0, 0.0], [12.0, 0.1, -0.4]])
    rng = np.random.default_rng(4)
    x = _points(rng, [4.0, 4.5, 5.5], c[0])
    g_near = Geometry(c, 14, near_gap=20.0)    # every point takes the series
    g_far = Geometry(c, 14, near_gap=0.5)      # every point takes the quadrature
    vsh = DenseVSH(g_near.grid, g_near.p, g_near.mmax)
    low = np.array([n <= 3 for (n, m) in vsh.modes])
    mu = rng.standard_normal((g_near.N, 3))
    for k in range(2):
        sl = g_near.sphere_nodes(k)
        coef = vsh.forward(mu[sl])
        coef[:, ~low] = 0.0
        mu[sl] = vsh.inverse(coef)
    for op in ("S", "D", "DN_BIE"):
        a = field.evaluate(g_near, mu, x, op)
        b = field.evaluate(g_far, mu, x, op)
        assert np.abs(a - b).max() < 1e-12 * np.abs(a).max(), op


def test_points_inside_a_sphere_are_rejected():
    g = Geometry(np.zeros((1, 3)), 4, near_gap=1.0)
    with pytest.raises(ValueError):
        field.evaluate(g, np.zeros((g.N, 3)), np.array([[0.2, 0.1, 0.0]]))
