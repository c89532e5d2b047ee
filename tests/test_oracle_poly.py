"""Pins of the polydisperse (per-sphere radius) oracle: scale invariance of the layer
operators, the exterior series on a sphere of radius a against brute-force quadrature,
the textbook flow past a fixed sphere of radius a, and unit radii reproducing the
monodisperse operators."""
import math

import numpy as np
import pytest

from oracle import kernels
from oracle import traction as tr
from oracle.grid import Geometry, sphere_grid
from oracle.harmonics import DenseVSH, vsh_at
from oracle.operators import Operators
from oracle.solvers import assemble


def poly_cluster(seed=3):
    """Six spheres of radii 0.35-1.4 with several near pairs (gaps 0.05-0.6)."""
    c = np.array([[0.0, 0.0, 0.0], [2.2, 0.3, -0.1], [0.4, 1.75, 0.5], [-1.5, -0.6, 0.9],
                  [1.3, -1.4, 1.2], [4.4, 2.2, 0.4]])
    a = np.array([1.0, 1.1, 0.45, 0.6, 0.35, 1.4])
    d = np.linalg.norm(c[:, None] - c[None, :], axis=-1) - a[:, None] - a[None, :]
    np.fill_diagonal(d, np.inf)
    assert d.min() > 0.04
    return c, a


def test_unit_radii_reproduce_the_monodisperse_operators():
    c, _a = poly_cluster()
    g0 = Geometry(c * 1.5, 5, near_gap=1.0)
    g1 = Geometry(c * 1.5, 5, near_gap=1.0, radii=np.ones(len(c)))
    mu = np.random.default_rng(1).standard_normal((g0.N, 3))
    for op in ("S", "D", "SD_BIE", "DN_BIE"):
        assert np.array_equal(Operators(g0).apply(op, mu), Operators(g1).apply(op, mu))
    assert np.array_equal(g0.near, g1.near)


@pytest.mark.parametrize("lam", [0.6, 1.7])
def test_scale_invariance(lam):
    # the single layer is homogeneous of degree 1 in the length scale, the double layer
    # and the traction of degree 0: scaling every centre and radius by lam maps the
    # same nodal density to lam * S, D, K (self, near and far parts together)
    c, a = poly_cluster()
    p = 5
    g = Geometry(c, p, near_gap=1.0, radii=a)
    gs = Geometry(lam * c, p, near_gap=1.0, radii=lam * a)
    assert np.array_equal(g.near, gs.near) and g.near.sum() > 0
    mu = np.random.default_rng(2).standard_normal((g.N, 3))
    o, os_ = Operators(g), Operators(gs)
    S, Ss = o.apply("S", mu), os_.apply("S", mu)
    D, Ds = o.apply("D", mu), os_.apply("D", mu)
    K, Ks = tr.TractionOps(g).apply_K(mu), tr.TractionOps(gs).apply_K(mu)
    assert np.abs(Ss - lam * S).max() < 1e-12 * np.abs(S).max() * 10
    assert np.abs(Ds - D).max() < 1e-12 * np.abs(D).max() * 10
    assert np.abs(Ks - K).max() < 1e-12 * np.abs(K).max() * 10


@pytest.mark.parametrize("radius", [0.4, 1.6])
def test_exterior_series_on_a_sphere_of_radius_a_matches_quadrature(radius):
    # band-limited density on a sphere of radius a, points 0.6 a - 2 a from its surface;
    # brute force on a fine grid of the same sphere (nodes a xhat, weights a^2 w)
    p = 5
    g = Geometry(np.zeros((1, 3)), p, n_phi=2 * p + 2)
    ops = Operators(g)
    rng = np.random.default_rng(3)
    mu = rng.standard_normal((g.P, 3))
    coef = DenseVSH(g.grid, p, g.mmax).forward(mu)[..., None]
    fine = sphere_grid(40, 82)
    _m, _Y, V, W, X = vsh_at(fine["xhat"], p, g.mmax)
    dens = (np.einsum("mki,m->ki", V, coef[0, :, 0]) + np.einsum("mki,m->ki", W, coef[1, :, 0])
            + np.einsum("mki,m->ki", X, coef[2, :, 0])).real
    d = rng.standard_normal((6, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = radius * (1.6 + 1.4 * rng.random(6))[:, None] * d
    q = (dens * (radius ** 2 * fine["wnode"])[:, None])[:, :, None]
    for a_s, a_d in ((1.0, 0.0), (0.0, 1.0), (1.0, 1.0)):
        series = ops.near_field_from(coef, np.zeros(3), x, a_s, a_d, radius)[..., 0]
        brute = kernels.direct_sum(x, radius * fine["xhat"], fine["xhat"], q, a_s, a_d)[..., 0]
        assert np.abs(series - brute).max() < 1e-11 * np.abs(brute).max(), (a_s, a_d)


def test_fixed_sphere_of_radius_a_in_a_uniform_stream():
    # Problem 1 on one sphere of radius a: the flow is the textbook one with a in place
    # of 1, and the sphere exerts -6 pi a U on the fluid (int mu over the surface)
    a = 0.45
    cen = np.array([0.3, -0.2, 0.5])
    g = Geometry(cen[None, :], 10, near_gap=1.0, radii=[a])
    ops = Operators(g)
    U = np.array([0.4, -1.1, 0.7])
    A = assemble(lambda m: ops.apply("SD_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    mu = np.linalg.solve(A, -np.tile(U, g.N)).reshape(g.N, 3)
    F = (mu * g.w[:, None]).sum(axis=0)
    assert np.abs(F + 6 * math.pi * a * U).max() < 1e-11
    rng = np.random.default_rng(4)
    d = rng.standard_normal((5, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = cen[None, :] + a * np.array([1.05, 1.4, 2.5, 4.0, 9.0])[:, None] * d
    coef = ops.coefficients(mu, 0)[..., None]
    u = U[None, :] + ops.near_field_from(coef, cen, x, 1.0, 1.0, a)[..., 0]
    r = x - cen[None, :]
    dd = np.linalg.norm(r, axis=1)[:, None]
    rU = (r @ U)[:, None]
    ref = U[None, :] - 0.75 * a * (U[None, :] / dd + rU * r / dd ** 3) - 0.25 * a ** 3 * (U[None, :] / dd ** 3
                                                                                          - 3 * rU * r / dd ** 5)
    assert np.abs(u - ref).max() < 1e-12


def test_near_classification_scales_with_the_source_radius():
    # gap 0.3 between a unit sphere and a sphere of radius 0.2: within d* = 1 of the
    # large source, beyond d* a_s = 0.2 of the small one
    c = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0]])
    g = Geometry(c, 4, near_gap=1.0, radii=[1.0, 0.2])
    assert g.near[1, 0] and not g.near[0, 1]


def test_isolated_sphere_of_radius_a_resistance():
    # Problem 5 on one sphere of radius a: F = 6 pi a v, T = 8 pi a^3 omega (Stokes)
    from oracle import solvers
    a = 0.6
    g = Geometry(np.array([[0.2, 0.4, -0.1]]), 6, radii=[a])
    v = np.array([[0.3, -1.0, 0.8]])
    om = np.array([[1.1, 0.2, -0.5]])
    F, T, _psi, info = solvers.solve_resistance(g, v, om, method="lu")
    assert np.abs(F - 6 * math.pi * a * v).max() < 1e-11
    assert np.abs(T - 8 * math.pi * a ** 3 * om).max() < 1e-11


def test_m0_inverts_the_isolated_completed_operator_of_radius_a():
    from oracle.precond import m0_resistance
    for a in (0.3, 1.0, 2.5):
        g = Geometry(np.zeros((1, 3)), 6, radii=[a])
        r = np.random.default_rng(5).standard_normal((g.N, 3))
        z = m0_resistance(g, Operators(g).apply("DN_BIE", r))
        assert np.abs(z - r).max() < 1e-11 * np.abs(r).max(), a


def test_resistance_scales_with_the_configuration():
    # scaling centres and radii by lam, a pure translation gives lam F and lam^2 T.  In
    # the completed form this holds because the rigid part of psi scales by 1/lam and the
    # rest not at all, which needs the double layer of a rigid density to vanish off its
    # sphere: exact for the operator, up to the far quadrature's error on the grid (p = 4
    # here: ~5e-5 relative)
    from oracle import solvers
    c, a = poly_cluster()
    lam = 1.4
    rng = np.random.default_rng(6)
    v = rng.standard_normal((len(c), 3))
    zero = np.zeros_like(v)
    g, gs = Geometry(c, 4, radii=a), Geometry(lam * c, 4, radii=lam * a)
    F1, T1, _p, _i = solvers.solve_resistance(g, v, zero, tol=1e-12)
    F2, T2, _p, _i = solvers.solve_resistance(gs, v, zero, tol=1e-12)
    assert np.abs(F2 - lam * F1).max() < 1e-3 * np.abs(F1).max()
    assert np.abs(T2 - lam ** 2 * T1).max() < 1e-3 * np.abs(T1).max()


def test_isolated_sphere_of_radius_a_mobility():
    # bordered mobility form on one sphere of radius a: v = F / (6 pi a), omega = T / (8 pi a^3)
    from oracle import solvers
    a = 1.7
    g = Geometry(np.array([[0.0, 1.0, 2.0]]), 6, radii=[a])
    F = np.array([[0.5, -1.5, 0.25]])
    T = np.array([[-0.4, 0.9, 1.3]])
    v, om, _mu, info = solvers.solve_mobility(g, F, T, method="lu")
    assert np.abs(v - F / (6 * math.pi * a)).max() < 1e-12
    assert np.abs(om - T / (8 * math.pi * a ** 3)).max() < 1e-12


def test_mobility_inverts_resistance_with_radii():
    # two spheres of different radii: the mobility solve driven by the resistance solve's
    # forces and torques returns the imposed rigid motions (both forms are discretised
    # from the same layer operators, so they agree to the discretisation error)
    from oracle import solvers
    c = np.array([[0.0, 0.0, 0.0], [2.0, 0.4, -0.3]])
    a = np.array([1.0, 0.6])
    g = Geometry(c, 8, radii=a)
    rng = np.random.default_rng(9)
    v = rng.standard_normal((2, 3))
    om = rng.standard_normal((2, 3))
    F, T, _psi, _i = solvers.solve_resistance(g, v, om, tol=1e-12)
    v2, om2, _mu, _i2 = solvers.solve_mobility(g, F, T, tol=1e-12)
    assert np.abs(v2 - v).max() < 1e-5 and np.abs(om2 - om).max() < 1e-5


def test_traction_mobility_with_radii():
    # Problem 2 in the paper's form on spheres of radius a: the isolated sphere moves
    # with F/(6 pi a), T/(8 pi a^3); two spheres of different radii agree with the
    # bordered form to the discretisation error (p = 8, gap 0.46 = 0.77 of the small
    # radius: ~2e-4)
    from oracle import solvers
    g1 = Geometry(np.array([[0.3, 0.0, -0.4]]), 6, radii=[0.55])
    F = np.array([[0.7, -0.2, 1.1]])
    T = np.array([[0.1, 0.9, -0.6]])
    v, om, mu, _i = tr.solve_mobility_traction(g1, F, T)
    assert np.abs(v - F / (6 * math.pi * 0.55)).max() < 1e-12
    assert np.abs(om - T / (8 * math.pi * 0.55 ** 3)).max() < 1e-12
    c = np.array([[0.0, 0.0, 0.0], [2.0, 0.4, -0.3]])
    g = Geometry(c, 8, radii=[1.0, 0.6])
    rng = np.random.default_rng(10)
    F = rng.standard_normal((2, 3))
    T = rng.standard_normal((2, 3))
    v1, o1, _m1, _i1 = tr.solve_mobility_traction(g, F, T, tol=1e-12)
    v2, o2, _m2, _i2 = solvers.solve_mobility(g, F, T, tol=1e-12)
    assert np.abs(v1 - v2).max() < 1e-3 * np.abs(v2).max() and np.abs(o1 - o2).max() < 1e-3 * np.abs(o2).max()


def test_fluid_points_around_a_fixed_sphere_of_radius_a():
    # Problem 1 on one sphere of radius a, the flow evaluated at fluid points: exterior
    # series within d* a of the surface (exact for this degree-one density), quadrature
    # beyond (p = 12: its error at 1.2 a from the surface, 1e-8 - 1.3e-7 by direction)
    from oracle import field
    a = 0.45
    cen = np.array([0.3, -0.2, 0.5])
    g = Geometry(cen[None, :], 12, near_gap=1.0, radii=[a])
    ops = Operators(g)
    U = np.array([0.4, -1.1, 0.7])
    A = assemble(lambda m: ops.apply("SD_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    mu = np.linalg.solve(A, -np.tile(U, g.N)).reshape(g.N, 3)
    d = np.random.default_rng(11).standard_normal((6, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = cen[None, :] + a * np.array([1.02, 1.3, 1.9, 2.2, 3.5, 8.0])[:, None] * d
    u = U[None, :] + field.evaluate(g, mu, x, "SD_BIE", ops)
    r = x - cen[None, :]
    dd = np.linalg.norm(r, axis=1)[:, None]
    rU = (r @ U)[:, None]
    ref = U[None, :] - 0.75 * a * (U[None, :] / dd + rU * r / dd ** 3) - 0.25 * a ** 3 * (U[None, :] / dd ** 3
                                                                                          - 3 * rU * r / dd ** 5)
    err = np.abs(u - ref).max(axis=1)
    assert err[:3].max() < 1e-12 and err[3:].max() < 3e-7 and err[4:].max() < 1e-12, err


def test_rigid_coarse_operator_with_radii():
    # R A P of the completed operator (radii) = the one-sided closed form; the two-sided
    # (polydisperse Rotne-Prager-Yamakawa) translation block = the Stokeslet averaged over
    # both spheres (quadrature); R M0 P = diag(3/(2a), 3/a) = A_c^-1 of one sphere
    from oracle import rigid
    from oracle.kernels import kernel_block
    from oracle.precond import m0_resistance
    c = np.array([[0.0, 0.0, 0.0], [2.9, 0.4, 0.2], [0.3, -2.9, 1.5]])
    a = np.array([1.0, 0.6, 0.8])
    g = Geometry(c, 10, near_gap=1.0, radii=a)
    assert g.near.sum() == 0
    ops = Operators(g)
    xh, w = g.grid["xhat"], g.grid["wnode"]
    cols = []
    for k in range(g.nb):
        for m in range(6):
            y = np.zeros(6)
            y[m] = 1.0
            f = np.zeros((g.N, 3))
            f[g.sphere_nodes(k)] = rigid.prolong(y, xh, a[k])
            u = ops.apply("DN_BIE", f)
            cols.append(np.concatenate([rigid.restrict(u[g.sphere_nodes(i)], xh, w, a[i]) for i in range(g.nb)]))
    rap = np.array(cols).T
    one = rigid.coarse_operator(c, two_sided=False, radii=a)
    assert np.abs(rap - one).max() < 1e-7 * np.abs(one).max()
    # two-sided translation block by quadrature over spheres of radii 0.7 and 0.4
    g24 = Geometry(np.zeros((1, 3)), 24, near_gap=1.0)
    xh24, w24 = g24.grid["xhat"], g24.grid["wnode"]
    e = np.array([0.36, -0.48, 0.8])
    ai, ak, d = 0.7, 0.4, 1.6
    K = kernel_block(d * e + ai * xh24, ak * xh24, xh24, 1.0, 0.0)
    avg = np.einsum("t,tisj,s->ij", w24, K, w24) / (4 * math.pi) ** 2
    M = rigid.mobility(np.stack([d * e, np.zeros(3)]), radii=[ai, ak])
    assert np.abs(M[0:3, 6:9] - avg).max() < 1e-10
    # isolated sphere of radius a
    for rad in (0.4, 2.0):
        g1 = Geometry(np.zeros((1, 3)), 8, near_gap=1.0, radii=[rad])
        y = np.random.default_rng(12).standard_normal(6)
        f = rigid.prolong(y, g1.grid["xhat"], rad)
        assert np.abs(rigid.restrict(f, g1.grid["xhat"], g1.grid["wnode"], rad) - y).max() < 1e-13
        z = m0_resistance(g1, f)
        assert np.abs(rigid.restrict(z, g1.grid["xhat"], g1.grid["wnode"], rad) - rigid.b0(rad) * y).max() < 1e-12
        Ac = rigid.coarse_operator(np.zeros((1, 3)), radii=[rad])
        assert np.abs(np.linalg.inv(Ac) - np.diag(rigid.b0(rad))).max() < 1e-12 * rigid.b0(rad).max()
        r = np.random.default_rng(13).standard_normal((g1.N, 3))
        z0 = m0_resistance(g1, r)
        assert np.abs(rigid.correct(g1, r, z0) - z0).max() < 1e-12


def test_polydisperse_rpy_is_positive_definite():
    from oracle import rigid
    c, a = poly_cluster()
    assert np.linalg.eigvalsh(rigid.mobility(c, radii=a)).min() > 0
