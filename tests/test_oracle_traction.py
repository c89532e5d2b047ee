"""Pins of the single-layer traction oracle and of Problem 2 in the paper's form
(oracle/traction.py) against the exterior series, central differences, brute-force
quadrature, the printed Eqs. 3.19-3.21 and Table 3.12, force balance, and the
isolated-sphere mobility."""
import math

import numpy as np
import pytest

from oracle import solvers, spectra
from oracle import traction as tr
from oracle.grid import Geometry, sphere_grid
from oracle.harmonics import mode_list, vsh_at
from oracle.operators import Operators


def real_coefficients(p, mmax, rng, families=(0, 1, 2)):
    """Random VSH coefficients (3, M, 1) of a real density (c_{n,-m} = conj(c_{n,m}))."""
    modes = mode_list(p, mmax)
    idx = {nm: i for i, nm in enumerate(modes)}
    c = np.zeros((3, len(modes), 1), complex)
    for (n, m), i in idx.items():
        if m < 0:
            continue
        for f in families:
            if f > 0 and n == 0:
                continue
            z = rng.standard_normal() + (1j * rng.standard_normal() if m > 0 else 0.0)
            c[f, i, 0] = z
    for (n, m), i in idx.items():
        if m < 0:
            c[:, i] = np.conj(c[:, idx[(n, -m)]])
    return c


def density_on(grid, coef, p, mmax):
    _m, _Y, V, W, X = vsh_at(grid["xhat"], p, mmax)
    return (np.einsum("mki,m->ki", V, coef[0, :, 0]) + np.einsum("mki,m->ki", W, coef[1, :, 0])
            + np.einsum("mki,m->ki", X, coef[2, :, 0])).real


POINTS = np.array([[1.3, 0.4, -0.9], [0.1, 0.05, 2.2], [-2.0, 1.0, 0.3], [0.7, -1.1, 0.2]])


def test_harmonic_form_reproduces_exterior_series():
    p, mmax = 6, 5
    coef = real_coefficients(p, mmax, np.random.default_rng(0))
    g = Geometry(np.zeros((1, 3)), p, n_phi=2 * mmax + 2)
    ops = Operators(g)
    u, G, _p = tr.single_layer_flow(coef, p, mmax, POINTS)
    ref = ops.near_field_from(coef, np.zeros(3), POINTS, 1.0, 0.0)
    assert np.abs(u - ref).max() < 1e-14 * np.abs(ref).max() * 10
    # incompressible (A.4)
    assert np.abs(np.einsum("xiib->xb", G)).max() < 1e-13


def test_velocity_gradient_matches_central_differences():
    p, mmax = 5, 5
    coef = real_coefficients(p, mmax, np.random.default_rng(1))
    g = Geometry(np.zeros((1, 3)), p, n_phi=2 * mmax + 2)
    ops = Operators(g)
    _u, G, _p = tr.single_layer_flow(coef, p, mmax, POINTS)
    h = 1e-4
    Gfd = np.zeros_like(G)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        up = ops.near_field_from(coef, np.zeros(3), POINTS + e, 1.0, 0.0)
        um = ops.near_field_from(coef, np.zeros(3), POINTS - e, 1.0, 0.0)
        Gfd[:, :, j] = (up - um) / (2 * h)
    assert np.abs(G - Gfd).max() < 1e-7 * np.abs(G).max()


def test_traction_and_pressure_match_quadrature_for_any_normal():
    # brute force: the density is band-limited, so it is known exactly on a fine grid;
    # the points are >= 0.6 from the sphere, where the fine-grid quadrature converges
    p, mmax = 6, 6
    rng = np.random.default_rng(2)
    coef = real_coefficients(p, mmax, rng)
    fine = sphere_grid(40, 82)
    q = density_on(fine, coef, p, mmax) * fine["wnode"][:, None]
    pts = POINTS[:3]
    nrm = rng.standard_normal((len(pts), 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    t = tr.single_layer_traction(coef, p, mmax, pts, nrm)[..., 0]
    tq = tr.traction_sum(pts, nrm, fine["xhat"], q)
    assert np.abs(t - tq).max() < 1e-12 * np.abs(tq).max()
    _u, _G, pr = tr.single_layer_flow(coef, p, mmax, pts)
    pq = tr.pressure_sum(pts, fine["xhat"], q)
    assert np.abs(pr[:, 0] - pq).max() < 1e-12 * np.abs(pq).max()


@pytest.mark.parametrize("n", [0, 1, 2, 4])
def test_radial_normal_reproduces_printed_exterior_formulas(n):
    # Eqs. 3.19-3.21 (r > 1) for pure modes, target normal e_r, several m
    p = 5
    rng = np.random.default_rng(3 + n)
    modes = mode_list(p, p)
    pts = rng.standard_normal((5, 3))
    pts *= (1.2 + rng.random(5))[:, None] / np.linalg.norm(pts, axis=1)[:, None]
    r = np.linalg.norm(pts, axis=1)
    er = pts / r[:, None]
    _mm, _Y, V, W, X = vsh_at(er, p, p)
    for m in sorted({0, min(n, 1), n}):
        i = modes.index((n, m))
        kvv, kww, kwv, kxx = tr.exterior_K_er(n, r)
        for f in range(3 if n > 0 else 1):
            c = np.zeros((3, len(modes), 1), complex)
            c[f, i, 0] = 1.0
            t = _complex_traction(c, p, pts, er)
            if f == 0:
                ref = kvv[:, None] * V[i]
            elif f == 1:
                ref = kww[:, None] * W[i] + kwv[:, None] * V[i]
            else:
                ref = kxx[:, None] * X[i]
            assert np.abs(t - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), (n, m, f)


def _complex_traction(c, p, pts, nrm):
    """Traction of the flow of one complex mode (no real part taken)."""
    _u, G, pr = tr.single_layer_flow_complex(c, p, p, pts)
    t = np.einsum("xijb,xj->xib", G, nrm) + np.einsum("xjib,xj->xib", G, nrm)
    return (t - nrm[:, :, None] * pr[:, None, :])[..., 0]


def test_surface_limit_is_the_exterior_eigenvalue():
    # r -> 1+: Eqs. 3.19-3.21 tend to the K_+ row of Table 3.12 (mode by mode)
    for n in range(0, 6):
        kvv, kww, kwv, kxx = tr.exterior_K_er(n, 1.0)
        v, w, x = tr.eig_Kplus(n)
        assert abs(kvv - v) < 1e-15 and abs(kww - w) < 1e-15 and abs(kxx - x) < 1e-15 and abs(kwv) < 1e-15
        # and K_+ - K_- = -1 on every mode that exists (jump A.6)
        km = tr.eig_Kminus(n)
        for a, b, exists in zip((v, w, x), km, (True, n >= 1, n >= 1)):
            if exists:
                assert abs(a - b + 1.0) < 1e-14


def test_principal_value_equals_double_layer_principal_value():
    # the mean of the K rows equals the mean of the D rows on every mode: on the unit
    # sphere the surface operators K_pv and D_pv coincide (K is the adjoint of D)
    for n in range(0, 12):
        a = tr.eig_Kpv(n)
        b = spectra.eig_Dpv(n)
        for f, (x, y) in enumerate(zip(a, b)):
            if n == 0 and f > 0:
                continue
            assert abs(x - y) < 1e-15


def test_traction_on_a_closed_sphere_carries_no_force_or_torque():
    # the flow of sphere s is regular inside a neighbouring ball: the traction integrated
    # over its surface balances (div sigma = 0 inside), force and torque both vanish
    p, mmax = 6, 6
    coef = real_coefficients(p, mmax, np.random.default_rng(4))
    ct = np.array([0.3, 2.1, 0.5])                     # gap about 0.2 to the source
    grid = sphere_grid(30, 62)
    pts = ct[None, :] + grid["xhat"]
    t = tr.single_layer_traction(coef, p, mmax, pts, grid["xhat"])[..., 0]
    F = (t * grid["wnode"][:, None]).sum(axis=0)
    T = (np.cross(grid["xhat"], t) * grid["wnode"][:, None]).sum(axis=0)
    scale = (np.abs(t) * grid["wnode"][:, None]).sum()
    assert np.abs(F).max() < 1e-10 * scale and np.abs(T).max() < 1e-10 * scale


def test_ladder_projection_is_exact():
    # e_i . V_n^m lies in the span of degree n+1 harmonics (and nothing else)
    p = 4
    L = tr.ladder(p, p)
    mi = mode_list(p, p)
    mo = mode_list(p + 1, p + 1)
    for a, (n, m) in enumerate(mi):
        for b, (n2, _m2) in enumerate(mo):
            if n2 != n + 1:
                assert np.abs(L[:, b, a]).max() < 1e-13
    pts = np.random.default_rng(5).standard_normal((20, 3))
    pts /= np.linalg.norm(pts, axis=1)[:, None]
    _m, _Y, V, _W, _X = vsh_at(pts, p, p)
    _mo, Yo, _Vo, _Wo, _Xo = vsh_at(pts, p + 1, p + 1)
    rec = np.einsum("iom,ok->mki", L, Yo)
    assert np.abs(rec - V).max() < 1e-13


def test_isolated_sphere_moves_with_stokes_mobility():
    g = Geometry(np.array([[0.5, -1.0, 2.0]]), 6)
    F = np.array([[1.0, -2.0, 0.5]])
    T = np.array([[0.3, 0.7, -1.1]])
    v, om, mu, info = tr.solve_mobility_traction(g, F, T)
    assert np.abs(v - F / (6 * math.pi)).max() < 1e-13
    assert np.abs(om - T / (8 * math.pi)).max() < 1e-13
    assert np.abs(mu).max() < 1e-12


def test_paper_mobility_agrees_with_bordered_formulation():
    # two formulations of Problem 2 on the same discretisation: they agree to the
    # discretisation error, which shrinks with p
    c = np.array([[0.0, 0.0, 0.0], [2.6, 0.3, -0.2], [0.4, 2.5, 0.9]])
    rng = np.random.default_rng(6)
    F = rng.standard_normal((3, 3))
    T = rng.standard_normal((3, 3))
    errs, moms = [], []
    for p in (4, 8):
        g = Geometry(c, p, near_gap=1.0)
        v, om, mu, info = tr.solve_mobility_traction(g, F, T, tol=1e-12)
        assert info["rel_residual"] < 1e-11
        v2, om2, _mu2, _i2 = solvers.solve_mobility(g, F, T, tol=1e-12)
        errs.append(max(np.abs(v - v2).max() / np.abs(v2).max(), np.abs(om - om2).max() / np.abs(om2).max()))
        # L selects the mu with no net force or torque; the discrete rigid modes are
        # left null vectors of 1/2 I + K up to the discretisation error, so the moments
        # of the discrete solution vanish at that rate
        Fm, Tm = Operators(g).moments(mu)
        moms.append(max(np.abs(Fm).max(), np.abs(Tm).max()))
    # spectral convergence of both (p = 4: ~5e-4 / 3e-4, p = 8: ~2e-6 / 8e-7)
    assert errs[1] < 1e-5 and errs[1] < 0.01 * errs[0], errs
    assert moms[1] < 1e-5 and moms[1] < 0.01 * moms[0], moms
