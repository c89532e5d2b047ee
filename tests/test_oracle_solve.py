"""Pins for oracle/operators.py and oracle/solvers.py (Sections 4.1, 4.3, 5, 6):
Stokes drag of an isolated sphere and its closed-form densities, near series against
brute force on an upsampled band-limited density, reproduction of exterior Stokes flows
by the solved second-kind equations (the validation protocol of Section 6, Eqs. 6.1-6.2,
on unit spheres), the two-sphere far-field limit, GMRES against dense LU."""
import math

import numpy as np
import pytest

from oracle import kernels
from oracle.grid import Geometry, mmax_for, sphere_grid
from oracle.harmonics import DenseVSH, vsh_at
from oracle.operators import Operators
from oracle.solvers import assemble, gmres, solve_mobility, solve_resistance


@pytest.mark.parametrize("p", [2, 4, 8])
@pytest.mark.parametrize("method", ["lu", "gmres"])
def test_isolated_sphere_resistance(p, method):
    g = Geometry(np.array([[0.3, -1.0, 2.0]]), p)
    v = np.array([[1.0, -2.0, 0.5]])
    om = np.array([[0.3, 0.7, -1.1]])
    F, T, psi, info = solve_resistance(g, v, om, method=method, tol=1e-13)
    assert np.abs(F - 6 * math.pi * v).max() < 1e-11
    assert np.abs(T - 8 * math.pi * om).max() < 1e-11
    x = g.xhat
    vv = v[0]
    exact = 1.5 * vv + (5.0 / 12.0) * (vv[None] - 3 * (x @ vv)[:, None] * x) + 3 * np.cross(om[0], x)
    assert np.abs(psi - exact).max() < 1e-11


@pytest.mark.parametrize("p", [2, 6])
@pytest.mark.parametrize("method", ["lu", "gmres"])
def test_isolated_sphere_mobility(p, method):
    g = Geometry(np.zeros((1, 3)), p)
    F = np.array([[1.0, 2.0, 3.0]])
    T = np.array([[-1.0, 0.5, 2.0]])
    v, om, mu, info = solve_mobility(g, F, T, method=method, tol=1e-13)
    assert np.abs(v - F / (6 * math.pi)).max() < 1e-12
    assert np.abs(om - T / (8 * math.pi)).max() < 1e-12
    exact = F[0][None] / (4 * math.pi) + (3 / (8 * math.pi)) * np.cross(T[0], g.xhat)
    assert np.abs(mu - exact).max() < 1e-12


def test_near_series_vs_upsampled_brute_force():
    # a band-limited density is known exactly on any finer grid, so the smooth
    # quadrature there converges to the exact layer potential at the gap used here
    p = 6
    src = Geometry(np.zeros((1, 3)), p)
    ops = Operators(src)
    rng = np.random.default_rng(3)
    mu = ops.vsh.inverse(ops.vsh.forward(rng.standard_normal((src.P, 3))))   # band-limited
    coef = ops.vsh.forward(mu)[..., None]
    fine = sphere_grid(140)
    modes = ops.vsh.modes
    _, _, Vf, Wf, Xf = vsh_at(fine["xhat"], p, src.mmax)
    mu_f = np.einsum("fmpc,fm->pc", np.stack([Vf, Wf, Xf]), coef[..., 0]).real
    tgt = Geometry(np.array([[0.0, 0.0, 0.0], [2.15, 0.4, -0.3]]), p).nodes[src.P:]
    for a_s, a_d in [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0)]:
        series = ops.near_field_from(coef, np.zeros(3), tgt, a_s, a_d)[..., 0]
        K = kernels.kernel_block(tgt, fine["xhat"], fine["xhat"], a_s, a_d)
        brute = np.einsum("tisj,sj->ti", K, mu_f * fine["wnode"][:, None])
        assert np.abs(series - brute).max() < 1e-9 * np.abs(brute).max()


def _stokeslet_data(points, forces, x):
    """sum_l G(x, p_l) f_l (Eq. 2.19)."""
    u = np.zeros_like(x)
    for pl, fl in zip(points, forces):
        u += kernels.stokeslet_rotlet(x, pl, fl[:, None], np.zeros((3, 1)))[..., 0]
    return u


def _exterior_eval(ops, dens, op, x):
    """Evaluate the representation sum_k (a_S S_k + a_D D_k [+ N_k])[dens] at exterior
    points x with the exterior series of every sphere."""
    g = ops.g
    a_s, a_d = (1.0, 1.0) if op == "SD" else (0.0, 1.0)
    u = np.zeros((x.shape[0], 3))
    for k in range(g.nb):
        coef = ops.coefficients(dens[..., None], k)
        u += ops.near_field_from(coef, g.centres[k], x, a_s, a_d)[..., 0]
    if op == "DN":
        F, T = ops.moments(dens[..., None])
        for k in range(g.nb):
            u += kernels.stokeslet_rotlet(x, g.centres[k], F[k], T[k])[..., 0]
    return u


@pytest.mark.parametrize("op", ["SD", "DN"])
def test_exterior_flow_reproduction_converges(op):
    # Section 6 "BIE data" protocol on unit spheres: boundary data from point forces
    # inside the particles is an exterior Stokes flow; the solved equation must
    # reproduce it away from the spheres, with error falling as p grows
    centres = np.array([[0.0, 0.0, 0.0], [2.6, 0.3, -0.2], [0.4, 2.5, 0.6]])
    rng = np.random.default_rng(7)
    dirs = rng.standard_normal((3, 3))
    pts = centres + 0.5 * dirs / np.linalg.norm(dirs, axis=1)[:, None]
    fs = rng.standard_normal((3, 3))
    xt = np.array([[1.3, -1.4, 0.2], [-1.0, 1.6, 1.2], [3.0, 2.6, 0.1], [1.2, 1.0, 2.0]])
    exact = _stokeslet_data(pts, fs, xt)
    errs = []
    for p in (4, 8, 12):
        g = Geometry(centres, p, near_gap=1.0)
        ops = Operators(g)
        b = _stokeslet_data(pts, fs, g.nodes).reshape(-1)
        name = "SD_BIE" if op == "SD" else "DN_BIE"
        fn = lambda z: ops.apply(name, z.reshape(g.N, 3)).reshape(-1)
        dens, info = gmres(fn, b, tol=1e-12, restart=200, max_iter=600)
        u = _exterior_eval(ops, dens.reshape(g.N, 3), op, xt)
        errs.append(np.abs(u - exact).max() / np.abs(exact).max())
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 3, errs
    assert errs[2] < 1e-5, errs


@pytest.mark.parametrize("d", [10.0, 20.0])
def test_two_sphere_mobility_far_field_rotne_prager(d):
    dh = np.array([1.0, 2.0, -0.5]) / np.linalg.norm([1.0, 2.0, -0.5])
    g = Geometry(np.stack([np.zeros(3), d * dh]), 4)
    F = np.array([[0.3, -1.0, 0.8], [0.0, 0.0, 0.0]])
    v, om, mu, info = solve_mobility(g, F, np.zeros((2, 3)), tol=1e-13)
    rp = (1 / (8 * math.pi * d)) * ((1 + 2 / (3 * d * d)) * F[0] + (1 - 2 / (d * d)) * dh * (dh @ F[0]))
    assert np.abs(v[1] - rp).max() / np.abs(rp).max() < 10.0 / d ** 4
    assert np.abs(v[0] - F[0] / (6 * math.pi)).max() < 10.0 / d ** 4


def test_gmres_matches_lu_and_translation_invariance():
    rng = np.random.default_rng(11)
    c = np.array([[0.0, 0.0, 0.0], [2.4, 0.5, 0.3]])
    g = Geometry(c, 4, near_gap=1.0)
    v = rng.standard_normal((2, 3))
    om = rng.standard_normal((2, 3))
    F1, T1, psi1, _ = solve_resistance(g, v, om, method="lu")
    F2, T2, psi2, info = solve_resistance(g, v, om, method="gmres", tol=1e-13)
    assert np.abs(F1 - F2).max() < 1e-10 and np.abs(psi1 - psi2).max() < 1e-10
    g3 = Geometry(c + np.array([5.0, -3.0, 7.5]), 4, near_gap=1.0)
    F3, T3, _, _ = solve_resistance(g3, v, om, method="lu")
    assert np.abs(F3 - F1).max() < 1e-11 and np.abs(T3 - T1).max() < 1e-11
    Fm = rng.standard_normal((2, 3))
    Tm = rng.standard_normal((2, 3))
    a = solve_mobility(g, Fm, Tm, method="lu")
    b = solve_mobility(g, Fm, Tm, method="gmres", tol=1e-13)
    assert np.abs(a[0] - b[0]).max() < 1e-10 and np.abs(a[1] - b[1]).max() < 1e-10


def test_grand_resistance_matrix_is_symmetric_positive():
    # reciprocity: the 12 x 12 resistance matrix of two spheres is symmetric positive
    # definite up to discretisation error
    g = Geometry(np.array([[0.0, 0.0, 0.0], [2.5, 0.3, 0.0]]), 8, near_gap=1.0)
    R = np.zeros((12, 12))
    for j in range(12):
        e = np.zeros(12)
        e[j] = 1.0
        F, T, _, _ = solve_resistance(g, e[:6].reshape(2, 3), e[6:].reshape(2, 3), tol=1e-12)
        R[:, j] = np.concatenate([F.reshape(-1), T.reshape(-1)])
    assert np.abs(R - R.T).max() / np.abs(R).max() < 1e-3
    assert np.linalg.eigvalsh(0.5 * (R + R.T)).min() > 0
