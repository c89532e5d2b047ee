"""Pins of the pole-rotation near evaluation oracle (oracle/rotation_near.py, Section 4.2)."""
import math

import numpy as np
import pytest

from oracle import rotation_near as rn
from oracle.grid import Geometry
from oracle.harmonics import DenseVSH, vsh_at
from oracle.operators import Operators


def _rot(axis, a):
    c, s = math.cos(a), math.sin(a)
    if axis == "z":
        return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def test_rotation_to_pole():
    rng = np.random.default_rng(0)
    for _ in range(5):
        d = rng.standard_normal(3) * 3
        Q = rn.rotation_to_pole(d)
        assert np.abs(Q @ Q.T - np.eye(3)).max() < 1e-14 and abs(np.linalg.det(Q) - 1) < 1e-14
        assert np.abs(Q @ d - np.array([0, 0, np.linalg.norm(d)])).max() < 1e-13


def test_wigner_matrices():
    rng = np.random.default_rng(1)
    Q = rn.rotation_to_pole(rng.standard_normal(3))
    for n in range(6):
        D = rn.wigner(n, Q)
        assert np.abs(D @ D.conj().T - np.eye(2 * n + 1)).max() < 1e-13
        assert np.abs(rn.wigner(n, Q.T) - D.conj().T).max() < 1e-13
        a = 0.7
        Dz = rn.wigner(n, _rot("z", a))
        assert np.abs(Dz - np.diag(np.exp(-1j * np.arange(-n, n + 1) * a))).max() < 1e-13
        # composition
        Q2 = _rot("y", 0.4) @ _rot("z", -1.1)
        assert np.abs(rn.wigner(n, Q @ Q2) - rn.wigner(n, Q) @ rn.wigner(n, Q2)).max() < 1e-12


def test_rotated_coefficients_resynthesise_the_rotated_field():
    p = 5
    rng = np.random.default_rng(2)
    modes = rn.full_modes(p)
    c = rng.standard_normal((3, len(modes))) + 1j * rng.standard_normal((3, len(modes)))
    Q = rn.rotation_to_pole(rng.standard_normal(3))
    cR = rn.rotate(c, p, Q)
    x = rng.standard_normal((20, 3))
    x /= np.linalg.norm(x, axis=1)[:, None]

    def synth(coef, pts):
        _m, _Y, V, W, X = vsh_at(pts, p, p)
        return np.einsum("mkc,m->kc", V, coef[0]) + np.einsum("mkc,m->kc", W, coef[1]) + np.einsum("mkc,m->kc", X, coef[2])

    direct = synth(c, x @ Q) @ Q.T          # Q f(Q^T x), rows
    assert np.abs(synth(cR, x) - direct).max() < 1e-12


def test_pair_on_the_pole_is_the_projection_of_the_direct_series():
    c = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.3]])
    g = Geometry(c, 6, near_gap=1.0)
    ops = Operators(g)
    vsh = DenseVSH(g.grid, g.p, g.mmax)
    mu = np.random.default_rng(3).standard_normal((g.N, 3))
    coef = vsh.forward(mu[g.sphere_nodes(0)])
    got = rn.pair_coefficients(g, coef, c[1] - c[0], 1.0, 1.0, vsh)
    direct = ops.near_field_from(coef[:, :, None], c[0], g.nodes[g.sphere_nodes(1)], 1.0, 1.0)[..., 0]
    assert np.abs(got - vsh.forward(direct)).max() < 1e-13 * np.abs(got).max()


@pytest.mark.parametrize("op", [(1.0, 0.0), (0.0, 1.0)])
def test_converges_to_the_direct_series(op):
    a_s, a_d = op
    rng = np.random.default_rng(4)
    d = rng.standard_normal(3)
    c = np.array([[0.0, 0.0, 0.0], 2.5 * d / np.linalg.norm(d)])
    errs = []
    for p in (6, 10, 14):
        g = Geometry(c, p, near_gap=1.0)
        ops = Operators(g)
        vsh = DenseVSH(g.grid, p, g.mmax)
        low = np.array([n <= 3 for (n, m) in vsh.modes])
        mu = np.random.default_rng(5).standard_normal((g.N, 3))
        for k in range(2):
            cf = vsh.forward(mu[g.sphere_nodes(k)])
            cf[:, ~low] = 0
            mu[g.sphere_nodes(k)] = vsh.inverse(cf)
        a = rn.near_part(g, mu, a_s, a_d)
        b = ops.near_part(mu, a_s, a_d)
        errs.append(np.abs(a - b).max() / np.abs(b).max())
    # the difference is the band-limited projection of the near field on the target
    # (gap 0.5 here): geometric decay in p
    assert errs[1] < 0.2 * errs[0] and errs[2] < 0.2 * errs[1], errs
    assert errs[2] < 1e-3, errs


@pytest.mark.parametrize("radii", [(0.6, 1.3), (1.3, 0.6)])
def test_pair_on_the_pole_with_radii_is_the_projection_of_the_direct_series(radii):
    # spheres of radii a_s, a_t on the z axis with gap 0.4: the rotation is the identity
    # and the scheme reduces to projecting the direct series (evaluated at the target's
    # own nodes, which the radius-aware geometry places at c_t + a_t x) on the target
    a_s, a_t = radii
    c = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, a_s + a_t + 0.4]])
    g = Geometry(c, 6, near_gap=1.0, radii=list(radii))
    ops = Operators(g)
    vsh = DenseVSH(g.grid, g.p, g.mmax)
    mu = np.random.default_rng(31).standard_normal((g.N, 3))
    coef = vsh.forward(mu[g.sphere_nodes(0)])
    for op in ((1.0, 0.0), (0.0, 1.0)):
        got = rn.pair_coefficients(g, coef, c[1] - c[0], op[0], op[1], vsh, a_s, a_t)
        direct = ops.near_field_from(coef[:, :, None], c[0], g.nodes[g.sphere_nodes(1)], op[0], op[1], a_s)[..., 0]
        assert np.abs(got - vsh.forward(direct)).max() < 1e-13 * np.abs(got).max()


@pytest.mark.parametrize("op", [(1.0, 0.0), (0.0, 1.0)])
def test_converges_to_the_direct_series_with_radii(op):
    a_s, a_d = op
    rng = np.random.default_rng(32)
    d = rng.standard_normal(3)
    rad = np.array([0.7, 1.2])
    c = np.array([[0.0, 0.0, 0.0], (rad.sum() + 0.5) * d / np.linalg.norm(d)])
    errs = []
    for p in (6, 10, 14, 18):
        g = Geometry(c, p, near_gap=1.0, radii=rad)
        assert g.near[0, 1] and g.near[1, 0]
        ops = Operators(g)
        vsh = DenseVSH(g.grid, p, g.mmax)
        low = np.array([n <= 3 for (n, m) in vsh.modes])
        mu = np.random.default_rng(33).standard_normal((g.N, 3))
        for k in range(2):
            cf = vsh.forward(mu[g.sphere_nodes(k)])
            cf[:, ~low] = 0
            mu[g.sphere_nodes(k)] = vsh.inverse(cf)
        a = rn.near_part(g, mu, a_s, a_d)
        b = ops.near_part(mu, a_s, a_d)
        errs.append([np.abs(a - b)[g.sphere_nodes(k)].max() / np.abs(b[g.sphere_nodes(k)]).max() for k in range(2)])
    e = np.array(errs)
    # the difference is the projection error of the near field on each target: geometric
    # on the small target (radius 0.7, measured 2e-3 / 3e-2 at p = 6 down to 5e-8 / 9e-7 at
    # p = 18), slower and less regular on the large one, which sees a source of 0.58 its
    # radius at gap 0.42 of it (1e-1 / 2e-1 down to 4e-5 / 9e-4); a wrong radius scaling
    # would stall at O(1)
    assert (e[1:, 0] < 0.2 * e[:-1, 0]).all(), e
    assert e[3, 0] < 2e-6 and e[3, 1] < 2e-3 and e[3, 1] < 0.02 * e[0, 1], e


def test_scaling_a_configuration_with_radii():
    # centres and radii times lam: the single layer's near field scales by lam, the
    # double layer's is unchanged (same node values of the density)
    c = np.array([[0.0, 0.0, 0.0], [1.5, 0.6, 0.3], [-0.4, 1.4, 0.9]])
    rad = np.array([0.8, 0.55, 0.6])
    lam = 1.7
    g1 = Geometry(c, 6, near_gap=1.0, radii=rad)
    g2 = Geometry(lam * c, 6, near_gap=1.0, radii=lam * rad)
    assert (g1.near == g2.near).all() and g1.near.sum() >= 3
    mu = np.random.default_rng(34).standard_normal((g1.N, 3))
    s1, s2 = rn.near_part(g1, mu, 1.0, 0.0), rn.near_part(g2, mu, 1.0, 0.0)
    d1, d2 = rn.near_part(g1, mu, 0.0, 1.0), rn.near_part(g2, mu, 0.0, 1.0)
    assert np.abs(s2 - lam * s1).max() < 1e-12 * np.abs(s2).max()
    assert np.abs(d2 - d1).max() < 1e-12 * np.abs(d1).max()
