"""Pins for oracle/coarse.py, oracle/mlp.py and oracle/precond.py (learned coarse
correction): basis facts, equivariance, adjointness, finite-difference gradients, and
M0 as the exact inverse of the isolated-sphere operator."""
import math

import numpy as np
import pytest

from oracle import coarse, mlp
from oracle.grid import Geometry, sphere_grid
from oracle.harmonics import DenseVSH
from oracle.operators import Operators
from oracle.precond import m0_resistance


def _rand_rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("p", [3, 6])
def test_restrict_prolong_identity_and_span(p):
    g = sphere_grid(p)
    rng = np.random.default_rng(0)
    rho = rng.standard_normal(coarse.NLOW)
    f = coarse.prolong(rho, g["xhat"])
    assert np.abs(coarse.restrict(f, g["xhat"], g["wnode"]) - rho).max() < 1e-12
    # the 25 fields lie in the span of V, W, X of degree <= 2
    vsh = DenseVSH(g, p, min(p, g["n_phi"] // 2 - 1))
    c = vsh.forward(f)
    high = np.array([n > 2 for (n, m) in vsh.modes])
    assert np.abs(c[:, high]).max() < 1e-12
    # and span it: 1 + 9 + 15 = 25 independent fields
    F = coarse.lowmode_fields(g["xhat"]).transpose(1, 0, 2).reshape(25, -1)
    assert np.linalg.matrix_rank(F) == 25


def test_theta_adjoint_and_axisymmetry():
    rng = np.random.default_rng(1)
    th = rng.standard_normal(coarse.NTHETA)
    dK = rng.standard_normal((25, 25))
    K = coarse.K_from_theta(th)
    assert abs(np.sum(K * dK) - th @ coarse.theta_grad_from_K(dK)) < 1e-12
    for phi in (0.3, 1.7, -2.2):
        Rz = np.array([[math.cos(phi), -math.sin(phi), 0], [math.sin(phi), math.cos(phi), 0], [0, 0, 1]])
        Rm = coarse.rot25(Rz)
        assert np.abs(Rm @ K - K @ Rm).max() < 1e-12


def test_rot25_is_the_rotation_of_the_fields():
    # rotating a low-mode field by G equals rotating its 25 coefficients by rot25(G)
    rng = np.random.default_rng(2)
    g = sphere_grid(5)
    G = _rand_rot(rng)
    rho = rng.standard_normal(25)
    x = g["xhat"]
    f_rot = (G @ coarse.prolong(rho, x @ G).T).T           # (G f)(G^T x)
    assert np.abs(coarse.restrict(f_rot, x, g["wnode"]) - coarse.rot25(G) @ rho).max() < 1e-12


def _cluster():
    return np.array([[0.0, 0.0, 0.0], [2.1, 0.3, -0.2], [0.5, 2.15, 0.4], [2.6, 2.4, 0.1], [-1.2, 1.0, 1.9]])


def test_correction_is_rotation_equivariant_and_frame_independent():
    rng = np.random.default_rng(3)
    c = _cluster()
    g = Geometry(c, 4, near_gap=1.0)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    w = mlp.init_weights(4, out_scale=1.0)
    theta, _ = mlp.forward(w, feats)
    rho = rng.standard_normal((g.nb, 25))
    z = coarse.coarse_apply(pairs, dirs, theta, rho)
    G = _rand_rot(rng)
    c2 = c @ G.T
    g2 = Geometry(c2, 4, near_gap=1.0)
    pairs2, feats2, dirs2 = coarse.pair_features(c2, g2.near, 1.0)
    assert np.array_equal(pairs, pairs2) and np.abs(feats - feats2).max() < 1e-12
    theta2, _ = mlp.forward(w, feats2)
    R25 = coarse.rot25(G)
    z2 = coarse.coarse_apply(pairs2, dirs2, theta2, rho @ R25.T)
    assert np.abs(z2 - z @ R25.T).max() < 1e-10
    # any transverse axes of the pair frame give the same block (axisymmetric K)
    e = 0
    Q = coarse.pair_frame(dirs[e])
    phi = 0.8
    Rz = np.array([[math.cos(phi), -math.sin(phi), 0], [math.sin(phi), math.cos(phi), 0], [0, 0, 1]])
    Ko = coarse.K_from_theta(theta[e, :coarse.NTHETA])
    b1 = coarse.rot25(Q).T @ Ko @ coarse.rot25(Q)
    b2 = coarse.rot25(Rz @ Q).T @ Ko @ coarse.rot25(Rz @ Q)
    assert np.abs(b1 - b2).max() < 1e-12


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    c = _cluster()
    g = Geometry(c, 4, near_gap=1.0)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    data = [dict(pairs=pairs, feats=feats, dirs=dirs, xi=rng.standard_normal((2, g.nb, 25)),
                 t=rng.standard_normal((2, g.nb, 25)))]
    w = mlp.init_weights(7, out_scale=0.3)
    L, grad = mlp.loss_and_grad(w, data)
    idx = rng.choice(w.size, 40, replace=False)
    for k in idx:
        h = 1e-6
        wp = w.copy()
        wp[k] += h
        wm = w.copy()
        wm[k] -= h
        fd = (mlp.loss_and_grad(wp, data)[0] - mlp.loss_and_grad(wm, data)[0]) / (2 * h)
        assert abs(fd - grad[k]) < 1e-7 * max(1.0, abs(fd)), (k, fd, grad[k])


def test_m0_inverts_the_isolated_resistance_operator():
    g = Geometry(np.zeros((1, 3)), 6)
    ops = Operators(g)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((g.N, 3))
    z = m0_resistance(g, r)
    assert np.abs(ops.apply("DN_BIE", z) - r).max() < 1e-12
