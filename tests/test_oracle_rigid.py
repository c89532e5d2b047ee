"""Pins of the rigid-mode coarse correction oracle (oracle/rigid.py) against the oracle's
operator, brute-force surface quadrature and the isolated-sphere inverse."""
import math

import numpy as np
import pytest

from oracle import rigid
from oracle.grid import Geometry
from oracle.kernels import kernel_block
from oracle.operators import Operators
from oracle.precond import m0_resistance


def _rap(c, p):
    """R A P of the completed double-layer operator, column by column."""
    g = Geometry(c, p, near_gap=1.0)
    ops = Operators(g)
    xh, w = g.grid["xhat"], g.grid["wnode"]
    cols = []
    for k in range(g.nb):
        for m in range(6):
            y = np.zeros(6)
            y[m] = 1.0
            f = np.zeros((g.N, 3))
            f[g.sphere_nodes(k)] = rigid.prolong(y, xh)
            u = ops.apply("DN_BIE", f)
            cols.append(np.concatenate([rigid.restrict(u[g.sphere_nodes(i)], xh, w) for i in range(g.nb)]))
    return np.array(cols).T, g


def test_restriction_of_the_operator_is_the_one_sided_closed_form():
    # separated spheres: far field only
    c = np.array([[0.0, 0.0, 0.0], [3.1, 0.4, 0.2], [0.3, -2.6, 1.5]])
    rap, g = _rap(c, 10)
    assert g.near.sum() == 0
    one = rigid.coarse_operator(c, two_sided=False)
    assert np.abs(rap - one).max() < 1e-7 * np.abs(one).max()
    # a near pair (gap 0.4 < d*): the near series of a rigid density vanishes, the
    # completion flow is evaluated pointwise; only quadrature error remains
    c2 = np.array([[0.0, 0.0, 0.0], [2.4, 0.0, 0.0], [0.5, 3.3, -0.7]])
    rap2, g2 = _rap(c2, 12)
    assert g2.near.sum() > 0
    one2 = rigid.coarse_operator(c2, two_sided=False)
    assert np.abs(rap2 - one2).max() < 1e-5 * np.abs(one2).max()
    # the two-sided (Rotne-Prager) operator differs only in the translation blocks
    two2 = rigid.coarse_operator(c2, two_sided=True)
    mask = np.ones((18, 18), bool)
    for i in range(3):
        for k in range(3):
            mask[6 * i:6 * i + 3, 6 * k:6 * k + 3] = False
    assert np.abs((two2 - one2)[mask]).max() < 1e-15


@pytest.mark.parametrize("d", [2.3, 3.0, 5.0])
def test_translation_block_is_the_two_sided_surface_average(d):
    # mean over both unit spheres of the Stokeslet (brute-force quadrature, fine grid)
    g = Geometry(np.zeros((1, 3)), 24, near_gap=1.0)
    xh, w = g.grid["xhat"], g.grid["wnode"]
    e = np.array([0.36, -0.48, 0.8])
    x = d * e + xh
    K = kernel_block(x, xh, xh, 1.0, 0.0)                  # (T, 3, S, 3)
    avg = np.einsum("t,tisj,s->ij", w, K, w) / (4 * math.pi) ** 2
    M = rigid.mobility(np.stack([d * e, np.zeros(3)]))
    assert np.abs(M[0:3, 6:9] - avg).max() < 1e-10
    # the one-sided average (target sphere only, point force at the source centre)
    Kc = kernel_block(x, np.zeros((1, 3)), np.zeros((1, 3)), 1.0, 0.0)[:, :, 0, :]
    avg1 = np.einsum("t,tij->ij", w, Kc) / (4 * math.pi)
    M1 = rigid.mobility(np.stack([d * e, np.zeros(3)]), two_sided=False)
    assert np.abs(M1[0:3, 6:9] - avg1).max() < 1e-10


def test_restrict_prolong_and_m0_on_rigid_modes():
    g = Geometry(np.zeros((1, 3)), 8, near_gap=1.0)
    xh, w = g.grid["xhat"], g.grid["wnode"]
    rng = np.random.default_rng(0)
    y = rng.standard_normal(6)
    assert np.abs(rigid.restrict(rigid.prolong(y, xh), xh, w) - y).max() < 1e-13
    # R M0 P = diag(3/2, 3) = inverse of the isolated coarse block
    z = m0_resistance(g, rigid.prolong(y, xh))
    assert np.abs(rigid.restrict(z, xh, w) - rigid.B0 * y).max() < 1e-12
    Ac = rigid.coarse_operator(np.zeros((1, 3)))
    assert np.abs(np.linalg.inv(Ac) - np.diag(rigid.B0)).max() < 1e-13
    # a field with no rigid part restricts to zero (degree-2 and V_1 modes)
    f = np.stack([xh[:, 0] * xh[:, 1], xh[:, 2] ** 2 - 1 / 3, xh[:, 0]], 1) + (np.array([1, 2, 3]) - 3 * (xh @ [1, 2, 3])[:, None] * xh)
    f = f - rigid.prolong(rigid.restrict(f, xh, w), xh)
    assert np.abs(rigid.restrict(f, xh, w)).max() < 1e-13


def test_correction_is_a_no_op_on_an_isolated_sphere():
    g = Geometry(np.array([[1.0, -2.0, 0.5]]), 6, near_gap=1.0)
    r = np.random.default_rng(1).standard_normal((g.N, 3))
    z0 = m0_resistance(g, r)
    assert np.abs(rigid.correct(g, r, z0) - z0).max() < 1e-12


def test_rotne_prager_mobility_is_positive_definite():
    from paper_1707_06551_amd.inputs import box_side, place_spheres
    rng = np.random.default_rng(2)
    dense = None
    for n, phi, gap in ((60, 0.25, 0.02), (40, 0.10, 0.001)):
        c = place_spheres(n, box_side(n, phi), gap, rng)
        dense = c if dense is None else dense
        M = rigid.mobility(c)
        assert np.abs(M - M.T).max() < 1e-16
        assert np.linalg.eigvalsh(M).min() > 0
    # the one-sided restriction is indefinite in a dense suspension (why it is not used)
    assert np.linalg.eigvalsh(rigid.mobility(dense, two_sided=False)).min() < 0
