"""Pins for oracle/grid.py (Eqs. 4.2-4.4): quadrature facts that hold independently
of the oracle's own arithmetic."""
import math

import numpy as np
import pytest

from oracle.grid import Geometry, mmax_for, sphere_grid


@pytest.mark.parametrize("p", [1, 2, 4, 8, 12, 16])
def test_area_and_unit_nodes(p):
    g = sphere_grid(p)
    assert g["xhat"].shape == ((p + 1) * 2 * p, 3)
    assert abs(g["wnode"].sum() - 4 * math.pi) < 1e-13
    assert np.abs(np.linalg.norm(g["xhat"], axis=1) - 1).max() < 1e-15
    assert np.all(np.diff(g["theta"]) > 0)


def test_gauss_legendre_two_point_closed_form():
    g = sphere_grid(1)
    assert np.allclose(g["t"], [1 / math.sqrt(3), -1 / math.sqrt(3)], atol=1e-15)
    assert np.allclose(g["lam"], [1.0, 1.0], atol=1e-15)


@pytest.mark.parametrize("p", [4, 8, 12])
def test_polynomial_moments(p):
    # sphere moments of monomials: int x^2 = 4pi/3, int x^4 = 4pi/5, int x^2 y^2 = 4pi/15,
    # int x^2 y^2 z^2 = 4pi/105, odd moments vanish
    g = sphere_grid(p)
    x, y, z = g["xhat"].T
    w = g["wnode"]
    assert abs(w @ (x * x) - 4 * math.pi / 3) < 1e-13
    assert abs(w @ (z ** 4) - 4 * math.pi / 5) < 1e-13
    assert abs(w @ (x * x * y * y) - 4 * math.pi / 15) < 1e-13
    assert abs(w @ (x * x * y * y * z * z) - 4 * math.pi / 105) < 1e-13
    assert abs(w @ (x * y * z * z)) < 1e-14
    assert abs(w @ (x ** 3)) < 1e-14


def test_azimuthal_band_limit():
    assert mmax_for(8, 16) == 7
    assert mmax_for(8, 18) == 8
    assert mmax_for(12, 24) == 11


def test_geometry_near_classification():
    c = np.array([[0, 0, 0], [2.5, 0, 0], [0, 3.2, 0], [10, 0, 0]], dtype=float)
    g = Geometry(c, 4, near_gap=1.0)
    # gaps: 0.5 (near), 1.2 (far), 6 (far)
    assert g.near[0, 1] and g.near[1, 0]
    assert not g.near[0, 2] and not g.near[0, 3]
    assert not g.near[0, 0]
    assert g.N == 4 * 5 * 8
