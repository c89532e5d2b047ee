"""GPU parity of the Laplace operators and the magnetostatic problem (Problem 3) against
the oracle (oracle/laplace.py) and the textbook magnetisable sphere."""
import numpy as np
import pytest

from oracle import laplace
from oracle.grid import Geometry
from tests.gpu_common import assert_close, poly_cluster, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cluster():
    from paper_1707_06551_amd import bie
    c = small_cluster(10, 7.0, 0.05, 21)
    p = 5
    s = bie.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    yield c, s, g
    s.close()


def test_magnetic_operator_matches_oracle(cluster):
    c, s, g = cluster
    assert g.near.sum() > 0
    lap = laplace.Laplace(g)
    q = np.random.default_rng(1).standard_normal(g.N)
    out = host(s.apply_laplace(0, dev(q), eta=0.6))
    ref = lap.magnetic_bie(q, 0.6)
    assert_close(out, ref, 1e-11)


def test_gradient_matches_oracle(cluster):
    c, s, g = cluster
    lap = laplace.Laplace(g)
    q = np.random.default_rng(2).standard_normal(g.N)
    out = host(s.apply_laplace(1, dev(q))).reshape(g.N, 3)
    _v, ref = lap.potential_and_gradient(q)
    assert_close(out, ref, 1e-11)


def test_gradient_on_a_grid_of_more_than_1024_nodes():
    # p = 16 on 64 longitudes: 1088 nodes per sphere, more than one work-group of threads
    # in the near-series kernel
    from paper_1707_06551_amd import bie
    c = small_cluster(3, 5.0, 0.2, 14)
    s = bie.Spheres(c, 16, n_phi=64, near_gap=1.0)
    g = Geometry(c, 16, n_phi=64, near_gap=1.0)
    assert g.P == 1088 and g.near.any()
    q = np.random.default_rng(3).standard_normal(g.N)
    out = host(s.apply_laplace(1, dev(q))).reshape(g.N, 3)
    _v, ref = laplace.Laplace(g).potential_and_gradient(q)
    assert_close(out, ref, 1e-11)
    s.close()


def test_magnetisable_sphere():
    from paper_1707_06551_amd import bie
    mu = 5.0
    eta = (mu - 1) / (mu + 1)
    H0 = np.array([0.2, 0.9, -0.4])
    s = bie.Spheres(np.array([[1.0, 2.0, 3.0]]), 6, near_gap=1.0)
    F, T, q, info = s.solve_magnetic(H0, eta, tol=1e-13, want_q=True)
    assert info["converged"], info
    xyz, _w = s.nodes()
    n = xyz - np.array([1.0, 2.0, 3.0])
    assert np.abs(host(q) - 6 * eta / (3 - eta) * (n @ H0)).max() < 1e-11
    assert np.abs(F).max() < 1e-11 and np.abs(T).max() < 1e-11
    s.close()


def test_magnetic_forces_match_oracle_and_move_the_spheres():
    from paper_1707_06551_amd import bie
    c = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 2.6], [2.9, 0.4, 0.8]])
    p = 5
    eta = 0.5
    H0 = np.array([0.0, 0.0, 1.0])
    s = bie.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    F, T, q, info = s.solve_magnetic(H0, eta, tol=1e-13, want_q=True)
    assert info["converged"], info
    q_ref, F_ref, T_ref, _H = laplace.solve_magnetic(g, H0, eta)
    assert_close(host(q), q_ref, 1e-10)
    assert_close(F, F_ref, 1e-9)
    assert_close(T, T_ref, 1e-8)
    # Problem 3: the loads drive the mobility problem; the pair stacked along the field
    # attracts, so spheres 0 and 1 approach each other
    v, om, _mu, info2 = s.solve_mobility(F, T, tol=1e-10, precond=bie.PC_M0)
    assert info2["converged"], info2
    d = c[1] - c[0]
    assert np.dot(v[1] - v[0], d) < 0
    s.close()


@pytest.fixture(scope="module")
def poly():
    # six spheres of radii 0.35-1.4 with near pairs between unequal radii
    from paper_1707_06551_amd import bie
    c, a = poly_cluster()
    p = 5
    s = bie.Spheres(c, p, near_gap=1.0, radii=a)
    g = Geometry(c, p, near_gap=1.0, radii=a)
    yield c, a, s, g
    s.close()


def test_laplace_operators_with_radii_match_oracle(poly):
    c, a, s, g = poly
    assert g.near.sum() > 0
    lap = laplace.Laplace(g)
    q = np.random.default_rng(3).standard_normal(g.N)
    out = host(s.apply_laplace(0, dev(q), eta=0.6))
    ref = lap.magnetic_bie(q, 0.6)
    assert_close(out, ref, 1e-11)
    grad = host(s.apply_laplace(1, dev(q))).reshape(g.N, 3)
    _v, gref = lap.potential_and_gradient(q)
    assert_close(grad, gref, 1e-11)


def test_magnetic_problem_with_radii_matches_oracle(poly):
    c, a, s, g = poly
    H0 = np.array([0.3, -0.2, 1.0])
    F, T, q, info = s.solve_magnetic(H0, 0.5, tol=1e-13, want_q=True)
    assert info["converged"], info
    q_ref, F_ref, T_ref, _H = laplace.solve_magnetic(g, H0, 0.5)
    assert_close(host(q), q_ref, 1e-10)
    assert_close(F, F_ref, 1e-9)
    assert_close(T, T_ref, 1e-8)


@pytest.mark.parametrize("rad", [0.3, 2.5])
def test_magnetisable_sphere_of_radius_a(rad):
    # the density 6 eta / (3 - eta) n . H0 does not depend on the radius; no net load
    from paper_1707_06551_amd import bie
    eta = 0.6
    H0 = np.array([0.2, 0.9, -0.4])
    s = bie.Spheres(np.array([[1.0, 2.0, 3.0]]), 6, near_gap=1.0, radii=[rad])
    F, T, q, info = s.solve_magnetic(H0, eta, tol=1e-13, want_q=True)
    assert info["converged"], info
    xyz, _w = s.nodes()
    n = (xyz - np.array([1.0, 2.0, 3.0])) / rad
    assert np.abs(host(q) - 6 * eta / (3 - eta) * (n @ H0)).max() < 1e-11
    assert np.abs(F).max() < 1e-11 * rad ** 2 and np.abs(T).max() < 1e-11 * rad ** 3
    s.close()
