"""GPU parity of the fluid-point evaluation (bie_eval_field) and the porous-media solve
(Problem 1, bie_solve with BIE_OP_SD_BIE) against the oracle (oracle/field.py) and the
textbook flow past a fixed sphere."""
import numpy as np
import pytest

from oracle import field
from oracle.grid import Geometry
from oracle.operators import Operators
from oracle.solvers import assemble
from paper_1707_06551_amd.inputs import lattice_centres
from tests.gpu_common import assert_close, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS = {"S": 1, "D": 2, "SD_BIE": 3, "DN_BIE": 4}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def fluid_points(c, n, rng, gaps=(0.02, 0.3, 0.9, 1.5, 4.0)):
    """Points at given distances from the surfaces of random spheres, kept outside all."""
    pts = []
    while len(pts) < n:
        k = rng.integers(len(c))
        d = rng.standard_normal(3)
        x = c[k] + (1.0 + gaps[len(pts) % len(gaps)]) * d / np.linalg.norm(d)
        if (np.linalg.norm(c - x[None, :], axis=1) > 1.001).all():
            pts.append(x)
    return np.array(pts)


@pytest.mark.parametrize("opname", list(OPS))
def test_field_matches_oracle(opname):
    from paper_1707_06551_amd import bie
    c = small_cluster(9, 7.5, 0.1, 13)
    p = 6
    s = bie.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    rng = np.random.default_rng(5)
    mu = rng.standard_normal((g.N, 3))
    x = fluid_points(c, 60, rng)
    out = host(s.eval_field(OPS[opname], dev(mu), x)).reshape(-1, 3)
    ref = field.evaluate(g, mu, x, opname)
    assert_close(out, ref, 1e-11)
    s.close()


def test_point_inside_a_sphere_is_an_error():
    from paper_1707_06551_amd import bie
    c = small_cluster(4, 6.0, 0.3, 2)
    s = bie.Spheres(c, 4, near_gap=1.0)
    x = np.concatenate([fluid_points(c, 5, np.random.default_rng(1)), c[:1] + 0.5])
    u = torch.zeros(3 * len(x), dtype=torch.float64, device="cuda")
    with pytest.raises(bie.BieError):
        s.eval_field(bie.OP_SD_BIE, dev(np.ones((s.N, 3))), x, u=u)
    v = host(u).reshape(-1, 3)
    assert np.isfinite(v[:5]).all() and np.isnan(v[5]).all()
    s.close()


def test_flow_past_a_fixed_sphere():
    # Problem 1 with one sphere: solve (1/2 + S + D) mu = -U, then u = U + (S + D)[mu]
    from paper_1707_06551_amd import bie
    c = np.array([[0.3, -0.2, 0.5]])
    U = np.array([0.4, -1.1, 0.7])
    s = bie.Spheres(c, 12, near_gap=1.0)
    b = dev(np.tile(-U, s.N))
    for precision, precond in ((bie.FP64, bie.PC_NONE), (bie.MIXED, bie.PC_M0)):
        mu, info = s.solve(bie.OP_SD_BIE, b, tol=1e-12 if precision == bie.FP64 else 1e-10,
                           precision=precision, precond=precond)
        assert info["converged"], info
        rng = np.random.default_rng(1)
        d = rng.standard_normal((6, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        x = c[0] + np.array([1.02, 1.3, 1.9, 2.2, 3.5, 8.0])[:, None] * d
        u = U[None, :] + host(s.eval_field(bie.OP_SD_BIE, mu, x)).reshape(-1, 3)
        r = x - c[0]
        dd = np.linalg.norm(r, axis=1)[:, None]
        rU = (r @ U)[:, None]
        ref = U - 0.75 * (U / dd + rU * r / dd ** 3) - 0.25 * (U / dd ** 3 - 3 * rU * r / dd ** 5)
        err = np.abs(u - ref).max(axis=1)
        assert err[:3].max() < 1e-9, err     # exterior series
        assert err[3:].max() < 3e-8, err     # smooth quadrature, p = 12
    s.close()


def test_porous_media_solve_matches_oracle_lu():
    # flow through the 2 x 2 x 2 densely packed lattice (gap 2/15, near series active)
    from paper_1707_06551_amd import bie
    c = lattice_centres(1, 4)
    p = 5
    s = bie.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    ops = Operators(g)
    U = np.array([1.0, 0.2, -0.4])
    A = assemble(lambda m: ops.apply("SD_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    mu_ref = np.linalg.solve(A, -np.tile(U, g.N))
    mu, info = s.solve(bie.OP_SD_BIE, dev(np.tile(-U, g.N)), tol=1e-12, precond=bie.PC_M0)
    assert info["converged"], info
    assert_close(host(mu), mu_ref, 1e-10)
    x = fluid_points(c, 30, np.random.default_rng(3), gaps=(0.01, 0.05, 0.5, 2.0))
    u = host(s.eval_field(bie.OP_SD_BIE, mu, x)).reshape(-1, 3)
    ref = field.evaluate(g, mu_ref.reshape(g.N, 3), x, "SD_BIE", ops)
    assert_close(u, ref, 1e-9)
    s.close()


def test_sd_block_preconditioner_inverts_an_isolated_sphere():
    from paper_1707_06551_amd import bie
    s = bie.Spheres(np.array([[1.0, 2.0, -0.5]]), 7, near_gap=1.0)
    r = dev(np.random.default_rng(2).standard_normal(3 * s.N))
    z = s.apply_precond(bie.OP_SD_BIE, r, precond=bie.PC_M0)
    back = host(s.apply(bie.OP_SD_BIE, z))
    assert_close(back, host(r), 1e-12)
    s.close()
