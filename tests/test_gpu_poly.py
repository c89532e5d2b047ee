"""GPU parity of the polydisperse operators (spheres of several radii: S, D, S + D, K and
the porous-media solve) against the oracle with per-sphere radii (oracle/grid.py,
oracle/operators.py, oracle/traction.py)."""
import math

import numpy as np
import pytest

from oracle import traction as tr
from oracle.grid import Geometry
from oracle.operators import OPS as ORACLE_OPS, Operators
from oracle.solvers import assemble
from tests.gpu_common import assert_close, poly_cluster, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS = {"S": 1, "D": 2, "SD_BIE": 3, "DN_BIE": 4}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cluster():
    from paper_1707_06551_amd import bie
    c, a = poly_cluster()
    p = 6
    s = bie.Spheres(c, p, near_gap=1.0, radii=a)
    g = Geometry(c, p, near_gap=1.0, radii=a)
    yield c, a, s, g
    s.close()


def test_nodes_and_near_pairs(cluster):
    c, a, s, g = cluster
    xyz, w = s.nodes()
    assert np.abs(xyz - g.nodes).max() < 1e-14 and np.abs(w - g.w).max() < 1e-15
    pairs = s.near_pairs()
    ref = sorted((t, q) for t in range(g.nb) for q in range(g.nb) if g.near[t, q])
    assert sorted(map(tuple, pairs.T.tolist())) == ref
    assert not np.array_equal(g.near, g.near.T)   # the radius-scaled test is directed


@pytest.mark.parametrize("opname", ["S", "D", "SD_BIE", "DN_BIE"])
@pytest.mark.parametrize("precision", [0, 1])
def test_operators_match_oracle(cluster, opname, precision):
    c, a, s, g = cluster
    ops = Operators(g)
    mu = np.random.default_rng(1).standard_normal((g.N, 3))
    out = host(s.apply(OPS[opname], dev(mu), precision=precision)).reshape(g.N, 3)
    ref = ops.apply(opname, mu)
    tol = 1e-11 if precision == 0 else 1e-6
    assert_close(out, ref, tol)


@pytest.mark.parametrize("stage", ["self", "near", "far"])
def test_stages_match_oracle(cluster, stage):
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    ops = Operators(g)
    mu = np.random.default_rng(2).standard_normal((g.N, 3))
    bits = {"self": bie.STAGE_SELF, "near": bie.STAGE_NEAR, "far": bie.STAGE_FAR}[stage]
    out = host(s.apply(bie.OP_SD_BIE | bits, dev(mu))).reshape(g.N, 3)
    if stage == "self":
        ref = ops.self_part(mu, 1.0, 1.0) + 0.5 * mu
    elif stage == "near":
        ref = ops.near_part(mu, 1.0, 1.0)
    else:
        ref = ops.far_part(mu, 1.0, 1.0)
    assert_close(out, ref, 1e-11)


@pytest.mark.parametrize("precision", [0, 1])
def test_traction_matches_oracle(cluster, precision):
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    mu = np.random.default_rng(3).standard_normal((g.N, 3))
    out = host(s.apply(bie.OP_K, dev(mu), precision=precision)).reshape(g.N, 3)
    ref = tr.TractionOps(g).apply_K(mu)
    tol = 1e-11 if precision == 0 else 1e-6
    assert_close(out, ref, tol)


def test_scaled_configuration(cluster):
    # scaling all centres and radii by lam multiplies S by lam and leaves D, K unchanged
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    lam = 1.7
    s2 = bie.Spheres(lam * c, g.p, near_gap=1.0, radii=lam * a)
    mu = dev(np.random.default_rng(4).standard_normal(3 * g.N))
    for op, f in ((bie.OP_S, lam), (bie.OP_D, 1.0), (bie.OP_K, 1.0)):
        u1 = host(s.apply(op, mu))
        u2 = host(s2.apply(op, mu))
        assert_close(u2, f * u1, 1e-12)
    s2.close()


def test_unit_radii_take_the_monodisperse_path():
    from paper_1707_06551_amd import bie
    c, _a = poly_cluster()
    s0 = bie.Spheres(1.5 * c, 5, near_gap=1.0)
    s1 = bie.Spheres(1.5 * c, 5, near_gap=1.0, radii=np.ones(len(c)))
    mu = dev(np.random.default_rng(5).standard_normal(3 * s0.N))
    for op in (bie.OP_SD_BIE, bie.OP_DN_BIE):
        assert np.array_equal(host(s0.apply(op, mu)), host(s1.apply(op, mu)))
    s0.close()
    s1.close()


@pytest.mark.parametrize("op", [3, 4])
def test_m0_inverts_an_isolated_sphere_of_radius_a(op):
    from paper_1707_06551_amd import bie
    for a in (0.4, 2.5):
        s = bie.Spheres(np.array([[0.2, 0.1, -0.3]]), 7, radii=[a])
        mu = np.random.default_rng(6).standard_normal(3 * s.N)
        z = host(s.apply_precond(op, s.apply(op, dev(mu)), precond=bie.PC_M0))
        assert_close(z, mu, 1e-12)
        s.close()


def test_resistance_of_an_isolated_sphere_of_radius_a():
    # Problem 5: F = 6 pi a v, T = 8 pi a^3 omega
    from paper_1707_06551_amd import bie
    a = 0.45
    s = bie.Spheres(np.array([[0.5, 0.2, -1.0]]), 6, radii=[a])
    v = np.array([[0.3, -1.0, 0.8]])
    om = np.array([[1.1, 0.2, -0.5]])
    F, T, _psi, info = s.solve_resistance(v, om, tol=1e-13, precond=bie.PC_M0)
    assert info["converged"], info
    assert np.abs(F - 6 * math.pi * a * v).max() < 1e-11
    assert np.abs(T - 8 * math.pi * a ** 3 * om).max() < 1e-11
    s.close()


def test_resistance_matches_oracle(cluster):
    from oracle import solvers
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    rng = np.random.default_rng(8)
    v = rng.standard_normal((g.nb, 3))
    om = rng.standard_normal((g.nb, 3))
    F, T, psi, info = s.solve_resistance(v, om, tol=1e-12, precond=bie.PC_M0, want_psi=True)
    assert info["converged"], info
    F_o, T_o, psi_o, _i = solvers.solve_resistance(g, v, om, method="lu")
    assert_close(F, F_o, 1e-9)
    assert_close(T, T_o, 1e-9)
    assert_close(host(psi).reshape(g.N, 3), psi_o, 1e-8)
    F2, T2, _p, info2 = s.solve_resistance(v, om, tol=1e-10, precision=bie.MIXED, precond=bie.PC_M0)
    assert info2["converged"], info2
    assert_close(F2, F_o, 1e-8)
    assert_close(T2, T_o, 1e-8)
    print(f"polydisperse resistance, 6 spheres p = 6: GMRES {info['iters']} (M0), mixed {info2['iters']}")


def test_bordered_mobility_operator_and_m0(cluster):
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    ops = Operators(g)
    x = np.random.default_rng(10).standard_normal(3 * g.N + 6 * g.nb)
    out = host(s.apply(bie.OP_MOBILITY, dev(x)))
    ref = ops.apply_mobility(x)
    assert_close(out, ref, 1e-11)
    for rad in (0.4, 2.5):
        s1 = bie.Spheres(np.array([[0.2, 0.1, -0.3]]), 7, radii=[rad])
        y = np.random.default_rng(11).standard_normal(3 * s1.N + 6)
        z = host(s1.apply_precond(bie.OP_MOBILITY, s1.apply(bie.OP_MOBILITY, dev(y)), precond=bie.PC_M0))
        assert_close(z, y, 1e-12)
        s1.close()


def test_mobility_matches_oracle(cluster):
    from oracle import solvers
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    rng = np.random.default_rng(12)
    F = rng.standard_normal((g.nb, 3))
    T = rng.standard_normal((g.nb, 3))
    v, om, _mu, info = s.solve_mobility(F, T, tol=1e-12, precond=bie.PC_M0)
    assert info["converged"], info
    v_o, om_o, _mu_o, _i = solvers.solve_mobility(g, F, T, method="lu")
    assert_close(v, v_o, 1e-9)
    assert_close(om, om_o, 1e-9)
    v2, om2, _m2, info2 = s.solve_mobility(F, T, tol=1e-10, precision=bie.MIXED, precond=bie.PC_M0)
    assert info2["converged"], info2
    assert_close(v2, v_o, 1e-8)
    assert_close(om2, om_o, 1e-8)
    print(f"polydisperse mobility, 6 spheres p = 6: GMRES {info['iters']} (M0), mixed {info2['iters']}")
    # an isolated sphere of radius a: v = F / (6 pi a), omega = T / (8 pi a^3)
    s1 = bie.Spheres(np.array([[1.0, 2.0, 3.0]]), 6, radii=[0.7])
    v1, o1, _m, i1 = s1.solve_mobility(F[:1], T[:1], tol=1e-13, precond=bie.PC_M0)
    assert np.abs(v1 - F[:1] / (6 * math.pi * 0.7)).max() < 1e-12
    assert np.abs(o1 - T[:1] / (8 * math.pi * 0.7 ** 3)).max() < 1e-12
    s1.close()


def test_traction_form_with_radii(cluster):
    # 1/2 I + K + L and Problem 2 in the paper's form (Eqs. 5.7-5.8) on spheres of radii
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    to = tr.TractionOps(g)
    mu = np.random.default_rng(13).standard_normal((g.N, 3))
    out = host(s.apply(bie.OP_KL_BIE, dev(mu))).reshape(g.N, 3)
    ref = to.apply_KL_BIE(mu)
    assert_close(out, ref, 1e-11)
    for rad in (0.4, 2.5):
        s1 = bie.Spheres(np.array([[0.2, 0.1, -0.3]]), 7, radii=[rad])
        y = np.random.default_rng(14).standard_normal(3 * s1.N)
        z = host(s1.apply_precond(bie.OP_KL_BIE, s1.apply(bie.OP_KL_BIE, dev(y)), precond=bie.PC_M0))
        assert_close(z, y, 1e-12)
        F1 = np.array([[0.7, -0.2, 1.1]])
        T1 = np.array([[0.1, 0.9, -0.6]])
        v1, o1, _m, i1 = s1.solve_mobility_traction(F1, T1, tol=1e-13)
        assert np.abs(v1 - F1 / (6 * math.pi * rad)).max() < 1e-12
        assert np.abs(o1 - T1 / (8 * math.pi * rad ** 3)).max() < 1e-12
        s1.close()
    rng = np.random.default_rng(15)
    F = rng.standard_normal((g.nb, 3))
    T = rng.standard_normal((g.nb, 3))
    v, om, mu_d, info = s.solve_mobility_traction(F, T, tol=1e-12, want_mu=True)
    assert info["converged"], info
    v_o, om_o, mu_o, _i = tr.solve_mobility_traction(g, F, T, tol=1e-12)
    assert_close(v, v_o, 1e-9)
    assert_close(om, om_o, 1e-9)
    assert_close(host(mu_d).reshape(g.N, 3), mu_o, 1e-8)
    print(f"polydisperse traction-form mobility, 6 spheres p = 6: GMRES {info['iters']}")


@pytest.mark.parametrize("opname", ["SD_BIE", "DN_BIE"])
def test_fluid_points_match_oracle(cluster, opname):
    # points near every sphere (series) and away from them (quadrature), with radii
    from oracle import field
    c, a, s, g = cluster
    rng = np.random.default_rng(16)
    pts = []
    for k in range(g.nb):
        d = rng.standard_normal((6, 3))
        d /= np.linalg.norm(d, axis=1)[:, None]
        pts.append(c[k] + a[k] * (1.02 + 2.5 * rng.random(6))[:, None] * d)
    x = np.concatenate(pts)
    gap = np.linalg.norm(x[:, None, :] - c[None, :, :], axis=-1) - a[None, :]
    x = x[gap.min(axis=1) > 0.01]
    mu = rng.standard_normal((g.N, 3))
    out = host(s.eval_field(OPS[opname], dev(mu), x)).reshape(-1, 3)
    ref = field.evaluate(g, mu, x, opname)
    assert_close(out, ref, 1e-11)


def test_rigid_coarse_correction_with_radii(cluster):
    # the global rigid-mode correction (polydisperse Rotne-Prager-Yamakawa coarse
    # operator) against the oracle's dense coarse solve, its no-op on isolated spheres,
    # and the resistance solve it preconditions
    from oracle import rigid
    from oracle.precond import m0_resistance
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    r = np.random.default_rng(17).standard_normal((g.N, 3))
    z = host(s.apply_precond(bie.OP_DN_BIE, dev(r), precond=bie.PC_M0 | bie.PC_RIGID)).reshape(g.N, 3)
    ref = rigid.correct(g, r, m0_resistance(g, r))
    assert_close(z, ref, 1e-6)
    z0 = host(s.apply_precond(bie.OP_DN_BIE, dev(r), precond=bie.PC_M0)).reshape(g.N, 3)
    assert rel_err(z, z0) > 1e-3
    for rad in (0.4, 2.5):
        s1 = bie.Spheres(np.array([[0.2, 0.1, -0.3]]), 6, radii=[rad])
        y = dev(np.random.default_rng(18).standard_normal(3 * s1.N))
        z1 = host(s1.apply_precond(bie.OP_DN_BIE, y, precond=bie.PC_M0 | bie.PC_RIGID))
        z2 = host(s1.apply_precond(bie.OP_DN_BIE, y, precond=bie.PC_M0))
        assert_close(z1, z2, 1e-12)
        s1.close()
    rng = np.random.default_rng(19)
    v = rng.standard_normal((g.nb, 3))
    om = rng.standard_normal((g.nb, 3))
    F0, T0, _p, i0 = s.solve_resistance(v, om, tol=1e-11, precond=bie.PC_M0)
    F1, T1, _p, i1 = s.solve_resistance(v, om, tol=1e-11, precond=bie.PC_M0 | bie.PC_RIGID)
    assert i0["converged"] and i1["converged"]
    assert_close(F1, F0, 1e-8)
    assert_close(T1, T0, 1e-8)
    print(f"polydisperse resistance, 6 spheres: M0 {i0['iters']} its, M0 + rigid {i1['iters']} its")


def test_rigid_correction_gain_on_a_polydisperse_suspension():
    # 200 spheres of radii 0.5 and 1 (random sequential addition, gaps >= 0.1), p = 4:
    # the resistance form under M0 needs many more iterations than with the correction
    from paper_1707_06551_amd import bie
    from paper_1707_06551_amd.inputs import place_spheres_radii
    rng = np.random.default_rng(20)
    radii = np.where(rng.random(200) < 0.5, 0.5, 1.0)
    c = place_spheres_radii(radii, 16.0, 0.1, rng)
    s = bie.Spheres(c, 4, near_gap=1.0, radii=radii)
    v = rng.standard_normal((200, 3))
    om = rng.standard_normal((200, 3))
    F0, T0, _p, i0 = s.solve_resistance(v, om, tol=1e-8, precision=bie.MIXED, precond=bie.PC_M0)
    F1, T1, _p, i1 = s.solve_resistance(v, om, tol=1e-8, precision=bie.MIXED, precond=bie.PC_M0 | bie.PC_RIGID)
    print(f"200 polydisperse spheres, p = 4: M0 {i0['iters']} its, M0 + rigid {i1['iters']} its")
    assert i0["converged"] and i1["converged"]
    assert_close(F1, F0, 1e-6)
    assert_close(T1, T0, 1e-6)
    assert i1["iters"] < 0.7 * i0["iters"], (i0["iters"], i1["iters"])
    s.close()


def test_porous_media_solve_matches_oracle(cluster):
    # Problem 1: spheres held fixed in a uniform stream U, (1/2 + S + D) mu = -U
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    U = np.array([0.3, -0.8, 0.5])
    b = -np.tile(U, g.N)
    x, info = s.solve(bie.OP_SD_BIE, dev(b), tol=1e-12, precond=bie.PC_M0)
    assert info["converged"], info
    ops = Operators(g)
    A = assemble(lambda m: ops.apply("SD_BIE", m.reshape(g.N, 3, -1)).reshape(3 * g.N, -1), 3 * g.N)
    mu = np.linalg.solve(A, b)
    assert_close(host(x), mu, 1e-9)
    x2, info2 = s.solve(bie.OP_SD_BIE, dev(b), tol=1e-10, precision=bie.MIXED, precond=bie.PC_M0)
    assert info2["converged"], info2
    assert_close(host(x2), mu, 1e-8)
    print(f"polydisperse porous media, 6 spheres p = 6: GMRES {info['iters']} (M0), mixed {info2['iters']}")


def test_fixed_sphere_of_radius_a_drag():
    from paper_1707_06551_amd import bie
    a = 0.3
    s = bie.Spheres(np.array([[1.0, -2.0, 0.5]]), 8, radii=[a])
    U = np.array([1.0, 0.5, -0.25])
    x, info = s.solve(bie.OP_SD_BIE, dev(-np.tile(U, s.N)), tol=1e-13, precond=bie.PC_M0)
    _xyz, w = s.nodes()
    F = (host(x).reshape(-1, 3) * w[:, None]).sum(axis=0)
    assert np.abs(F + 6 * math.pi * a * U).max() < 1e-11
    s.close()


def test_polydisperse_rejects_unit_only_features(cluster):
    from paper_1707_06551_amd import bie
    c, a, s, g = cluster
    mu = dev(np.zeros(3 * g.N))
    with pytest.raises(bie.BieError):
        s.apply_precond(bie.OP_SD_BIE, mu, precond=bie.PC_MLP)
    with pytest.raises(bie.BieError):
        bie.Spheres(c, 4, radii=np.full(len(a), 1.2))   # overlapping
    with pytest.raises(bie.BieError):
        s_rot = bie.Spheres(c, 4, radii=a, near_method=1)
        try:
            s_rot.apply(bie.OP_K, mu[:3 * s_rot.N])       # the traction has no rotation variant
        finally:
            s_rot.close()
