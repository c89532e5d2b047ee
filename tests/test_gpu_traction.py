"""GPU parity of the single-layer traction operator K, the operator of Eq. 5.8 and the
mobility problem in the paper's form (Problem 2, Eqs. 5.7-5.8) against the oracle
(oracle/traction.py), and against the bordered formulation of the same problem."""
import math

import numpy as np
import pytest

from oracle import traction as tr
from oracle.grid import Geometry
from tests.gpu_common import assert_close, rel_err, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cluster():
    # 10 spheres with several near pairs (gaps down to 0.05); p = 6 with n_phi = 2p
    # (mmax = p - 1), so the derivative potentials reach m = mmax + 1 < p + 1
    from paper_1707_06551_amd import bie
    c = small_cluster(10, 7.0, 0.05, 21)
    p = 6
    s = bie.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    yield c, s, g, tr.TractionOps(g)
    s.close()


@pytest.mark.parametrize("stage", ["self", "near", "far"])
def test_traction_stages_match_oracle(cluster, stage):
    from paper_1707_06551_amd import bie
    c, s, g, to = cluster
    assert g.near.sum() > 0
    mu = np.random.default_rng(1).standard_normal((g.N, 3))
    bits = {"self": bie.STAGE_SELF, "near": bie.STAGE_NEAR, "far": bie.STAGE_FAR}[stage]
    out = host(s.apply(bie.OP_K | bits, dev(mu))).reshape(g.N, 3)
    ref = {"self": to.self_part, "near": to.near_part, "far": to.far_part}[stage](mu)
    assert_close(out, ref, 1e-11)


@pytest.mark.parametrize("precision", [0, 1])
def test_kl_operator_matches_oracle(cluster, precision):
    c, s, g, to = cluster
    from paper_1707_06551_amd import bie
    mu = np.random.default_rng(2).standard_normal((g.N, 3))
    out = host(s.apply(bie.OP_KL_BIE, dev(mu), precision=precision)).reshape(g.N, 3)
    ref = to.apply_KL_BIE(mu)
    tol = 1e-11 if precision == 0 else 1e-6
    assert_close(out, ref, tol)


def test_far_traction_on_a_wider_azimuthal_grid():
    # n_phi = 2p + 2 (mmax = p): the derivative potentials reach m = p + 1
    from paper_1707_06551_amd import bie
    c = small_cluster(7, 7.5, 0.3, 5)
    p = 5
    s = bie.Spheres(c, p, n_phi=2 * p + 2, near_gap=1.0)
    g = Geometry(c, p, n_phi=2 * p + 2, near_gap=1.0)
    assert g.near.sum() > 0 and g.mmax == p
    to = tr.TractionOps(g)
    mu = np.random.default_rng(3).standard_normal((g.N, 3))
    out = host(s.apply(bie.OP_K, dev(mu))).reshape(g.N, 3)
    ref = to.apply_K(mu)
    assert_close(out, ref, 1e-11)
    s.close()


def test_m0_inverts_the_isolated_sphere():
    from paper_1707_06551_amd import bie
    s = bie.Spheres(np.array([[0.3, -0.2, 0.5]]), 7)
    mu = np.random.default_rng(4).standard_normal(3 * s.N)
    a = s.apply(bie.OP_KL_BIE, dev(mu))
    z = host(s.apply_precond(bie.OP_KL_BIE, a, precond=bie.PC_M0))
    assert_close(z, mu, 1e-12)
    s.close()


def test_mobility_traction_matches_oracle(cluster):
    c, s, g, to = cluster
    rng = np.random.default_rng(5)
    F = rng.standard_normal((g.nb, 3))
    T = rng.standard_normal((g.nb, 3))
    v, om, mu, info = s.solve_mobility_traction(F, T, tol=1e-12, want_mu=True)
    assert info["converged"], info
    v_o, om_o, mu_o, info_o = tr.solve_mobility_traction(g, F, T, tol=1e-12)
    assert_close(v, v_o, 1e-9)
    assert_close(om, om_o, 1e-9)
    assert_close(host(mu).reshape(g.N, 3), mu_o, 1e-8)
    print(f"traction mobility, 10 spheres p = 6: GMRES {info['iters']} (oracle {info_o['iters']})")


def test_isolated_sphere_stokes_mobility():
    from paper_1707_06551_amd import bie
    s = bie.Spheres(np.array([[1.0, 2.0, -0.5]]), 6)
    F = np.array([[0.4, -1.0, 2.0]])
    T = np.array([[1.5, 0.2, -0.3]])
    v, om, _mu, info = s.solve_mobility_traction(F, T, tol=1e-12)
    assert info["converged"]
    assert np.abs(v - F / (6 * math.pi)).max() < 1e-13
    assert np.abs(om - T / (8 * math.pi)).max() < 1e-13
    s.close()


def test_agrees_with_bordered_formulation_and_mixed_precision():
    # the two formulations of Problem 2 differ by the discretisation error; mixed
    # precision (float32 transforms and far field inside refinement) matches float64
    from paper_1707_06551_amd import bie
    from paper_1707_06551_amd.inputs import make_workload
    w = make_workload("spheres8_p8")
    rng = np.random.default_rng(6)
    F = rng.standard_normal((8, 3))
    T = rng.standard_normal((8, 3))
    s = bie.Spheres(w["centres"], 10, near_gap=1.0)
    v1, o1, _m1, i1 = s.solve_mobility_traction(F, T, tol=1e-10)
    v2, o2, _m2, i2 = s.solve_mobility(F, T, tol=1e-10, precond=bie.PC_M0)
    v3, o3, _m3, i3 = s.solve_mobility_traction(F, T, tol=1e-10, precision=bie.MIXED)
    assert i1["converged"] and i2["converged"] and i3["converged"]
    e_form = max(rel_err(v1, v2), rel_err(o1, o2))
    e_mix = max(rel_err(v3, v1), rel_err(o3, o1))
    print(f"8 spheres p = 10: traction vs bordered {e_form:.2e}, mixed vs float64 {e_mix:.2e}, "
          f"iterations {i1['iters']} / {i2['iters']} / {i3['iters']}")
    assert e_form < 1e-5 and e_mix < 1e-7
    s.close()


def test_traction_rejects_unsupported_options():
    from paper_1707_06551_amd import bie
    c = small_cluster(4, 6.0, 0.3, 2)
    s = bie.Spheres(c, 4, near_gap=1.0, near_method=1)
    mu = dev(np.zeros(3 * s.N))
    with pytest.raises(bie.BieError):
        s.apply(bie.OP_K, mu)
    s.close()
    s = bie.Spheres(c, 4, near_gap=1.0)
    with pytest.raises(bie.BieError):
        s.apply_precond(bie.OP_KL_BIE, dev(np.zeros(3 * s.N)), precond=bie.PC_M0 | bie.PC_RIGID)
    with pytest.raises(bie.BieError):
        s.solve_mobility_traction(np.zeros((4, 3)), np.ones((4, 3)), precond=bie.PC_MLP)
    s.close()
