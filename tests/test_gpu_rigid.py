"""GPU parity of the global rigid-mode coarse correction (BIE_PC_RIGID) against the oracle
(oracle/rigid.py): the preconditioner application, its no-op on an isolated sphere,
solves that still reach the stored oracle solution, and the iteration gain it buys on a
dilute many-sphere resistance problem."""
import json
import os

import numpy as np
import pytest

from oracle import coarse, mlp, rigid
from oracle.grid import Geometry
from oracle.precond import m0_resistance
from tests.gpu_common import assert_close, rel_err, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bie():
    from paper_1707_06551_amd import bie
    return bie


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,seed", [(10, 21), (37, 4)])
def test_rigid_correction_matches_oracle(n, seed):
    B = _bie()
    c = small_cluster(n, 7.0 if n == 10 else 12.0, 0.05, seed)
    p = 5
    s = B.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    r = np.random.default_rng(seed).standard_normal((g.N, 3))
    z = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_M0 | B.PC_RIGID)).reshape(g.N, 3)
    ref = rigid.correct(g, r, m0_resistance(g, r))
    # the coarse system is solved by conjugate gradients to relative residual 1e-7
    assert_close(z, ref, 1e-6)
    # the correction is not small: it changes the rigid part of M0 r
    z0 = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_M0)).reshape(g.N, 3)
    assert rel_err(z, z0) > 1e-3
    s.close()


def test_rigid_correction_on_the_learned_preconditioner():
    B = _bie()
    c = small_cluster(10, 7.0, 0.05, 21)
    p = 5
    s = B.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    w = mlp.init_weights(17, out_scale=0.2)
    s.load_precond(w.astype(np.float32))
    r = np.random.default_rng(8).standard_normal((g.N, 3))
    z = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_MLP | B.PC_RIGID)).reshape(g.N, 3)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    theta, _ = mlp.forward(w.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    rho = np.stack([coarse.restrict(r[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    # with the rigid correction the learned part acts on the non-rigid low modes: the
    # translation and rotation components (b, c) of rho and zeta are dropped
    rho[:, 4:10] = 0.0
    zeta = coarse.coarse_apply(pairs, dirs, theta, rho)
    zeta[:, 4:10] = 0.0
    # the rigid correction resets the rigid part of M0 r, the learned one is added after it
    ref = rigid.correct(g, r, m0_resistance(g, r)) + np.concatenate([coarse.prolong(zeta[k], xh) for k in range(g.nb)])
    assert_close(z, ref, 1e-5)
    s.close()


def test_isolated_sphere_and_flag_rules():
    B = _bie()
    s = B.Spheres(np.array([[0.5, -1.0, 2.0]]), 6, near_gap=1.0)
    r = dev(np.random.default_rng(3).standard_normal(3 * s.N))
    z0 = host(s.apply_precond(B.OP_DN_BIE, r, precond=B.PC_M0))
    z1 = host(s.apply_precond(B.OP_DN_BIE, r, precond=B.PC_M0 | B.PC_RIGID))
    assert_close(z1, z0, 1e-12)
    with pytest.raises(B.BieError):
        s.apply_precond(B.OP_DN_BIE, r, precond=B.PC_RIGID)
    s.close()
    # the mobility form ignores the flag
    c = small_cluster(6, 6.0, 0.2, 5)
    s = B.Spheres(c, 4, near_gap=1.0)
    rm = dev(np.random.default_rng(4).standard_normal(3 * s.N + 6 * s.nb))
    a = host(s.apply_precond(B.OP_MOBILITY, rm, precond=B.PC_M0))
    b = host(s.apply_precond(B.OP_MOBILITY, rm, precond=B.PC_M0 | B.PC_RIGID))
    assert np.array_equal(a, b)
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_rigid_solves_match_golden(precision):
    from paper_1707_06551_amd.inputs import make_workload
    B = _bie()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spheres8_p8.json")) as f:
        gold = json.load(f)
    w = make_workload("spheres8_p8")
    s = B.Spheres(w["centres"], 8, near_gap=1.0)
    F, T, _, info = s.solve_resistance(w["v"], w["omega"], tol=1e-10, precision=precision,
                                       precond=B.PC_M0 | B.PC_RIGID)
    assert info["converged"] and info["rel_residual"] < 1e-10, info
    assert_close(F, np.array(gold["resistance"]["F"]), 1e-8)
    assert_close(T, np.array(gold["resistance"]["T"]), 1e-8)
    s.close()


def test_rigid_correction_gain_on_a_dilute_suspension():
    # 400 spheres, p = 4, volume fraction 0.15, min gap 0.1: the collective rigid-mode
    # coupling through the completion flow dominates the GMRES iteration count under M0
    from paper_1707_06551_amd.inputs import box_side, place_spheres
    B = _bie()
    rng = np.random.default_rng(11)
    c = place_spheres(400, box_side(400, 0.15), 0.1, rng)
    v, om = rng.standard_normal((400, 3)), rng.standard_normal((400, 3))
    s = B.Spheres(c, 4, near_gap=1.0)
    F0, T0, _, i0 = s.solve_resistance(v, om, tol=1e-8, precond=B.PC_M0)
    F1, T1, _, i1 = s.solve_resistance(v, om, tol=1e-8, precond=B.PC_M0 | B.PC_RIGID)
    F2, T2, _, i2 = s.solve_resistance(v, om, tol=1e-8, precision=B.MIXED, precond=B.PC_M0 | B.PC_RIGID)
    assert i0["converged"] and i1["converged"] and i2["converged"]
    assert i1["fallback_used"] == 0 and i2["fallback_used"] == 0
    assert_close(F1, F0, 1e-6)
    assert_close(T1, T0, 1e-6)
    assert_close(F2, F0, 1e-6)
    print(f"GMRES iterations: M0 {i0['iters']}, M0 + rigid {i1['iters']}, mixed M0 + rigid {i2['iters']}")
    assert i1["iters"] <= 0.7 * i0["iters"], (i0["iters"], i1["iters"])
    s.close()


def test_network_trained_on_the_rigid_base_gains_over_it():
    # committed weights (paper_1707_06551_amd/weights/precond_dn_rigid.npz): trained with
    # base M0 + BIE_PC_RIGID in the local-residual composition (BIE_PC_LOCAL) on 64-sphere
    # windows of 1024-sphere placements at volume fraction 0.30; held out here: two windows
    # of a placement seeded apart from the training, holdout and selection seeds
    from paper_1707_06551_amd.precond_train import DEFAULT_FILES, load_weights, window_configs
    B = _bie()
    w, meta = load_weights(DEFAULT_FILES["m0r"])
    assert meta["base"] == "m0r" and meta["composition"] == "local"
    pc = B.PC_MLP | B.PC_RIGID | B.PC_LOCAL
    rng = np.random.default_rng(3)
    base, learned = [], []
    for c in window_configs(2, 16, seed0=700000, procs=1):
        v, om = rng.standard_normal((len(c), 3)), rng.standard_normal((len(c), 3))
        s = B.Spheres(c, 16)
        s.load_precond(w)
        F0, T0, _, i0 = s.solve_resistance(v, om, tol=1e-8, precond=B.PC_M0 | B.PC_RIGID)
        F1, T1, _, i1 = s.solve_resistance(v, om, tol=1e-8, precond=pc)
        assert i0["converged"] and i1["converged"] and i1["fallback_used"] == 0
        assert_close(F1, F0, 1e-6)
        assert_close(T1, T0, 1e-6)
        base.append(i0["iters"])
        learned.append(i1["iters"])
        s.close()
    print(f"GMRES iterations M0 + rigid {base}, + learned {learned}")
    assert sum(learned) <= 0.92 * sum(base), (base, learned)
