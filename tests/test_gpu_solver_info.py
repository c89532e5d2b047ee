"""GPU: the solver's boundary options and report (bie_solve_opts.x0 / res_hist,
bie_solve_info.t_stage_s / pairs_evaluated / near_evals) through the C ABI.

A converged solution passed back as the initial guess returns after the one float64
residual check (0 iterations); a partial solve resumed from its own result reaches the
same solution as a solve from zero; the residual history has one entry per iteration;
the per-step device times are positive where the step ran and add up to at most the
solve's wall time; the pair counts equal matvecs times the pairs of one pass."""
import numpy as np
import pytest

from tests.gpu_common import assert_close, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def sph():
    from paper_1707_06551_amd import bie
    c = small_cluster(12, 9.0, 0.15, 3)
    s = bie.Spheres(c, 6, near_gap=1.0)
    yield s
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_resistance_resumes_from_its_solution(sph, precision):
    from paper_1707_06551_amd import bie
    rng = np.random.default_rng(7)
    v, om = rng.standard_normal((sph.nb, 3)), rng.standard_normal((sph.nb, 3))
    F, T, psi, info = sph.solve_resistance(v, om, tol=1e-10, precision=precision, precond=bie.PC_M0, want_psi=True)
    assert info["converged"] and info["iters"] > 3, info
    F2, T2, psi2, info2 = sph.solve_resistance(v, om, tol=1e-10, precision=precision, precond=bie.PC_M0,
                                               want_psi=True, x0=psi)
    assert info2["converged"] and info2["iters"] == 0 and info2["matvecs_fp64"] == 1, info2
    assert_close(F2, F, 1e-12)
    assert_close(T2, T, 1e-12)
    assert_close(host(psi2), host(psi), 1e-14)


def test_partial_solve_resumed_matches_a_full_solve(sph):
    from paper_1707_06551_amd import bie
    rng = np.random.default_rng(8)
    v, om = rng.standard_normal((sph.nb, 3)), rng.standard_normal((sph.nb, 3))
    F, T, _, info = sph.solve_resistance(v, om, tol=1e-11, precond=bie.PC_M0)
    _, _, psi_a, ia = sph.solve_resistance(v, om, tol=1e-3, precond=bie.PC_M0, want_psi=True)
    Fb, Tb, _, ib = sph.solve_resistance(v, om, tol=1e-11, precond=bie.PC_M0, x0=psi_a)
    assert ia["converged"] and ib["converged"], (ia, ib)
    assert 0 < ib["iters"] < info["iters"], (ia["iters"], ib["iters"], info["iters"])
    assert_close(Fb, F, 1e-9)
    assert_close(Tb, T, 1e-9)


def test_mobility_resumes_from_its_solution(sph):
    from paper_1707_06551_amd import bie
    rng = np.random.default_rng(9)
    Fa, Ta = rng.standard_normal((sph.nb, 3)), rng.standard_normal((sph.nb, 3))
    v, om, mu, info = sph.solve_mobility(Fa, Ta, tol=1e-10, precision=bie.MIXED, precond=bie.PC_M0, want_mu=True)
    assert info["converged"], info
    x0 = torch.cat([mu, torch.from_numpy(np.concatenate([v.reshape(-1), om.reshape(-1)])).to(mu.device)])
    v2, om2, _, info2 = sph.solve_mobility(Fa, Ta, tol=1e-10, precision=bie.MIXED, precond=bie.PC_M0, x0=x0)
    assert info2["converged"] and info2["iters"] == 0, info2
    assert_close(v2, v, 1e-13)
    assert_close(om2, om, 1e-13)


@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (1, 1)])
def test_history_stage_times_and_pair_counts(sph, precision, precond):
    rng = np.random.default_rng(10)
    v, om = rng.standard_normal((sph.nb, 3)), rng.standard_normal((sph.nb, 3))
    _, _, _, info = sph.solve_resistance(v, om, tol=1e-10, precision=precision, precond=precond, history=400)
    assert info["converged"], info
    h = info["res_hist"]
    assert info["res_hist_len"] == info["iters"] == h.size > 0
    assert np.all(h > 0) and h[0] < 1.0 and h[-1] <= 1e-9
    assert info["rel_residual"] <= 1e-10
    mv = info["matvecs_fp64"] + info["matvecs_mixed"]
    assert info["pairs_evaluated"] == mv * sph.far_node_pairs
    assert info["near_evals"] == mv * sph.n_near * sph.P and sph.n_near > 0
    t = info["t_stage_s"]
    for k in ("transform", "near", "far", "krylov"):
        assert t[k] > 0, (k, t)
    assert (t["precond"] > 0) == (precond != 0), t
    assert t["other"] == 0.0
    assert sum(t.values()) <= 1.05 * info["seconds"] + 1e-3, (t, info["seconds"])


def test_history_is_truncated_to_the_buffer(sph):
    rng = np.random.default_rng(11)
    v, om = rng.standard_normal((sph.nb, 3)), rng.standard_normal((sph.nb, 3))
    _, _, _, info = sph.solve_resistance(v, om, tol=1e-10, history=3)
    assert info["iters"] > 3 and info["res_hist_len"] == 3 and info["res_hist"].size == 3


def test_zero_right_hand_side_with_an_initial_guess_returns_zero(sph):
    from paper_1707_06551_amd import bie
    b = torch.zeros(3 * sph.N, dtype=torch.float64, device="cuda")
    x0 = torch.randn(3 * sph.N, dtype=torch.float64, device="cuda")
    x, info = sph.solve(bie.OP_DN_BIE, b, tol=1e-10, precond=bie.PC_M0, x0=x0)
    assert info["converged"] and info["iters"] == 0
    assert float(np.abs(host(x)).max()) == 0.0
