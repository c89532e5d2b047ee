"""GPU solves against stored oracle solutions: the 8-sphere, p = 8 workload
(tests/golden/spheres8_p8.json, written by tests/golden/make_golden.py from oracle/
only; float64 GMRES to 1e-10 and mixed-precision refinement to 1e-10, with and without
the block preconditioner: forces/torques and velocities to 1e-8) and a 64-sphere window
of a dense placement (tests/golden/window64_p8.json, make_golden_window64.py: the
oracle's full solve, its time beside the library's)."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1707_06551_amd.inputs import make_workload
from tests.gpu_common import assert_close

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spheres8_p8.json")


def _golden():
    with open(GOLD) as f:
        return json.load(f)


def test_golden_matches_the_workload_generator():
    g = _golden()
    w = make_workload("spheres8_p8")
    assert hashlib.sha256(np.ascontiguousarray(w["centres"]).tobytes()).hexdigest() == g["centres_sha256"]
    assert g["resistance"]["rel_residual"] < 1e-11 and g["mobility"]["rel_residual"] < 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("precision,precond", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_solves_match_golden(precision, precond):
    from paper_1707_06551_amd import bie
    g = _golden()
    w = make_workload("spheres8_p8")
    s = bie.Spheres(w["centres"], 8, near_gap=1.0)
    F, T, _, info = s.solve_resistance(w["v"], w["omega"], tol=1e-10, precision=precision, precond=precond)
    assert info["converged"] and info["rel_residual"] < 1e-10, info
    assert_close(F, np.array(g["resistance"]["F"]), 1e-8)
    assert_close(T, np.array(g["resistance"]["T"]), 1e-8)
    v, om, _, info = s.solve_mobility(w["v"], w["omega"], tol=1e-10, precision=precision, precond=precond)
    assert info["converged"] and info["rel_residual"] < 1e-10, info
    assert_close(v, np.array(g["mobility"]["v"]), 1e-8)
    assert_close(om, np.array(g["mobility"]["omega"]), 1e-8)
    s.close()


GOLD64 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "window64_p8.json")


def test_window64_golden_is_converged():
    with open(GOLD64) as f:
        g = json.load(f)
    assert g["rel_residual"] < 1e-10 and len(g["centres"]) == 64
    c = np.array(g["centres"])
    d = np.linalg.norm(c[:, None] - c[None], axis=2) + 10 * np.eye(64)
    assert d.min() >= 2.02 - 1e-12   # min gap 0.02


@pytest.mark.gpu
@pytest.mark.parametrize("precision,precond,tol", [(0, 1, 1e-8), (1, 1, 1e-7), (1, 0x11, 1e-7)])
def test_window64_resistance_matches_oracle_solve(precision, precond, tol):
    # the oracle's full unpreconditioned solve of a 64-sphere dense window (phi 0.30, gap
    # 0.02, p = 8) against the library's float64 and mixed-precision solves with M0 (and
    # the rigid-mode correction)
    from paper_1707_06551_amd import bie
    with open(GOLD64) as f:
        g = json.load(f)
    s = bie.Spheres(np.array(g["centres"]), g["p"], near_gap=g["near_gap"])
    F, T, _, info = s.solve_resistance(np.array(g["v"]), np.array(g["omega"]), tol=1e-10, precision=precision,
                                       precond=precond)
    assert info["converged"], info
    print(f"oracle {g['iters']} iterations in {g['oracle_seconds']:.1f} s on {g['oracle_processes']} host "
          f"processes; library {info['iters']} iterations in {info['seconds']:.3f} s "
          f"(precision {precision}, precond {precond})")
    assert_close(F, np.array(g["F"]), tol)
    assert_close(T, np.array(g["T"]), tol)
    s.close()
