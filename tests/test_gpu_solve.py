"""GPU solves of the 8-sphere, p = 8 workload against stored oracle values
(tests/golden/spheres8_p8.json, written by tests/golden/make_golden.py from oracle/
only).  Float64 GMRES to 1e-10 and mixed-precision refinement to 1e-10, with and
without the block preconditioner: forces/torques and velocities to 1e-8."""
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
