"""GPU parity of the near-pair evaluation by pole rotation (near_method = 1, Section 4.2)
against the oracle (oracle/rotation_near.py): the near stage alone, the full operator,
and a solve that stays within the projection error of the direct method."""
import json
import os

import numpy as np
import pytest

from oracle import rotation_near as rn
from oracle.grid import Geometry
from oracle.operators import OPS as ORACLE_OPS, Operators
from tests.gpu_common import assert_close, poly_cluster, rel_err, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS = {"S": 1, "D": 2, "SD_BIE": 3, "DN_BIE": 4}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


_case = {}


def case():
    if not _case:
        from paper_1707_06551_amd import bie
        c = small_cluster(10, 7.0, 0.05, 21)
        p = 6
        _case["c"] = c
        _case["s"] = bie.Spheres(c, p, near_gap=1.0, near_method=1)
        _case["g"] = Geometry(c, p, near_gap=1.0)
        _case["ops"] = Operators(_case["g"])
    return _case["c"], _case["s"], _case["g"], _case["ops"]


@pytest.mark.parametrize("opname", ["S", "D", "SD_BIE"])
def test_near_stage_matches_oracle(opname):
    from paper_1707_06551_amd import bie
    c, s, g, ops = case()
    assert g.near.sum() > 0
    a_s, a_d, _ci, _compl = ORACLE_OPS[opname]
    mu = np.random.default_rng(7).standard_normal((g.N, 3))
    out = host(s.apply(OPS[opname] | bie.STAGE_NEAR, dev(mu))).reshape(g.N, 3)
    # the stage call also zero-fills u before the near part is added
    ref = rn.near_part(g, mu, a_s, a_d)
    assert_close(out, ref, 1e-11)


@pytest.mark.parametrize("opname", ["SD_BIE", "DN_BIE"])
@pytest.mark.parametrize("precision", [0, 1])
def test_full_operator_matches_oracle(opname, precision):
    c, s, g, ops = case()
    a_s, a_d, ci, compl = ORACLE_OPS[opname]
    mu = np.random.default_rng(8).standard_normal((g.N, 3))
    out = host(s.apply(OPS[opname], dev(mu), precision=precision)).reshape(g.N, 3)
    ref = ops.self_part(mu, a_s, a_d) + ci * mu + rn.near_part(g, mu, a_s, a_d) + ops.far_part(mu, a_s, a_d)
    if compl:
        ref = ref + ops.completion_part(mu)
    tol = 1e-11 if precision == 0 else 1e-6
    assert_close(out, ref, tol)


def test_solve_stays_within_the_projection_error():
    # 8 spheres, p = 8, min gap 0.5: the rotated-projection near field differs from the
    # nodal series by the band-limited projection error, so the solution moves by that
    # much and no more
    from paper_1707_06551_amd import bie
    from paper_1707_06551_amd.inputs import make_workload
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "spheres8_p8.json")) as f:
        gold = json.load(f)
    w = make_workload("spheres8_p8")
    s = bie.Spheres(w["centres"], 8, near_gap=1.0, near_method=1)
    F, T, _, info = s.solve_resistance(w["v"], w["omega"], tol=1e-10, precond=bie.PC_M0)
    assert info["converged"], info
    eF = rel_err(F, np.array(gold["resistance"]["F"]))
    eT = rel_err(T, np.array(gold["resistance"]["T"]))
    print(f"rotation vs direct near evaluation, 8 spheres p = 8: |dF|/|F| {eF:.2e}, |dT|/|T| {eT:.2e}")
    assert eF < 1e-3 and eT < 1e-3
    s.close()


def test_near_stage_with_wider_azimuthal_grid():
    # n_phi = 2p + 2 (mmax = p): orders up to p are kept on the target grid
    from paper_1707_06551_amd import bie
    c = small_cluster(7, 7.5, 0.3, 5)
    p = 6
    s = bie.Spheres(c, p, n_phi=2 * p + 2, near_gap=1.0, near_method=1)
    g = Geometry(c, p, n_phi=2 * p + 2, near_gap=1.0)
    assert g.near.sum() > 0 and g.mmax == p
    mu = np.random.default_rng(9).standard_normal((g.N, 3))
    out = host(s.apply(OPS["SD_BIE"] | bie.STAGE_NEAR, dev(mu))).reshape(g.N, 3)
    ref = rn.near_part(g, mu, 1.0, 1.0)
    assert_close(out, ref, 1e-11)
    s.close()


_pcase = {}


def poly_case():
    # six spheres of radii 0.35-1.4 with near pairs in both directions between unequal
    # radii (gaps 0.12-0.9)
    if not _pcase:
        from paper_1707_06551_amd import bie
        c, a = poly_cluster()
        p = 6
        _pcase["s"] = bie.Spheres(c, p, near_gap=1.0, radii=a, near_method=1)
        _pcase["g"] = Geometry(c, p, near_gap=1.0, radii=a)
        _pcase["ops"] = Operators(_pcase["g"])
    return _pcase["s"], _pcase["g"], _pcase["ops"]


@pytest.mark.parametrize("opname", ["S", "D", "SD_BIE"])
def test_near_stage_with_radii_matches_oracle(opname):
    from paper_1707_06551_amd import bie
    s, g, ops = poly_case()
    assert g.near.sum() > 0 and not (g.near == g.near.T).all()
    a_s, a_d, _ci, _compl = ORACLE_OPS[opname]
    mu = np.random.default_rng(9).standard_normal((g.N, 3))
    out = host(s.apply(OPS[opname] | bie.STAGE_NEAR, dev(mu))).reshape(g.N, 3)
    ref = rn.near_part(g, mu, a_s, a_d)
    assert_close(out, ref, 1e-11)


@pytest.mark.parametrize("opname", ["SD_BIE", "DN_BIE"])
@pytest.mark.parametrize("precision", [0, 1])
def test_full_operator_with_radii_matches_oracle(opname, precision):
    s, g, ops = poly_case()
    a_s, a_d, ci, compl = ORACLE_OPS[opname]
    mu = np.random.default_rng(10).standard_normal((g.N, 3))
    out = host(s.apply(OPS[opname], dev(mu), precision=precision)).reshape(g.N, 3)
    ref = ops.self_part(mu, a_s, a_d) + ci * mu + rn.near_part(g, mu, a_s, a_d) + ops.far_part(mu, a_s, a_d)
    if compl:
        ref = ref + ops.completion_part(mu)
    tol = 1e-11 if precision == 0 else 1e-6
    assert_close(out, ref, tol)


def test_polydisperse_solve_with_rotation():
    # porous-media solve on the polydisperse cluster with the rotation near stage: it
    # converges and stays within the near-field projection error of the direct method
    from paper_1707_06551_amd import bie
    s, g, _ops = poly_case()
    s0 = bie.Spheres(g.centres, g.p, near_gap=1.0, radii=g.radii)
    b = dev(np.tile([-1.0, 0.2, 0.0], g.N))
    x1, i1 = s.solve(bie.OP_SD_BIE, b, tol=1e-10, precond=bie.PC_M0)
    x0, i0 = s0.solve(bie.OP_SD_BIE, b, tol=1e-10, precond=bie.PC_M0)
    assert i1["converged"] and i0["converged"]
    d = rel_err(host(x1), host(x0))
    print(f"polydisperse porous media, rotation vs direct near stage: {d:.2e} ({i1['iters']} / {i0['iters']} its)")
    assert d < 0.1   # the operators themselves match the oracle to 1e-11 (tests above)
    s0.close()
