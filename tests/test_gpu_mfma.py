"""GPU parity of the matrix-core Legendre stages (bie_opts.legendre_mfma = 1): the
transforms against the oracle's dense projection and synthesis (Section 2.1, Eqs.
2.9-2.14), and every operator built on them against the FMA path of the same library
(same arithmetic up to rounding order).  Orders p = 4 to 20 cover one and two 16-row
tiles (p + 1 latitudes and degrees above 16 from p = 16 on) and n_phi > 2p."""
import numpy as np
import pytest

from oracle.grid import Geometry
from oracle.operators import Operators
from tests.gpu_common import assert_close, make_workload, oracle_coef_to_gpu, small_cluster

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _bie():
    from paper_1707_06551_amd import bie
    return bie


CASES = {
    # name: (centres, p, n_phi)
    "cluster12_p4": (lambda: small_cluster(12, 9.0, 0.15, 3), 4, 0),
    "cluster7_p6_nphi14": (lambda: small_cluster(7, 7.5, 0.3, 5), 6, 14),
    "three_p12": (lambda: np.array([[0.0, 0.0, 0.0], [2.6, 0.3, -0.2], [0.4, 3.1, 0.5]]), 12, 0),
    "two_p17": (lambda: np.array([[0.0, 0.0, 0.0], [1.3, 2.1, 0.9]]), 17, 0),
    "two_p20_nphi44": (lambda: np.array([[0.0, 0.0, 0.0], [-2.2, 0.4, 1.5]]), 20, 44),
}

_cache = {}


def setup_case(name):
    if name in _cache:
        return _cache[name]
    mk, p, nphi = CASES[name]
    c = mk()
    B = _bie()
    s1 = B.Spheres(c, p, n_phi=nphi, near_gap=1.0, legendre_mfma=1)
    s0 = B.Spheres(c, p, n_phi=nphi, near_gap=1.0)
    g = Geometry(c, p, n_phi=(nphi or None), near_gap=1.0)
    _cache[name] = (s1, s0, g, Operators(g))
    return _cache[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-6)])
def test_forward_transform_on_matrix_cores(name, precision, tol):
    s1, s0, g, ops = setup_case(name)
    mu = np.random.default_rng(41).standard_normal((g.N, 3))
    coef = host(s1.vsh_forward(dev(mu), precision=precision)).reshape(g.nb, 3, s1.ncoef, 2)
    ref = oracle_coef_to_gpu(ops, [ops.coefficients(mu[..., None], k)[..., 0] for k in range(g.nb)], g.nb)
    assert_close(coef, ref, tol)
    fma = host(s0.vsh_forward(dev(mu), precision=precision)).reshape(coef.shape)
    assert_close(coef, fma, (1e-13 if precision == 0 else 1e-6))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-6)])
def test_inverse_transform_on_matrix_cores(name, precision, tol):
    s1, s0, g, ops = setup_case(name)
    mu = np.random.default_rng(42).standard_normal((g.N, 3))
    coefs = [ops.coefficients(mu[..., None], k)[..., 0] for k in range(g.nb)]
    field = np.concatenate([ops.vsh.inverse(c) for c in coefs])
    cg = oracle_coef_to_gpu(ops, coefs, g.nb)
    out = host(s1.vsh_inverse(dev(cg), precision=precision)).reshape(g.N, 3)
    assert_close(out, field, tol)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("opname", ["S", "SD_BIE", "DN_BIE", "MOBILITY"])
@pytest.mark.parametrize("precision", [0, 1])
def test_operators_equal_the_fma_path(name, opname, precision):
    B = _bie()
    s1, s0, g, _ = setup_case(name)
    op = getattr(B, "OP_" + opname)
    rng = np.random.default_rng(43)
    n = 3 * g.N + (6 * g.nb if opname == "MOBILITY" else 0)
    x = dev(rng.standard_normal(n))
    a = host(s1.apply(op, x, precision=precision))
    b = host(s0.apply(op, x, precision=precision))
    assert_close(a, b, (1e-13 if precision == 0 else 1e-6))
    if opname in ("DN_BIE", "MOBILITY"):
        za = host(s1.apply_precond(op, x, precision=precision, precond=B.PC_M0))
        zb = host(s0.apply_precond(op, x, precision=precision, precond=B.PC_M0))
        assert_close(za, zb, (1e-13 if precision == 0 else 1e-6))


def test_mobility_solve_on_matrix_cores():
    B = _bie()
    c = make_workload("spheres8_p8")["centres"]
    rng = np.random.default_rng(44)
    F = rng.standard_normal((len(c), 3))
    T = rng.standard_normal((len(c), 3))
    out = []
    for mf in (1, 0):
        s = B.Spheres(c, 8, near_gap=1.0, legendre_mfma=mf)
        v, om, _mu, info = s.solve_mobility(F, T, tol=1e-10, precision=B.MIXED, precond=B.PC_M0)
        assert info["converged"]
        out.append((v, om, info["iters"]))
        s.close()
    assert_close(out[0][0], out[1][0], 1e-9)
    assert_close(out[0][1], out[1][1], 1e-9)
    assert abs(out[0][2] - out[1][2]) <= 1


def test_option_is_checked():
    B = _bie()
    with pytest.raises(B.BieError):
        B.Spheres(np.zeros((1, 3)), 4, legendre_mfma=2)
