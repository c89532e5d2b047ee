"""Pins of the oracle's separation-threshold measurement (Eq. 4.5 with the shell test of
Section 6, Fig. 5).  The pins come from outside the measurement itself: a published test
vector of the random stream, a brute-force quadrature on a much finer grid as the exact
value, the decay rate that the quadrature's exactness predicts, and the ordering of the
thresholds in p and in the tolerance."""
import math

import numpy as np
import pytest

from oracle.calibration import ShellTest, calibrated_gap, gap_grid, splitmix64, uniform
from oracle.grid import sphere_grid
from oracle.harmonics import vsh_at
from oracle.kernels import direct_sum


def test_splitmix64_published_vector():
    # SplitMix64 started from state 0 (Steele, Lea and Flood, 2014): the first outputs of
    # the reference generator
    assert [splitmix64(i) for i in range(4)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    u = np.array([uniform(i) for i in range(4000)])
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.05 and abs(u.var() - 1.0 / 3.0) < 0.02


def test_gap_grid():
    assert gap_grid(0) == 1.0 / 64.0
    assert gap_grid(48) == 1.0
    assert gap_grid(104) == 128.0


@pytest.mark.parametrize("p", [4, 8, 12])
def test_quadrature_and_formulas_agree_far_away(p):
    # at a gap of 100 the smooth quadrature is exact to rounding, so the exterior
    # formulas and the quadrature of the same density must agree
    st = ShellTest(p)
    assert st.error(100.0) < 1e-10 * (1.0 if p > 4 else 10.0)


@pytest.mark.parametrize("p", [4, 8])
def test_exact_values_match_fine_grid_quadrature(p):
    # the exact potentials on shells at gaps 0.5 and 1 equal a brute-force smooth
    # quadrature of the same density on a grid of order 4p + 40 (converged there), so a
    # wrong term in the exterior formulas shows up as an O(1) discrepancy
    st = ShellTest(p)
    pf = 4 * p + 40
    gf = sphere_grid(pf)
    modes, _Y, V, W, X = vsh_at(gf["xhat"], p, st.mmax)
    B = st.coef.shape[0]
    sig = np.zeros((gf["xhat"].shape[0], 3, B))
    for d in range(B):
        f = np.zeros((gf["xhat"].shape[0], 3), dtype=np.complex128)
        for i, _nm in enumerate(modes):
            f += st.coef[d, 0, i] * V[i] + st.coef[d, 1, i] * W[i] + st.coef[d, 2, i] * X[i]
        sig[:, :, d] = f.real
    q = sig * gf["wnode"][:, None, None]
    for gap in (0.5, 1.0):
        R = 1.0 + gap
        for op, (a_s, a_d) in (("S", (1.0, 0.0)), ("D", (0.0, 1.0))):
            ref = direct_sum(R * st.dirs, gf["xhat"], gf["xhat"], q, a_s, a_d)
            assert np.abs(ref - st.exact(R, op)).max() / st.sigma_max < 1e-11, (gap, op)


@pytest.mark.parametrize("p", [4, 8, 12])
def test_error_decays_at_the_predicted_rate(p):
    # The trapezoid rule on n_phi = 2p longitudes integrates e^{i m phi} exactly for
    # |m| < 2p.  The Cartesian components of a degree-p vector harmonic reach azimuthal
    # order mmax + 1 = p, so the first term of the kernel's expansion about the source
    # centre that aliases has degree p and decays like R^-(p+1): the error falls as
    # (1 + g)^-(p+1) once the gap is a few radii.
    st = ShellTest(p)
    e5, e10 = st.error(5.0), st.error(10.0)
    slope = math.log(e5 / e10) / math.log(11.0 / 6.0)
    assert p + 0.8 < slope < p + 1.4, slope


def test_threshold_meets_tolerance_and_orders():
    table = {}
    for p in (8, 12):
        for tol in (1e-4, 1e-8):
            d = calibrated_gap(p, tol)
            table[p, tol] = d
            st = ShellTest(p)
            assert st.error(d) <= tol / 10.0
            # one grid step closer fails, i.e. d* is the smallest passing grid gap
            k = round(8 * math.log2(64 * d))
            assert st.error(gap_grid(k - 1)) > tol / 10.0
    assert table[8, 1e-8] > table[8, 1e-4] and table[12, 1e-8] > table[12, 1e-4]
    assert table[8, 1e-4] > table[12, 1e-4] and table[8, 1e-8] > table[12, 1e-8]


def test_unreachable_tolerance_gives_every_pair_near():
    # at p = 2 the quadrature error decays like (1 + g)^-3: 1e-14 is out of reach within
    # the grid's largest gap, so every pair is near
    assert calibrated_gap(2, 1e-14) == math.inf
