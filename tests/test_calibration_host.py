"""The library's separation threshold (bie_near_gap_for, host code) against the oracle's
measurement of the same quantity (Eq. 4.5 with the shell test of Section 6): the same
grid point for every order and precision, and the oracle's quadrature error at the
library's threshold within a tenth of the tolerance."""
import math
import os

import pytest

from oracle.calibration import ShellTest, calibrated_gap

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1707_06551_amd", "libbie.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libbie.so not built")


@pytest.mark.parametrize("p", [4, 8, 12, 16])
def test_threshold_equals_the_oracles_and_meets_the_tolerance(p):
    from paper_1707_06551_amd import bie
    st = ShellTest(p)
    for tol in (1e-4, 1e-6, 1e-8):
        d = bie.near_gap_for(p, tol)
        assert d == calibrated_gap(p, tol), (p, tol)
        assert st.error(d) <= tol / 10.0, (p, tol, d)


def test_wider_grid_and_unreachable_precision():
    from paper_1707_06551_amd import bie
    assert bie.near_gap_for(6, 1e-6, n_phi=14) == calibrated_gap(6, 1e-6, n_phi=14)
    assert bie.near_gap_for(2, 1e-14) == math.inf == calibrated_gap(2, 1e-14)


@pytest.mark.parametrize("args", [(0, 0, 1e-8), (21, 0, 1e-8), (4, 7, 1e-8), (4, 6, 1e-8), (4, 0, 0.0),
                                  (4, 0, 1.0), (4, 0, float("nan"))])
def test_bad_arguments(args):
    from paper_1707_06551_amd import bie
    with pytest.raises(bie.BieError):
        bie.near_gap_for(args[0], args[2], n_phi=args[1])
