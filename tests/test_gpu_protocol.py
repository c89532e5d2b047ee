"""The validation protocol of Section 6 (Eq. 6.2) on spheres of the printed radii
(0.903, 0.510, 0.262): the solved completed double layer reproduces the exterior flow of
point forces inside the spheres up to the surfaces, with error falling as p grows.  The
reference is the exact Stokeslet flow (Eq. 2.19), not the oracle."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_protocol_converges_up_to_the_boundary():
    from paper_1707_06551_amd.run_protocol import run
    r6 = run(6)
    r12 = run(12)
    print(f"Eq. 6.2 protocol: p = 6 {r6['max_rel_err']:.2e} ({r6['iters']} its), "
          f"p = 12 {r12['max_rel_err']:.2e} ({r12['iters']} its)")
    assert r6["converged"] and r12["converged"]
    assert r12["max_rel_err"] < 0.1 * r6["max_rel_err"], (r6, r12)
    # no loss of accuracy towards the surface: points 1e-6 r away are as accurate as
    # points 1e-2 r away (the near series carries the solved density's accuracy to the
    # boundary; measured 1.5e-4 against 2.7e-4 at p = 12)
    per = r12["max_rel_err_by_distance"]
    assert per["1e-6"] <= 10 * per["1e-2"], per
