"""GPU: bie_apply_bio_noalloc (work buffers in the library's static device array, no
allocation) against bie_apply_bio on the same inputs, called through the C ABI: two
calls in a row on different contexts, the second smaller, for every operator and both
precisions; sizes beyond the array are refused."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import assert_close, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _lib():
    from paper_1707_06551_amd import bie
    L = bie.lib()
    L.bie_apply_bio_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.bie_apply_bio_noalloc.restype = ctypes.c_int
    return bie, L


def _noalloc(bie, L, s, op, x, precision):
    u = torch.full((s.dof(op),), float("nan"), dtype=torch.float64, device="cuda")
    rc = L.bie_apply_bio_noalloc(s._h, op, precision, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(u.data_ptr()))
    assert rc == 0, (rc, L.bie_last_error())
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_apply_bio_on_two_calls(precision):
    bie, L = _lib()
    cases = [(small_cluster(12, 9.0, 0.15, 3), 6), (small_cluster(5, 6.0, 0.3, 4), 4)]   # the second is smaller
    tol = 1e-11 if precision == 0 else 1e-6
    for centres, p in cases:
        s = bie.Spheres(centres, p, near_gap=1.0)
        assert s.n_near > 0
        for op in (bie.OP_S, bie.OP_D, bie.OP_SD_BIE, bie.OP_DN_BIE, bie.OP_MOBILITY,
                   bie.OP_SD_BIE | bie.STAGE_NEAR, bie.OP_DN_BIE | bie.STAGE_FAR):
            x = torch.from_numpy(np.random.default_rng(op).standard_normal(s.dof(op))).cuda()
            ref = s.apply(op, x, precision=precision).cpu().numpy()
            got = _noalloc(bie, L, s, op, x, precision)
            assert_close(got, ref, tol, f"op {op:#x} p {p}")
        s.close()


def test_noalloc_refuses_work_beyond_the_array_and_bad_ops():
    bie, L = _lib()
    s = bie.Spheres(small_cluster(4, 6.0, 0.3, 4), 4, near_gap=1.0)
    x = torch.zeros(s.dof(bie.OP_K), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(x)
    for op in (bie.OP_K, bie.OP_KL_BIE, 0x99):
        assert L.bie_apply_bio_noalloc(s._h, op, 0, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(u.data_ptr())) == -1
    s.close()
    # 4096 spheres at p = 12: 1,277,952 nodes, work buffers above 96 MiB
    g = np.arange(16) * 2.5
    c = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    big = bie.Spheres(c, 12, near_gap=1.0)
    xb = torch.zeros(3 * big.N, dtype=torch.float64, device="cuda")
    ub = torch.zeros_like(xb)
    assert L.bie_apply_bio_noalloc(big._h, bie.OP_SD_BIE, 0, ctypes.c_void_p(xb.data_ptr()),
                                   ctypes.c_void_p(ub.data_ptr())) == -1
    assert b"exceed" in L.bie_last_error()
    big.close()
