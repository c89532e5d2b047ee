"""Shared helpers of the GPU parity tests (seeded inputs, oracle comparison)."""
import numpy as np

from paper_1707_06551_amd.inputs import make_workload, place_spheres


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_close(out, ref, tol, what=""):
    """Parity of a GPU result with the oracle: the relative 2-norm of the difference below
    tol (the stated tolerance), and every entry within an entry bound.

    Entry bound.  float64 results (tol < 1e-7): |out_i - ref_i| <= tol (|ref_i| + rms(ref)).
    The floor is the reference's RMS because the rounding error of an entry (a sum of
    many node contributions, or a solve) scales with the magnitudes summed into it, which
    are of the field's typical size, not with the entry: an entry near zero is a
    cancellation of terms of typical size.  float32-level results (tol >= 1e-7):
    |out_i - ref_i| <= 2 tol (|ref_i| + max|ref|): float32 sums round each partial sum,
    so the error of an entry is a few float32 ulps of the largest contributions to it,
    and the largest entry-wise error measured is about twice the 2-norm error (far-field
    double layer, 8 spheres: 4.8e-7 in the 2-norm, 1.07e-6 of the largest entry).  Either
    way a defect confined to a few entries fails here although it may pass the 2-norm."""
    a = np.asarray(out, dtype=np.float64).reshape(-1)
    b = np.asarray(ref, dtype=np.float64).reshape(-1)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), (what, "non-finite entries", int(np.count_nonzero(~np.isfinite(a))))
    if b.size == 0:
        return
    rms = float(np.sqrt(np.mean(b * b)))
    bmax = float(np.abs(b).max())
    if tol >= 1e-7:
        bound = 2.0 * tol * (np.abs(b) + bmax)
    else:
        bound = tol * (np.abs(b) + rms)
    err = np.abs(a - b)
    worst = int(np.argmax(err / np.maximum(bound, 1e-300)))
    ratio = float(err[worst] / max(bound[worst], 1e-300))
    re = rel_err(a, b)
    assert ratio <= 1.0, (what, f"entry {worst}: |out - ref| = {err[worst]:.3e} > {bound[worst]:.3e} "
                                f"(ratio {ratio:.2f}); ref {b[worst]:.6e}, rms {rms:.3e}, max {bmax:.3e}; "
                                f"rel 2-norm {re:.3e}; max|d|/max|ref| {err.max() / max(bmax, 1e-300):.3e}")
    assert re < tol, (what, f"relative 2-norm {re:.3e} >= {tol:.1e} (worst entry ratio {ratio:.2f})")


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def small_cluster(n=12, box=9.0, gap=0.15, seed=3):
    """A dense cluster with several near pairs and a ragged node count."""
    rng = np.random.default_rng(seed)
    return place_spheres(n, box, gap, rng)


def poly_cluster():
    """Six spheres of radii 0.35-1.4, gaps 0.12-0.9 among the near pairs."""
    c = np.array([[0.0, 0.0, 0.0], [2.2, 0.3, -0.1], [0.4, 1.75, 0.5], [-1.5, -0.6, 0.9],
                  [1.3, -1.4, 1.2], [4.4, 2.2, 0.4]])
    a = np.array([1.0, 1.1, 0.45, 0.6, 0.35, 1.4])
    return c, a


def oracle_coef_to_gpu(ops, coef_o, nb):
    """Oracle coefficients (per sphere list of (3, M)) -> GPU layout (nb, 3, ncoef, 2)."""
    g = ops.g
    slots = [(m, n) for m in range(g.mmax + 1) for n in range(m, g.p + 1)]
    idx = [ops.vsh.modes.index((n, m)) for (m, n) in slots]
    out = np.zeros((nb, 3, len(slots), 2))
    for k in range(nb):
        c = coef_o[k][:, idx]
        out[k, :, :, 0] = c.real
        out[k, :, :, 1] = c.imag
    return out


__all__ = ["rel_err", "assert_close", "max_rel", "small_cluster", "poly_cluster", "oracle_coef_to_gpu", "make_workload"]
