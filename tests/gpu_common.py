"""Shared helpers of the GPU parity tests (seeded inputs, oracle comparison)."""
import numpy as np

from paper_1707_06551_amd.inputs import make_workload, place_spheres


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


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


__all__ = ["rel_err", "max_rel", "small_cluster", "poly_cluster", "oracle_coef_to_gpu", "make_workload"]
