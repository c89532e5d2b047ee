"""Velocity at arbitrary points of the fluid, and the porous-media problem (Problem 1).

Test infrastructure only (see ``oracle/__init__.py``).

For a density on the n_b unit spheres, the layer potential a_S S + a_D D (plus, for the
completed form, the completion flow N of Eqs. 5.18-5.19) is evaluated at a point x of
the fluid sphere by sphere, with the same separation test as on the surfaces (Eq. 4.5,
read as: near iff the distance from x to the surface of sphere k, |x - c_k| - 1, is
below d*):

* near spheres: the exterior series of Eqs. 3.6-3.11 from the sphere's VSH coefficients
  (Section 3; the series converges for |x - c_k| > 1);
* other spheres: the smooth quadrature of Eq. 4.4 over the sphere's nodes;
* completion: Stokeslet of int psi and rotlet of int (y - c_k) x psi at every centre.

Problem 1 (Eqs. 5.3-5.4): spheres held fixed in an imposed flow u_inf; the density solves
(1/2 I + sum_k (S_k + D_k)) mu = -u_inf on the surfaces and the flow is
u = u_inf + sum_k (S_k + D_k)[mu].

Parity: pinned by tests/test_oracle_field.py (one sphere in a uniform stream against the
textbook flow past a fixed sphere; the exterior limit at the surface equals
1/2 mu + S mu + D_pv mu (jump relation, Eq. A.7); series and quadrature agree where both
converge).
"""
import numpy as np

from . import kernels
from .operators import OPS, Operators


def evaluate(geom, mu, x, op="SD_BIE", ops=None):
    """Layer potential of `op` (S, D, SD_BIE or DN_BIE; the identity term of the
    second-kind forms is a surface term and does not enter) of the node density mu (N, 3)
    at fluid points x (K, 3).  Raises ValueError for a point inside a sphere."""
    ops = ops or Operators(geom)
    a_s, a_d, _c, compl = OPS[op]
    g = geom
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    mu = np.asarray(mu, dtype=np.float64).reshape(g.N, 3)
    # distance to the surface; spheres of radius a: near when below d* a (Eq. 4.5 scaled)
    dist = np.linalg.norm(x[:, None, :] - g.centres[None, :, :], axis=-1) - g.radii[None, :]
    if (dist <= 0.0).any():
        raise ValueError("evaluation point inside or on a sphere")
    q = mu * g.w[:, None]
    out = np.zeros((x.shape[0], 3))
    for k in range(g.nb):
        sl = g.sphere_nodes(k)
        near = dist[:, k] < g.near_gap * g.radii[k]
        if near.any():
            coef = ops.coefficients(mu[:, :, None], k)
            out[near] += ops.near_field_from(coef, g.centres[k], x[near], a_s, a_d, g.radii[k])[..., 0]
        far = ~near
        if far.any():
            out[far] += kernels.direct_sum(x[far], g.nodes[sl], g.xhat[sl], q[sl][:, :, None], a_s, a_d)[..., 0]
    if compl:
        F, T = ops.moments(mu[:, :, None])
        for k in range(g.nb):
            out += kernels.stokeslet_rotlet(x, g.centres[k], F[k], T[k])[..., 0]
    return out
