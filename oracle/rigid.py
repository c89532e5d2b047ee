"""Global rigid-mode coarse correction of the resistance form: the definitions the HIP
path must reproduce.

Test infrastructure only (see ``oracle/__init__.py``).

The paper has no preconditioner.  In the completed double-layer form (Eqs. 5.18-5.19)
the rigid-body densities of a sphere (W_1 and X_1, the null space of D_+ in Table 3.12)
interact with the other spheres only through the completion flow N: a rigid density
a + b x x on sphere k carries the force F = 4 pi a and torque T = 8 pi / 3 b, its
exterior double layer vanishes, and the Stokeslet + rotlet it induces decays like 1/r.
Over many spheres that coupling has a wide spectrum, which the sphere-by-sphere inverse
M0 cannot see.  The correction solves for it on the coarse space of 6 rigid modes per
sphere:

    z = z0 + P (y - R z0),   A_c y = R r,   z0 = M0 r (or the learned correction's output),

* R f = per sphere (a, b): a = (1/4 pi) int f, b = (3/8 pi) int x x f (Eq. 4.4 weights),
  the projection onto the rigid fields (W_1 and X_1 are orthogonal to every other vector
  spherical harmonic, Definition 2.2); P (a, b) = a + b x x.  R P = I.
* A_c = M S, S = diag(4 pi I, 8 pi / 3 I) per sphere (rigid coefficients -> F, T), and
  M the Rotne-Prager-Yamakawa grand mobility of unit spheres (translation-translation
  (1/8 pi d)[(1 + 2/(3 d^2)) I + (1 - 2/d^2) e e], translation-rotation and
  rotation-translation -(1/8 pi d^3) [r]_x, rotation-rotation -(1/16 pi d^3)(I - 3 e e);
  self blocks I/(6 pi), I/(8 pi)), r = c_i - c_k, d = |r|, e = r/d.
  The exact restriction R A P of the discretised operator is the same except that its
  translation-translation block averages the Stokeslet over the target sphere only
  ((1 + 1/(3 d^2)) I + (1 - 1/d^2) e e); that one-sided matrix is indefinite for close
  pairs (gap 0.02), the Rotne-Prager one is positive definite for any configuration of
  non-overlapping spheres, so it is the one used.
* For M0, R M0 P = diag(3/2, 3) = (A_c of an isolated sphere)^-1: on one sphere the
  correction vanishes.
* Spheres of radius a: R f = (int f / (4 pi a^2), 3 int (x - c) x f / (8 pi a^4)) (the
  mean velocity and rotation of f), P (a, b) = a + b x (x - c), S = diag(4 pi a^2,
  8 pi a^4 / 3) (the force and torque of a rigid density, Eq. 5.19's N), and M the
  polydisperse Rotne-Prager-Yamakawa mobility: self blocks I/(6 pi a), I/(8 pi a^3),
  translation-translation (1/8 pi d)[(1 + (a_i^2 + a_k^2)/(3 d^2)) I +
  (1 - (a_i^2 + a_k^2)/d^2) e e] (the Stokeslet averaged over both spheres), rotation
  blocks as above.  R M0 P = diag(3/(2a), 3/a) = (A_c of an isolated sphere)^-1.

Parity: pinned by tests/test_oracle_rigid.py (R A P of the oracle operator equals the
one-sided closed form; the translation block of M equals the two-sided surface average
of the Stokeslet by quadrature; the rotation blocks equal the one-sided restriction;
R P = I; R M0 P = diag(3/2, 3); positive definiteness; no-op on an isolated sphere).
"""
import math

import numpy as np

B0 = np.array([1.5] * 3 + [3.0] * 3)
S_DIAG = np.array([4.0 * math.pi] * 3 + [8.0 * math.pi / 3.0] * 3)


def b0(a=1.0):
    """R M0 P on a sphere of radius a."""
    return np.array([1.5 / a] * 3 + [3.0 / a] * 3)


def s_diag(a=1.0):
    return np.array([4.0 * math.pi * a ** 2] * 3 + [8.0 * math.pi * a ** 4 / 3.0] * 3)


def restrict(field, xhat, w, a=1.0):
    """(6,) rigid coefficients (a, b) of one sphere's node field (P, 3); xhat the unit
    offsets and w the unit-sphere weights, the sphere's radius a."""
    v = (w[:, None] * field).sum(0) / (4.0 * math.pi)
    b = (w[:, None] * np.cross(xhat, field)).sum(0) * (3.0 / (8.0 * math.pi * a))
    return np.concatenate([v, b])


def prolong(y, xhat, a=1.0):
    """Node field (P, 3) of the rigid coefficients y = (a, b): a + b x (x - c)."""
    return y[None, :3] + np.cross(y[None, 3:], a * xhat)


def _cross_matrix(r):
    x, y, z = r
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def mobility(centres, two_sided=True, radii=None):
    """(6 n_b, 6 n_b) grand mobility: Rotne-Prager-Yamakawa (two_sided) or the one-sided
    surface average that equals the operator's own restriction."""
    nb = len(centres)
    a = np.ones(nb) if radii is None else np.asarray(radii, dtype=np.float64)
    M = np.zeros((6 * nb, 6 * nb))
    I3 = np.eye(3)
    for i in range(nb):
        M[6 * i:6 * i + 3, 6 * i:6 * i + 3] = I3 / (6.0 * math.pi * a[i])
        M[6 * i + 3:6 * i + 6, 6 * i + 3:6 * i + 6] = I3 / (8.0 * math.pi * a[i] ** 3)
        for k in range(nb):
            if k == i:
                continue
            f = a[i] ** 2 + a[k] ** 2 if two_sided else a[i] ** 2
            r = centres[i] - centres[k]
            d = np.linalg.norm(r)
            e = r / d
            ee = np.outer(e, e)
            tt = ((1.0 / d + f / (3.0 * d ** 3)) * I3 + (1.0 / d - f / d ** 3) * ee) / (8.0 * math.pi)
            tr = -_cross_matrix(r) / (8.0 * math.pi * d ** 3)
            rr = -(I3 - 3.0 * ee) / (16.0 * math.pi * d ** 3)
            M[6 * i:6 * i + 3, 6 * k:6 * k + 3] = tt
            M[6 * i:6 * i + 3, 6 * k + 3:6 * k + 6] = tr
            M[6 * i + 3:6 * i + 6, 6 * k:6 * k + 3] = tr
            M[6 * i + 3:6 * i + 6, 6 * k + 3:6 * k + 6] = rr
    return M


def coarse_operator(centres, two_sided=True, radii=None):
    """A_c = M S: rigid coefficients of every sphere -> rigid part of the response."""
    nb = len(centres)
    a = np.ones(nb) if radii is None else np.asarray(radii, dtype=np.float64)
    return mobility(centres, two_sided, a) * np.concatenate([s_diag(x) for x in a])[None, :]


def correct(geom, r, z0):
    """z = z0 + P (A_c^-1 R r - R z0) over all spheres (dense solve)."""
    xh = geom.grid["xhat"]
    w = geom.grid["wnode"]
    nb = geom.nb
    a = geom.radii
    xi = np.concatenate([restrict(r[geom.sphere_nodes(k)], xh, w, a[k]) for k in range(nb)])
    zeta = np.concatenate([restrict(z0[geom.sphere_nodes(k)], xh, w, a[k]) for k in range(nb)])
    y = np.linalg.solve(coarse_operator(geom.centres, radii=a), xi)
    d = (y - zeta).reshape(nb, 6)
    out = z0.copy()
    for k in range(nb):
        out[geom.sphere_nodes(k)] += prolong(d[k], xh, a[k])
    return out
