"""Learned close-pair coarse correction: the definitions the HIP path must reproduce.

Test infrastructure only (see ``oracle/__init__.py``).

The paper gives no preconditioner; this is a learned block correction (an addition to
the method: a small per-sphere network over neighbour geometry that predicts the
coupling of close pairs), written here from its definition:

    M_MLP r = M0 r + P zeta,   zeta_i = sum_{j in near(i)} Q_ij^T [K_off(theta_ij) Q_ij rho_j
                                                              + K_self(theta_ij) Q_ij rho_i],
    rho = R r.

* Coarse space: per sphere the vector spherical harmonics of degree <= 2 (Definition
  2.2), in a Cartesian parametrisation (25 coefficients):
    s           V_0 = -x            (field s x)
    a (3)       V_1[a] = a - 3 (a.x) x
    b (3)       W_1[b] = b
    c (3)       X_1-type c x x
    tV (5)      V_2[T] = 2 T x - 5 (x.T x) x
    tW (5)      W_2[T] = 2 T x
    tX (5)      X_2[T] = 2 x x (T x)
  with T = sum_k t_k E_k over an orthonormal basis E_1..E_5 of symmetric traceless
  matrices (xy, yz, xz, xx - yy, 2zz - xx - yy; Frobenius-normalised).  x is the unit
  normal.  These span the same space as V, W, X with n <= 2 (W_n = grad of the solid
  harmonic r^n Y_n, V_n = W_n - (2n+1) Y_n x, X_n = x cross W_n).
* R r: weighted (Eq. 4.4) projection onto those 25 fields; P: synthesis.  R P = I.
* Pair frame of the directed near pair (i, j): rotation Q_ij with Q d = z, d the unit
  vector from c_i to c_j; a 25-vector rotates as (s, Q a, Q b, Q c, D2 tV, D2 tW, D2 tX)
  with D2_kl = tr(E_k Q E_l Q^T).
* K(theta): a 25 x 25 map in the pair frame that commutes with rotations about z:
  arbitrary on the 7 m = 0 components, alpha I + beta J on pairs of |m| = 1 and |m| = 2
  doublets (139 parameters).  theta_ij (278 = 2 x 139) comes from the MLP applied to
  the pair's features.

Parity: pinned by tests/test_oracle_coarse.py (R P = I, equivariance of the correction
under a rigid rotation of the configuration, invariance under the choice of the pair
frame's transverse axes, gradients against central finite differences).
"""
import math

import numpy as np

NLOW = 25
NTHETA = 139

_S2 = 1.0 / math.sqrt(2.0)
_S6 = 1.0 / math.sqrt(6.0)
E_BASIS = np.array([
    [[0, _S2, 0], [_S2, 0, 0], [0, 0, 0]],          # xy
    [[0, 0, 0], [0, 0, _S2], [0, _S2, 0]],          # yz
    [[0, 0, _S2], [0, 0, 0], [_S2, 0, 0]],          # xz
    [[_S2, 0, 0], [0, -_S2, 0], [0, 0, 0]],         # xx - yy
    [[-_S6, 0, 0], [0, -_S6, 0], [0, 0, 2 * _S6]],  # 2zz - xx - yy
])

# index layout of the 25-vector
I_S, I_A, I_B, I_C, I_TV, I_TW, I_TX = 0, 1, 4, 7, 10, 15, 20
# m = 0 components; |m| = 1 doublets (x-like, y-like); |m| = 2 doublets (cos-like, sin-like)
M0_IDX = [0, 3, 6, 9, 14, 19, 24]
M1_DOUBLETS = [(1, 2), (4, 5), (7, 8), (12, 11), (17, 16), (22, 21)]
M2_DOUBLETS = [(13, 10), (18, 15), (23, 20)]


def lowmode_fields(xhat):
    """The 25 basis fields at unit normals xhat (K, 3) -> (K, 25, 3)."""
    x = np.asarray(xhat, dtype=np.float64)
    K = x.shape[0]
    F = np.zeros((K, NLOW, 3))
    F[:, I_S] = x
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        F[:, I_A + k] = e[None, :] - 3.0 * x[:, k:k + 1] * x
        F[:, I_B + k] = e[None, :]
        F[:, I_C + k] = np.cross(e[None, :], x)
    for k in range(5):
        T = E_BASIS[k]
        Tx = x @ T.T
        xTx = np.einsum("ki,ki->k", x, Tx)
        F[:, I_TW + k] = 2.0 * Tx
        F[:, I_TV + k] = 2.0 * Tx - 5.0 * xTx[:, None] * x
        F[:, I_TX + k] = 2.0 * np.cross(x, Tx)
    return F


def norms(xhat, w):
    F = lowmode_fields(xhat)
    return np.einsum("k,kmc,kmc->m", w, F, F)


def restrict(field, xhat, w):
    """rho (25,) of a node field (K, 3) on one sphere: weighted projection."""
    F = lowmode_fields(xhat)
    return np.einsum("k,kmc,kc->m", w, F, field) / norms(xhat, w)


def prolong(rho, xhat):
    return np.einsum("m,kmc->kc", rho, lowmode_fields(xhat))


def pair_frame(d):
    """Rotation Q (rows e1, e2, d) with Q d = z."""
    d = np.asarray(d, dtype=np.float64) / np.linalg.norm(d)
    a = np.zeros(3)
    a[int(np.argmin(np.abs(d)))] = 1.0
    e1 = np.cross(a, d)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    return np.stack([e1, e2, d])


def rot25(Q):
    """25 x 25 matrix taking global-frame coefficients to the frame of Q."""
    Rm = np.zeros((NLOW, NLOW))
    Rm[I_S, I_S] = 1.0
    for base in (I_A, I_B, I_C):
        Rm[base:base + 3, base:base + 3] = Q
    D2 = np.array([[np.trace(E_BASIS[k] @ Q @ E_BASIS[l] @ Q.T) for l in range(5)] for k in range(5)])
    for base in (I_TV, I_TW, I_TX):
        Rm[base:base + 5, base:base + 5] = D2
    return Rm


def K_from_theta(theta):
    """Axisymmetric 25 x 25 block from 139 parameters (layout: 49 m=0 entries row-major,
    then (alpha, beta) for each of the 36 |m|=1 doublet pairs (out, in) row-major, then 9
    |m|=2 doublet pairs)."""
    K = np.zeros((NLOW, NLOW))
    t = 0
    for p in M0_IDX:
        for q in M0_IDX:
            K[p, q] = theta[t]
            t += 1
    for doublets in (M1_DOUBLETS, M2_DOUBLETS):
        for (xp, yp) in doublets:
            for (xq, yq) in doublets:
                al, be = theta[t], theta[t + 1]
                t += 2
                K[xp, xq] = al
                K[yp, yq] = al
                K[xp, yq] = -be
                K[yp, xq] = be
    assert t == NTHETA
    return K


def theta_grad_from_K(dK):
    """Adjoint of K_from_theta: d(loss)/d(theta) from d(loss)/dK."""
    g = np.zeros(NTHETA)
    t = 0
    for p in M0_IDX:
        for q in M0_IDX:
            g[t] = dK[p, q]
            t += 1
    for doublets in (M1_DOUBLETS, M2_DOUBLETS):
        for (xp, yp) in doublets:
            for (xq, yq) in doublets:
                g[t] = dK[xp, xq] + dK[yp, yq]
                g[t + 1] = -dK[xp, yq] + dK[yp, xq]
                t += 2
    return g


NFEAT = 8


def pair_features(centres, near, near_gap):
    """Directed near pairs (i, j) of a configuration, their features (n, 8) and unit
    directions d = (c_j - c_i)/|c_j - c_i|.  Features: gap g, log(g + 0.01),
    0.1/(g + 0.1), near counts of i and j / 8, smallest gap of i to a neighbour other
    than j and of j to a neighbour other than i (near_gap if none), crowding of i
    sum_{k in near(i)} 0.1/(g_ik + 0.1)."""
    c = np.asarray(centres, dtype=np.float64)
    nb = c.shape[0]
    gap = np.linalg.norm(c[:, None] - c[None], axis=-1) - 2.0
    pairs, feats, dirs = [], [], []
    cnt = near.sum(axis=1)
    for i in range(nb):
        for j in np.nonzero(near[i])[0]:
            g = gap[i, j]
            oi = [gap[i, k] for k in np.nonzero(near[i])[0] if k != j]
            oj = [gap[j, k] for k in np.nonzero(near[j])[0] if k != i]
            crowd = sum(0.1 / (gap[i, k] + 0.1) for k in np.nonzero(near[i])[0])
            feats.append([g, math.log(g + 0.01), 0.1 / (g + 0.1), cnt[i] / 8.0, cnt[j] / 8.0,
                          min(oi) if oi else near_gap, min(oj) if oj else near_gap, crowd])
            d = c[j] - c[i]
            dirs.append(d / np.linalg.norm(d))
            pairs.append((i, j))
    return (np.array(pairs, dtype=np.int64).reshape(-1, 2), np.array(feats).reshape(-1, NFEAT),
            np.array(dirs).reshape(-1, 3))


def coarse_apply(pairs, dirs, theta, rho):
    """zeta (nb, 25) from rho (nb, 25) and per-pair parameters theta (npairs, 278)."""
    zeta = np.zeros_like(rho)
    for e, (i, j) in enumerate(pairs):
        Rm = rot25(pair_frame(dirs[e]))
        Ko = K_from_theta(theta[e, :NTHETA])
        Ks = K_from_theta(theta[e, NTHETA:])
        zeta[i] += Rm.T @ (Ko @ (Rm @ rho[j]) + Ks @ (Rm @ rho[i]))
    return zeta
