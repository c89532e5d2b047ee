"""Stokes kernels and direct (smooth-quadrature) sums (Section 2.2, Eqs. 2.19-2.21; Eq. 4.4).

Test infrastructure only (see ``oracle/__init__.py``).

Viscosity is 1 (Section 5).  The double-layer kernel carries the conventional sign
D_ij(x, y) = +3/(4 pi) r_i r_j (r . n_y)/|r|^5, r = x - y, under which D[c] = -c inside a
sphere and 0 outside, matching Table 3.12 and the jump A.7 (the printed stresslet of
Eq. 2.20 has the opposite overall sign).

Parity: pinned by tests/test_oracle_spectra.py (double-layer identity, exterior
formulas by brute force) and tests/test_oracle_solve.py (Stokes drag 6 pi, 8 pi).
"""
import math

import numpy as np

C_S = 1.0 / (8.0 * math.pi)
C_D = 3.0 / (4.0 * math.pi)


def kernel_block(x, y, ny, a_s, a_d):
    """Dense block K[t, i, s, j] of a_s * Stokeslet(x_t, y_s) + a_d * double layer with
    source normal ny_s.  x (T, 3), y (S, 3), ny (S, 3) -> (T, 3, S, 3)."""
    r = x[:, None, :] - y[None, :, :]                         # (T, S, 3)
    r2 = np.einsum("tsi,tsi->ts", r, r)
    ir = 1.0 / np.sqrt(r2)
    ir2 = ir * ir
    rr = np.einsum("tsi,tsj->tisj", r, r)                     # (T, 3, S, 3)
    K = np.zeros_like(rr)
    if a_s != 0.0:
        eye = np.eye(3)[None, :, None, :]
        K += a_s * C_S * (eye * ir[:, None, :, None] + rr * (ir * ir2)[:, None, :, None])
    if a_d != 0.0:
        rn = np.einsum("tsi,si->ts", r, ny)
        K += a_d * C_D * rr * (rn * ir2 * ir2 * ir)[:, None, :, None]
    return K


def direct_sum(x, y, ny, q, a_s, a_d, chunk=4096):
    """u(x_t) = sum_s K(x_t, y_s) q_s with q = w * density already multiplied by the
    quadrature weight.  q (S, 3, B) -> (T, 3, B)."""
    T = x.shape[0]
    B = q.shape[2]
    out = np.zeros((T, 3, B))
    for s0 in range(0, y.shape[0], chunk):
        s1 = min(y.shape[0], s0 + chunk)
        K = kernel_block(x, y[s0:s1], ny[s0:s1], a_s, a_d)
        out += np.einsum("tisj,sjb->tib", K, q[s0:s1])
    return out


def stokeslet_rotlet(x, c, F, T):
    """Flow of a point force F (Stokeslet, Eq. 2.19) and a point torque T (rotlet,
    T x r / (8 pi |r|^3)) located at c, evaluated at x.  x (K, 3), F/T (3, B)."""
    r = x - c[None, :]
    r2 = np.sum(r * r, axis=1)
    ir = 1.0 / np.sqrt(r2)
    ir3 = ir ** 3
    rF = np.einsum("ki,ib->kb", r, F)
    u = C_S * (F[None, :, :] * ir[:, None, None] + r[:, :, None] * (rF * ir3[:, None])[:, None, :])
    Txr = np.cross(T.T[None, :, :], r[:, None, :], axis=-1)   # (K, B, 3)
    u += C_S * np.transpose(Txr, (0, 2, 1)) * ir3[:, None, None]
    return u
