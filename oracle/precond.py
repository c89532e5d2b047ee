"""Block preconditioner M0: the inverse of every sphere's isolated self operator.

Test infrastructure only (see ``oracle/__init__.py``).

Resistance form 1/2 + D_pv + N on one unit sphere (Eq. 5.19, Table 3.12): diagonal in
V, W, X with eigenvalue D_+ except on degree one, where D_+ vanishes on W_1 and X_1 and
the completion flow N maps W_1[b] -> 2/3 W_1[b] - 1/6 V_1[b] and X_1 -> 1/3 X_1; on the
grid complement of the band-limited space the operator is 1/2.  Hence
    M0 r = 2 r + Pi^+ (L - 2) Pi r,   L = 1/D_+ per mode except
    V_1: 5/3 (plus 5/12 of the W_1 coefficient), W_1: 3/2, X_1: 3.
On a sphere of radius a the completion's moments carry a^2 (force) and a^3 (torque) and
are felt at distance a, so N maps W_1 -> 2a/3 W_1 - a/6 V_1 and X_1 -> a/3 X_1: W_1 and
X_1 become 3/(2a) and 3/a, the V_1 coupling stays 5/12.

Parity: pinned by tests/test_oracle_coarse.py (M0 inverts the isolated operator).
"""
import numpy as np

from . import spectra
from .harmonics import DenseVSH


def m0_resistance(geom, r):
    vsh = DenseVSH(geom.grid, geom.p, geom.mmax)
    out = np.empty_like(r)
    lam = np.zeros((3, len(vsh.modes)))
    i1 = [i for i, (n, m) in enumerate(vsh.modes) if n == 1]
    for i, (n, m) in enumerate(vsh.modes):
        dp = spectra.eig_Dplus(n)
        for f in range(3):
            if f > 0 and n == 0:
                continue
            lam[f, i] = {0: 5.0 / 3.0, 1: 1.5, 2: 3.0}[f] if n == 1 else 1.0 / dp[f]
    for k in range(geom.nb):
        sl = geom.sphere_nodes(k)
        c = vsh.forward(r[sl])
        lk = lam.copy()
        lk[1, i1] /= geom.radii[k]
        lk[2, i1] /= geom.radii[k]
        d = (lk - 2.0) * c
        d[0, i1] += (5.0 / 12.0) * c[1, i1]
        out[sl] = 2.0 * r[sl] + vsh.inverse(d)
    return out
