"""Operator spectra and exterior layer-potential formulas (Section 3.2).

Test infrastructure only (see ``oracle/__init__.py``).

* Theorem 2 / Table 3.12: eigenvalues of S, D_+ (exterior limit), D_- (interior limit)
  on V_n^m, W_n^m, X_n^m.  The principal value on the surface is D_pv = D_+ - 1/2
  (jump condition A.7: D_+ - D_- = identity).
* Eqs. 3.6-3.11, exterior branches (r > 1): S[Z] and D[Z] away from the sphere.
  Only exterior branches are used: every target of a near correction lies outside its
  source sphere.

Degree zero: W_0 and X_0 vanish identically, so their entries are returned as 0.

Parity: pinned by tests/test_oracle_spectra.py against brute-force smooth quadrature on
an upsampled grid at several radii (which also fixes the surface eigenvalues through
the r -> 1 limit), the continuity equation A.4, the double-layer identity on rigid-body
densities, and the translating-sphere far field.
"""


def eig_S(n):
    """Table 3.12, row S: (V, W, X)."""
    v = n / ((2 * n + 1) * (2 * n + 3))
    w = (n + 1) / ((2 * n + 1) * (2 * n - 1)) if n >= 1 else 0.0
    x = 1.0 / (2 * n + 1) if n >= 1 else 0.0
    return v, w, x


def eig_Dplus(n):
    """Table 3.12, row D_+ (exterior limit): (V, W, X)."""
    v = (2 * n * n + 4 * n + 3) / ((2 * n + 1) * (2 * n + 3))
    w = 2.0 * (n - 1) * (n + 1) / ((2 * n + 1) * (2 * n - 1)) if n >= 1 else 0.0
    x = (n - 1) / (2 * n + 1) if n >= 1 else 0.0
    return v, w, x


def eig_Dminus(n):
    """Table 3.12, row D_- (interior limit): (V, W, X)."""
    v = -2.0 * n * (n + 2) / ((2 * n + 1) * (2 * n + 3))
    w = -(2.0 * n * n + 1) / ((2 * n + 1) * (2 * n - 1)) if n >= 1 else 0.0
    x = -(n + 2.0) / (2 * n + 1) if n >= 1 else 0.0
    return v, w, x


def eig_Dpv(n):
    """Principal value D_pv = D_+ - 1/2 on the surface (jump A.7); zero where the
    harmonic itself vanishes (W_0, X_0)."""
    v, w, x = eig_Dplus(n)
    return v - 0.5, (w - 0.5) if n >= 1 else 0.0, (x - 0.5) if n >= 1 else 0.0


def exterior_S(n, r):
    """Eqs. 3.6-3.8, r >= 1.  Returns (fVV, fWW, fWV, fXX): the field of S[V] is
    fVV V, of S[W] is fWW W + fWV V, of S[X] is fXX X (harmonics at the target angles)."""
    fvv = n / ((2 * n + 1) * (2 * n + 3)) * r ** (-n - 2)
    if n == 0:
        return fvv, 0.0, 0.0, 0.0
    fww = (n + 1) / ((2 * n + 1) * (2 * n - 1)) * r ** (-n)
    fwv = n / (4 * n + 2) * (r ** (-n - 2) - r ** (-n))
    fxx = 1.0 / (2 * n + 1) * r ** (-n - 1)
    return fvv, fww, fwv, fxx


def exterior_D(n, r):
    """Eqs. 3.9-3.11, r > 1.  Same layout as exterior_S."""
    fvv = (2 * n * n + 4 * n + 3) / ((2 * n + 1) * (2 * n + 3)) * r ** (-n - 2)
    if n == 0:
        return fvv, 0.0, 0.0, 0.0
    fww = 2.0 * (n + 1) * (n - 1) / ((2 * n + 1) * (2 * n - 1)) * r ** (-n)
    fwv = 2.0 * n * (n - 1) / (4 * n + 2) * (r ** (-n - 2) - r ** (-n))
    fxx = (n - 1) / (2 * n + 1) * r ** (-n - 1)
    return fvv, fww, fwv, fxx
