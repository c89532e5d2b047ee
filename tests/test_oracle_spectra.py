"""Pins for oracle/spectra.py and oracle/kernels.py (Theorem 2, Eqs. 3.6-3.12, A.4, A.7,
Eqs. 2.19-2.21): brute-force smooth quadrature of the kernels on a fine grid, the
continuity equation A.4, the double-layer identity and the translating-sphere flow."""
import math

import numpy as np
import pytest

from oracle import kernels, spectra
from oracle.grid import sphere_grid
from oracle.harmonics import vsh_at

FINE = sphere_grid(64)
FINE_Y = vsh_at(FINE["xhat"], 7, 7)


def _brute(density, x, a_s, a_d, grid=FINE):
    K = kernels.kernel_block(x, grid["xhat"], grid["xhat"], a_s, a_d)
    return np.einsum("tisj,sj->ti", K, density * grid["wnode"][:, None])


def _formula(fam, n, m, x, a_s, a_d):
    r = np.linalg.norm(x, axis=1)
    modes, _, V, W, X = vsh_at(x / r[:, None], n, n)
    j = modes.index((n, m))
    f = [a_s * np.asarray(s) + a_d * np.asarray(d) for s, d in zip(spectra.exterior_S(n, r), spectra.exterior_D(n, r))]
    fvv, fww, fwv, fxx = f
    if fam == 0:
        return fvv[:, None] * V[j]
    if fam == 1:
        return fww[:, None] * W[j] + fwv[:, None] * V[j]
    return fxx[:, None] * X[j]


TARGETS = np.array([[0.3, -0.4, 2.0], [1.5, 1.0, -1.2], [0.0, 0.0, 3.0], [-4.0, 2.5, 1.0], [0.0, 0.0, -2.2]])


# (n, family): V_n for n >= 0; W_n and X_n exist from n = 1 on (W_0 = X_0 = 0)
CASES = [(n, fam) for n in (0, 1, 2, 3, 5, 7) for fam in (0, 1, 2) if n > 0 or fam == 0]


@pytest.mark.parametrize("n,fam", CASES)
@pytest.mark.parametrize("op", [(1.0, 0.0), (0.0, 1.0)])
def test_exterior_formulas_vs_brute_force(n, fam, op):
    modes = FINE_Y[0]
    Z = FINE_Y[2 + fam]
    for m in sorted({0, min(n, 1), n, -n}):
        dens = Z[modes.index((n, m))]
        ub = _brute(dens, TARGETS, *op)
        uf = _formula(fam, n, m, TARGETS, *op)
        scale = max(1.0, np.abs(dens).max())
        assert np.abs(ub - uf).max() < 1e-11 * scale, (n, m, fam, op)


@pytest.mark.parametrize("n", [1, 2, 4])
def test_close_to_surface_limit_gives_table(n):
    # at r = 1.08 the fine quadrature is still accurate; the exterior formulas are
    # polynomials in 1/r, so agreement there plus the r -> 1 limit fixes Table 3.12
    grid = sphere_grid(160)
    modes, _, V, W, X = vsh_at(grid["xhat"], n, n)
    x = np.array([[0.0, 0.0, 1.08], [0.6, 0.0, -0.8 * 1.08 / 1.0]])
    x[1] *= 1.08 / np.linalg.norm(x[1])
    for fam, Z in enumerate([V, W, X]):
        dens = Z[modes.index((n, 1 if n >= 1 else 0))]
        for op in [(1.0, 0.0), (0.0, 1.0)]:
            ub = _brute(dens, x, *op, grid=grid)
            uf = _formula(fam, n, 1, x, *op)
            assert np.abs(ub - uf).max() < 1e-8
    # r -> 1 limits of the exterior branches equal the S and D_+ rows of Table 3.12
    for fam in range(3):
        s1 = spectra.exterior_S(n, 1.0)
        d1 = spectra.exterior_D(n, 1.0)
        diag = {0: 0, 1: 1, 2: 3}[fam]
        assert abs(s1[diag] - spectra.eig_S(n)[fam]) < 1e-15
        assert abs(d1[diag] - spectra.eig_Dplus(n)[fam]) < 1e-15
    assert abs(spectra.exterior_S(n, 1.0)[2]) < 1e-15 and abs(spectra.exterior_D(n, 1.0)[2]) < 1e-15


def test_jump_relation_and_principal_value():
    for n in range(0, 12):
        dp, dm, pv = spectra.eig_Dplus(n), spectra.eig_Dminus(n), spectra.eig_Dpv(n)
        for f in range(3):
            if n == 0 and f > 0:
                continue
            assert abs(dp[f] - dm[f] - 1.0) < 1e-14          # A.7
            assert abs(pv[f] - 0.5 * (dp[f] + dm[f])) < 1e-14


def test_double_layer_identity_on_constants():
    # D[c] = -c inside the sphere, 0 outside; on the surface the principal value is -c/2
    g = sphere_grid(48)
    c = np.array([0.4, -1.1, 2.0])
    dens = np.tile(c, (g["xhat"].shape[0], 1))
    inside = np.array([[0.0, 0.0, 0.0], [0.2, -0.3, 0.4], [-0.5, 0.1, 0.2]])
    outside = np.array([[0.0, 0.0, 2.5], [3.0, 1.0, -1.0]])
    assert np.abs(_brute(dens, inside, 0.0, 1.0, g) + c).max() < 1e-12
    assert np.abs(_brute(dens, outside, 0.0, 1.0, g)).max() < 1e-12
    assert spectra.eig_Dpv(1)[1] == -0.5 and spectra.eig_Dpv(1)[2] == -0.5


def test_continuity_equation_A4_exterior():
    # u = f V + g W + h X must satisfy (n+1) r f' + (n+1)(n+2) f - n r g' + n(n-1) g = 0
    r = np.linspace(1.2, 4.0, 9)
    h = 1e-6
    for n in range(1, 9):
        for ext in (spectra.exterior_S, spectra.exterior_D):
            # density W: f = fWV, g = fWW ; density V: f = fVV, g = 0
            for sel in [(2, 1), (0, None)]:
                fr = lambda rr: np.asarray(ext(n, rr)[sel[0]])
                gr = (lambda rr: np.asarray(ext(n, rr)[sel[1]])) if sel[1] is not None else (lambda rr: 0 * rr)
                fp = (fr(r + h) - fr(r - h)) / (2 * h)
                gp = (gr(r + h) - gr(r - h)) / (2 * h)
                res = (n + 1) * r * fp + (n + 1) * (n + 2) * fr(r) - n * r * gp + n * (n - 1) * gr(r)
                assert np.abs(res).max() < 1e-7, (n, ext.__name__, sel)


def test_translating_sphere_far_field():
    # S[c] for a constant density c is the flow of a sphere translating with U = 2c/3
    c = np.array([0.2, -0.7, 1.3])
    x = np.array([[0.0, 2.0, 1.0], [3.0, -1.0, 0.5], [0.0, 0.0, 1.5]])
    r = np.linalg.norm(x, axis=1)
    xh = x / r[:, None]
    cx = xh @ c
    exact = 0.5 * (c[None] / r[:, None] + cx[:, None] * xh / r[:, None]) \
        + (1.0 / 6.0) * (c[None] / r[:, None] ** 3 - 3 * cx[:, None] * xh / r[:, None] ** 3)
    # constant c = sqrt(4pi/3) sum over W_1 components; build it from the series directly
    modes, _, V, W, X = vsh_at(xh, 1, 1)
    g = sphere_grid(6)
    _, _, Vg, Wg, Xg = vsh_at(g["xhat"], 1, 1)
    dens = np.tile(c, (g["xhat"].shape[0], 1))
    u = np.zeros((3, 3), dtype=complex)
    for j, (n, m) in enumerate(modes):
        if n != 1:
            continue
        coef = np.sum(g["wnode"][:, None] * dens * np.conj(Wg[j])) / (n * (2 * n + 1))
        fvv, fww, fwv, fxx = spectra.exterior_S(1, r)
        u += coef * (fww[:, None] * W[j] + fwv[:, None] * V[j])
    assert np.abs(u.real - exact).max() < 1e-14
    dens_f = np.tile(c, (FINE["xhat"].shape[0], 1))
    assert np.abs(_brute(dens_f, x, 1.0, 0.0) - exact).max() < 1e-12
