"""Linear solves for the resistance and mobility problems (Section 5, Problems 4-5).

Test infrastructure only (see ``oracle/__init__.py``).

The paper names no iterative solver.  Two textbook solvers are used here:
* dense LU (numpy.linalg.solve) on the matrix assembled column by column from the
  operator (small cases only);
* restarted GMRES(m) with modified Gram-Schmidt Arnoldi and Givens rotations
  (Saad, "Iterative Methods for Sparse Linear Systems", Alg. 6.9), x0 = 0, stopping on
  the relative residual of the least-squares estimate and confirmed on the true residual.

Right-hand sides:
* resistance (Eq. 5.19): b = v_i + omega_i x (x - c_i) on the nodes of sphere i;
  outputs F_k = int psi, T_k = int (y - c_k) x psi (force and torque the particle exerts
  on the fluid; an isolated sphere gives 6 pi v and 8 pi omega);
* mobility (bordered Eq. 5.17 with Eq. 5.15 set to the applied F, T):
  b = [u_s; F / (4 pi); 3 T / (8 pi)]; outputs v, omega.

Parity: GMRES pinned against dense LU; the drivers pinned by the isolated-sphere drag
and its inverse, the two-sphere far-field (Rotne-Prager) limit and exterior-solution
reproduction (tests/test_oracle_solve.py).
"""
import math

import numpy as np

from .operators import Operators


def assemble(apply_fn, n, block=256):
    """Dense matrix of a linear map R^n -> R^n, column block by column block."""
    A = np.zeros((n, n))
    for c0 in range(0, n, block):
        c1 = min(n, c0 + block)
        E = np.zeros((n, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        A[:, c0:c1] = apply_fn(E)
    return A


def gmres(apply_fn, b, tol=1e-10, restart=100, max_iter=1000):
    """Restarted GMRES(m), MGS Arnoldi + Givens rotations.  Returns (x, info) with
    info = dict(iters, rel_residual (true), history)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, dict(iters=0, rel_residual=0.0, history=[0.0])
    hist = []
    it = 0
    while it < max_iter:
        r = b - apply_fn(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= tol:
            break
        m = min(restart, max_iter - it)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            w = apply_fn(V[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                h0 = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                h1 = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j], H[i + 1, j] = h0, h1
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k_used = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or it >= max_iter:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + V[:k_used].T @ y
    r = b - apply_fn(x)
    return x, dict(iters=it, rel_residual=float(np.linalg.norm(r) / bnorm), history=hist)


def rigid_rhs(geom, v, omega):
    """v_i + omega_i x (x - c_i) at every node (N, 3)."""
    k = geom.sphere_of
    return v[k] + np.cross(omega[k], geom.nodes - geom.centres[k])


def solve_resistance(geom, v, omega, method="gmres", tol=1e-10, restart=100, max_iter=1000):
    ops = Operators(geom)
    b = rigid_rhs(geom, np.asarray(v, float), np.asarray(omega, float)).reshape(-1)
    fn = lambda z: ops.apply("DN_BIE", z.reshape(geom.N, 3, -1) if z.ndim == 2 else z.reshape(geom.N, 3)).reshape(z.shape)
    if method == "lu":
        A = assemble(fn, b.size)
        psi = np.linalg.solve(A, b)
        info = dict(iters=0, rel_residual=float(np.linalg.norm(A @ psi - b) / np.linalg.norm(b)))
    else:
        psi, info = gmres(fn, b, tol=tol, restart=restart, max_iter=max_iter)
    psi = psi.reshape(geom.N, 3)
    F, T = ops.moments(psi)
    return F[..., 0], T[..., 0], psi, info


def solve_mobility(geom, F, T, slip=None, method="gmres", tol=1e-10, restart=100, max_iter=1000):
    ops = Operators(geom)
    us = np.zeros((geom.N, 3)) if slip is None else np.asarray(slip, float)
    b = np.concatenate([us.reshape(-1), (np.asarray(F, float) / (4 * math.pi)).reshape(-1),
                        (3.0 * np.asarray(T, float) / (8 * math.pi)).reshape(-1)])
    fn = ops.apply_mobility
    if method == "lu":
        A = assemble(fn, b.size)
        x = np.linalg.solve(A, b)
        info = dict(iters=0, rel_residual=float(np.linalg.norm(A @ x - b) / np.linalg.norm(b)))
    else:
        x, info = gmres(fn, b, tol=tol, restart=restart, max_iter=max_iter)
    N, nb = geom.N, geom.nb
    mu = x[:3 * N].reshape(N, 3)
    v = x[3 * N:3 * N + 3 * nb].reshape(nb, 3)
    om = x[3 * N + 3 * nb:].reshape(nb, 3)
    return v, om, mu, info
