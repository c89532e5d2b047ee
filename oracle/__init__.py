"""Plain FP64 CPU oracle for the sphere-suspension Stokes boundary integral method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports, links or calls it,
and this package imports nothing from the product.

Everything here is written for a reader who has the paper (Corona & Veerapaneni,
"Boundary integral equation analysis for suspension of spheres in Stokes flow",
arXiv:1707.06551) beside them: each function names the section / equation it follows.
The code is deliberately slow and direct: dense quadrature projections instead of fast
transforms, direct pair sums instead of tiles, textbook GMRES.

Readings of the paper taken here (each is pinned by a test under ``tests/``):

* Double-layer sign (Eqs. 2.20-2.21 vs Table 3.12 and Eq. A.7): the kernel used is
  D_ij(x, y) = +3/(4 pi) r_i r_j (r . n_y) / |r|^5 with r = x - y, which gives
  D[c] = -c inside a sphere and 0 outside, the convention under which the spectra of
  Theorem 2 and the jump [[D]] = mu hold.
* Azimuthal grid (Eq. 4.2 vs the unknown count of Section 6): n_phi is a parameter;
  the default is 2p, and the band limit is n <= p, |m| <= min(n, n_phi/2 - 1).
* Forward vector transform (Eqs. 2.7-2.8): implemented as the exact quadrature
  projection onto V, W, X (their L2 norms are (n+1)(2n+1), n(2n+1), n(n+1)), which the
  fast transform must reproduce on band-limited fields.
* Degree zero: W_0 = X_0 = 0, so only V_0 carries a coefficient at n = 0.
* Identity term of the second-kind equations: 1/2 I acts on the grid values, the layer
  operators act on the band-limited projection (Section 4.1, singular integrands).
* Completion flow N_k (Eq. 5.18-5.19): Stokeslet of strength int psi plus rotlet of
  torque int (y - c_k) x psi, both with the 1/(8 pi) normalisation of Eq. 2.19.

Parity status per function is stated in each module header.
"""
