/*
 * bie.h - C ABI of the MI355X boundary-integral library for suspensions of spheres in
 * Stokes flow (Corona & Veerapaneni, "Boundary integral equation analysis for
 * suspension of spheres in Stokes flow", arXiv:1707.06551).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Viscosity 1 (Section 5).  Spheres have radius 1 (bie_build_spheres) unless built
 *   with bie_build_spheres_radii, whose comment states what changes with a radius.
 * - Grid (Eq. 4.2): p+1 Gauss-Legendre latitudes (theta ascending) x n_phi uniform
 *   longitudes phi_l = 2 pi l / n_phi.  P = (p+1) n_phi nodes per sphere, N = n_b P.
 *   Node order: g = k*P + j*n_phi + l (sphere k, latitude j, longitude l).
 *   Band limit of the vector transform: n <= p, |m| <= mmax = min(p, n_phi/2 - 1).
 * - Node fields (densities, velocities) are N x 3 row-major float64 arrays.
 * - Pointers documented "device" are HIP device pointers; the library orders all its
 *   device work on the stream given in bie_opts (NULL = the legacy default stream) and
 *   returns after that work is enqueued unless stated otherwise.  Pointers documented
 *   "host" are ordinary host memory.  The caller owns every buffer it passes; the
 *   library keeps no pointer to caller memory after a call returns.
 * - Return codes: 0 success; BIE_ENOCONV (+1) solver stopped before the tolerance (the
 *   outputs hold the last iterate); negative values are errors (no output written),
 *   with a message retrievable by bie_last_error() on the same thread.
 * - A context is not thread safe: calls on one context must not overlap.
 */
#ifndef BIE_H
#define BIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BIE_OK 0
#define BIE_ENOCONV 1
#define BIE_EINVAL (-1)
#define BIE_EOVERLAP (-2)
#define BIE_EDEVICE (-3)
#define BIE_ENOMEM (-4)

/* Operators for bie_apply_bio.  Each is applied to a node density mu on all spheres.
 * The layer potentials of sphere s at a node x of sphere t are evaluated by
 *  - t == s: spectral self evaluation (Section 4.1, Eqs. 4.6-4.7): vector transform,
 *    diagonal signature of Theorem 2 / Table 3.12, inverse transform; the double layer
 *    is its principal value D_pv = D_+ - 1/2;
 *  - t != s and |c_t - c_s| - 2 < near_gap (the separation test of Eq. 4.5): the
 *    exterior formulas 3.6-3.11 on the source's vector-harmonic coefficients;
 *  - otherwise: the smooth quadrature of Eq. 4.4 (all-pairs sum over source nodes). */
#define BIE_OP_S 1        /* sum_k S_k[mu]                                             */
#define BIE_OP_D 2        /* sum_k D_k[mu] (principal value on the own sphere)          */
#define BIE_OP_SD_BIE 3   /* 1/2 mu + sum_k (S_k + D_k)[mu]          Eqs. 5.4 / 5.17     */
#define BIE_OP_DN_BIE 4   /* 1/2 psi + sum_k (D_k + N_k)[psi]        Eq. 5.19; N_k is the
                             Stokeslet + rotlet at c_k of strength int psi and torque
                             int (y - c_k) x psi, each with the 1/(8 pi) of Eq. 2.19     */
#define BIE_OP_MOBILITY 5 /* bordered Eq. 5.17 + Eq. 5.15 with applied force/torque:
                             input [mu (3N); v (3 n_b); omega (3 n_b)], output
                             [1/2 mu + sum (S+D) mu - v_i - omega_i x (x - c_i);
                              (1/4pi) int_k mu;  (3/8pi) int_k (y - c_k) x mu]           */
#define BIE_OP_K 6        /* sum_k K_k[sigma]: traction of the single layer at the target
                             node with the target's normal (Eq. 2.22, kernel
                             -3/(4 pi) r (r.sigma)(r.n_x)/|r|^5, r = x - y); on the own
                             sphere the principal value K_pv = (K_+ + K_-)/2 of Table 3.12
                             (equal to D_pv on every mode); near pairs by the traction of
                             the exterior series (Eqs. 3.17-3.18) at the node            */
#define BIE_OP_KL_BIE 7   /* 1/2 mu + sum_k (K_k + L_k)[mu], the operator of Eq. 5.8;
                             L_k[mu] = int_k mu + (int_k (y - c_k) x mu) x (x - c_k) on the
                             nodes of sphere k only                                      */
/* Stage selectors, OR-ed into op (testing and profiling; default = all stages). */
#define BIE_STAGE_SELF 0x100 /* identity + self term (+ bordered rows for MOBILITY)      */
#define BIE_STAGE_NEAR 0x200 /* near-pair series                                         */
#define BIE_STAGE_FAR 0x400  /* far-field all-pairs quadrature (+ completion for DN)     */

#define BIE_FP64 0  /* every stage in float64                                            */
#define BIE_MIXED 1 /* transforms and far-field pair sums in float32 (accumulated in
                       float32), near series and all vectors in float64                 */

typedef struct bie_ctx bie_ctx;

typedef struct {
  int p;             /* SH order, 1 <= p <= 20                                           */
  int n_phi;         /* azimuthal nodes; 0 selects 2p; must be even and >= 2p            */
  double near_gap;   /* surface-gap threshold d* of Eq. 4.5 (spheres t != s are near when
                        |c_t - c_s| - 2 < d*); > 0: taken as given (finite);  <= 0: d* is
                        measured for this grid at the precision near_tol, see
                        bie_near_gap_for                                                 */
  int device;        /* HIP device ordinal                                               */
  void* hip_stream;  /* hipStream_t for all device work (NULL = default stream)          */
  int near_method;   /* near-pair evaluation: 0 = exterior series at the target nodes
                        (Section 4.1), 1 = pole rotation with delayed evaluation
                        (Section 4.2, Fig. 2): the source expansion is rotated so that
                        its pole points at the target, evaluated on the translated
                        target grid, projected, rotated back and summed per target
                        before one inverse transform - the band-limited projection of
                        the near field instead of its nodal values                       */
  int legendre_mfma; /* Legendre stages of the transforms (Section 2.1, Eqs. 2.9-2.14):
                        0 = per-mode FMA loops from LDS, 1 = matrix cores (v_mfma 16x16x4
                        in float32 / float64, one tile per order m and row block of 16).
                        Same results up to rounding order; 0 is faster at every measured
                        size (the stage is latency-bound).  0 or 1, BIE_EINVAL otherwise */
  double near_tol;   /* precision that selects d* when near_gap <= 0 (Eq. 4.5: eta is set
                        from the user's precision); <= 0 selects 1e-8, NaN is BIE_EINVAL.
                        Ignored when near_gap > 0                                        */
} bie_opts;

/* The separation threshold d* of Eq. 4.5 (a surface gap, d* = 2 eta for unit spheres)
 * that the grid of order p on n_phi longitudes (0 selects 2p) needs for precision tol in
 * (0, 1): the smallest gap of the grid g_k = 2^(k/8) / 64 (k = 0..104) at which the smooth
 * quadrature of Eq. 4.4 stays within tol / 10 of the exact exterior potentials (Eqs.
 * 3.6-3.11) of the single and the double layer, measured as in the paper's Section 6
 * test (Fig. 5): two random densities of degree <= p with flat spectra (coefficients
 * uniform on [-1, 1) from a counter-based SplitMix64 stream), 256 targets on a shell of
 * radius 1 + g, the error against the density's largest nodal value.  The search walks
 * the grid down from g = 128 in steps of 8 and then of 1 while the error passes.  Writes
 * +infinity (every pair near) when g = 128 already fails.  Host computation only (no
 * device use; results are cached per (p, n_phi, tol)); BIE_EINVAL for p outside [1, 20],
 * a bad n_phi or tol outside (0, 1). */
int bie_near_gap_for(int p, int n_phi, double tol, double* d_star);

/* Builds the discretisation for n_spheres unit spheres (Eq. 4.2 grid, Legendre and
 * Fourier tables, eigenvalue tables of Table 3.12, near-pair lists of Eq. 4.5) and
 * uploads it to the device.  centres: host, n_spheres x 3 row-major.  Fails with
 * BIE_EOVERLAP when two centres are closer than 2 (overlapping spheres), BIE_EINVAL
 * on bad options, BIE_ENOMEM / BIE_EDEVICE on allocation or device errors.  Blocks
 * until the upload completes.  *out is owned by the caller and released by bie_free.
 * Device memory held: besides the tables and per-node fields, the far field's
 * partial-sum buffer of min(64, n_spheres / 2) source splits x 3N doubles (about
 * 1 GB at 640,000 nodes), from which each far-field launch uses the split count that
 * fills the device's last round of work-groups; the solver's Krylov basis is
 * allocated on the first solve. */
int bie_build_spheres(const double* centres, int64_t n_spheres, const bie_opts* opts, bie_ctx** out);

/* As bie_build_spheres for spheres of radii a_k (host, n_spheres, each in [1/16, 16];
 * NULL = all 1): polydisperse suspensions (Section 6, Figs. 4 (a), 8 (c)-(d)).  Node
 * x = c_k + a_k xhat with weight a_k^2 w (Eq. 4.4 scaled); the single layer on a sphere
 * of radius a scales with a (Table 3.12 eigenvalues times a, exterior series of
 * Eqs. 3.6-3.8 at (x - c)/a times a), the double layer and the traction K not at all.
 * Near pairs: |c_t - c_s| - a_t - a_s < near_gap * a_s (Eq. 4.5 with the gap measured in
 * the source's radius; directed).  Overlap: |c_t - c_s| < a_t + a_s -> BIE_EOVERLAP.  When
 * some radius differs from 1 the context supports bie_apply_bio with BIE_OP_S, _D,
 * _SD_BIE, _DN_BIE, _MOBILITY, _K and _KL_BIE, bie_solve with the second-kind forms
 * (porous media, Problem 1, with BIE_OP_SD_BIE), bie_solve_resistance (Problem 5: the
 * moments carry a^2 and a^3; an isolated sphere gives F = 6 pi a v, T = 8 pi a^3 omega),
 * bie_solve_mobility and bie_solve_mobility_traction (rho_k = F_k/(4 pi a^2) +
 * 3/(8 pi a^4) T_k x (x - c_k); v = F/(6 pi a), omega = T/(8 pi a^3) for an isolated
 * sphere), with BIE_PC_NONE or BIE_PC_M0 (per-sphere isolated inverses), the resistance
 * form also with BIE_PC_M0 | BIE_PC_RIGID (the coarse operator of spheres of radius a,
 * see BIE_PC_RIGID), bie_eval_field (near test |x - c_k| - a_k < near_gap a_k), the
 * transforms, nodes and near pairs, near_method 1 (the pole rotation in units of the
 * source radius), and bie_apply_laplace / bie_solve_magnetic (S^L of a sphere of
 * radius a is a times the unit layer at (x - c)/a: gradient and K^L scale-free; force
 * and torque carry a^2 and a^3); the learned correction returns BIE_EINVAL. */
int bie_build_spheres_radii(const double* centres, const double* radii, int64_t n_spheres, const bie_opts* opts,
                            bie_ctx** out);

void bie_free(bie_ctx* ctx);

/* Number of nodes N; number of spheres; P per sphere; mmax.  Host outputs, each
 * optional. */
int bie_sizes(const bie_ctx* ctx, int64_t* n_nodes, int64_t* n_spheres, int64_t* nodes_per_sphere, int64_t* mmax);

/* Number of nodes N = n_b (p + 1) n_phi of the grid of Eq. 4.2 (host output). */
int bie_num_nodes(const bie_ctx* ctx, int64_t* n_nodes);

/* The context's separation threshold d* of Eq. 4.5 (+infinity: every pair near) and the
 * precision it was measured for (0 when near_gap was given).  Host outputs, each
 * optional. */
int bie_near_gap(const bie_ctx* ctx, double* d_star, double* near_tol);

/* Node coordinates (N x 3) and quadrature weights (N, Eq. 4.4) in ABI node order.
 * Host outputs; either pointer may be NULL. */
int bie_get_nodes(const bie_ctx* ctx, double* xyz, double* weights);

/* Number of directed near pairs (t, s), and optionally the pairs themselves as
 * 2 x count int64 (row 0 targets, row 1 sources) into a host buffer of that size. */
int bie_near_pairs(const bie_ctx* ctx, int64_t* count, int64_t* pairs);

/* One application of an operator (BIE_OP_*, optionally OR-ed with BIE_STAGE_* bits)
 * in the given precision.  mu, u: device float64, length 3N (3N + 6 n_b for
 * BIE_OP_MOBILITY); u is overwritten.  mu and u must not alias. */
int bie_apply_bio(bie_ctx* ctx, int op, int precision, const double* mu, double* u);

/* Forward vector transform (Section 2.1: the quadrature projection onto V, W, X, equal
 * to Eqs. 2.7-2.14 on band-limited fields) of a node field mu (device, 3N float64) into
 * coef (device float64): per sphere k, family f in (V, W, X), modes ordered by m
 * (0..mmax) then n (m..p) - the ordering of Fig. 1 - as (re, im) pairs:
 * coef[((k*3 + f) * ncoef + i) * 2 + {0,1}], ncoef = sum_{m=0}^{mmax} (p + 1 - m).
 * Entries of W, X at n = 0 are zero.  Negative m follow from c_{n,-m} = conj(c_{n,m}). */
int bie_vsh_forward(bie_ctx* ctx, int precision, const double* mu, double* coef);
/* Inverse transform (Eqs. 2.15-2.17 / synthesis) of coef (layout above) into u (3N). */
int bie_vsh_inverse(bie_ctx* ctx, int precision, const double* coef, double* u);

/* Solver options.  The paper names no iterative method; the library uses restarted,
 * right-preconditioned flexible GMRES with classical Gram-Schmidt twice (CGS2) in
 * float64.  precision = BIE_MIXED runs iterative refinement: float64 residuals
 * b - A x with a float64 matvec, inner GMRES on the correction with BIE_MIXED matvecs
 * to relative tolerance inner_tol. */
#define BIE_PC_NONE 0 /* no preconditioner                                             */
#define BIE_PC_M0 1   /* exact inverse of every sphere's isolated self operator        */
#define BIE_PC_MLP 2  /* M0 plus the learned close-pair coarse correction              */
/* Flag, OR-ed with BIE_PC_M0 or BIE_PC_MLP: global rigid-mode coarse correction of the
 * resistance form (no counterpart in the paper).  With z0 = M0 r, z = z0 + P (y - R z0)
 * with M_RPY S y = R r (with BIE_PC_MLP the learned correction is then added to z, acting
 * on the 19 non-rigid low modes only - the rigid ones are this correction's - so weights
 * for this combination are trained on that base): R projects each sphere's field onto
 * its six rigid modes (W_1, X_1 of Definition 2.2; a = int f / 4 pi, b = 3 int x x f /
 * 8 pi), P (a, b) = a + b x x, S = diag(4 pi, 8 pi / 3) turns them into the force and
 * torque the completion flow of Eqs. 5.18-5.19 carries, and M_RPY is the Rotne-Prager-
 * Yamakawa grand mobility of the unit spheres (translation (1/8 pi d)[(1 + 2/(3d^2)) I +
 * (1 - 2/d^2) e e], coupling -[r]_x / (8 pi d^3), rotation -(I - 3 e e)/(16 pi d^3),
 * self blocks I/6pi and I/8pi).  Spheres of radius a (bie_build_spheres_radii): R f =
 * (int f / (4 pi a^2), 3 int (x - c) x f / (8 pi a^4)), P (a, b) = a + b x (x - c),
 * S = diag(4 pi a^2, 8 pi a^4 / 3), self blocks I/(6 pi a), I/(8 pi a^3), and the
 * translation block (1/8 pi d)[(1 + (a_i^2 + a_k^2)/(3d^2)) I + (1 - (a_i^2 + a_k^2)/d^2)
 * e e].  The coarse system is solved on the device by Jacobi-
 * preconditioned conjugate gradients (float64, relative residual 1e-7, at most 400
 * iterations) with a matrix-free all-pairs product over the centres.  n_b <= 65536
 * (BIE_EINVAL beyond).  Other forms ignore the flag (the mobility form carries its rigid motions as
 * unknowns with their own rows). */
#define BIE_PC_RIGID 0x10
/* Flag, OR-ed with BIE_PC_MLP (optionally with BIE_PC_RIGID): the learned correction
 * acts on the residual that the base preconditioner leaves under the local part of the
 * operator instead of on r itself:
 *   z0 = B r,  z = z0 + P zeta(R (r - A_loc z0)),
 * B = M0 (with the rigid-mode correction when BIE_PC_RIGID is set), A_loc the self term
 * and the near-pair series of the operator (no far field), P, R, zeta as for
 * BIE_PC_MLP.  Costs one transform and one near-series pass per application; needs
 * weights trained for this composition (bie_precond_sample with the same flag).  With
 * BIE_PC_RIGID the learned part acts on the non-rigid low modes, as with the additive
 * composition.  BIE_EINVAL without BIE_PC_MLP. */
#define BIE_PC_LOCAL 0x20

typedef struct {
  double tol;        /* stop when ||b - A x||_2 <= tol ||b||_2 (true residual)         */
  int restart;       /* Krylov dimension per cycle (<= 0 selects 100, > 500 BIE_EINVAL) */
  int max_iter;      /* total inner iterations (<= 0 selects 1000)                      */
  int precision;     /* BIE_FP64 or BIE_MIXED                                           */
  int precond;       /* BIE_PC_NONE, _M0 or _MLP, optionally | BIE_PC_RIGID (resistance
                        form), BIE_PC_MLP optionally | BIE_PC_LOCAL                      */
  double inner_tol;  /* BIE_MIXED inner tolerance (<= 0 selects 1e-4)                   */
  const double* x0;  /* initial guess (device float64, the solve's own unknown vector:
                        psi (3N) for resistance, [mu; v; omega] (3N + 6 n_b) for the
                        bordered mobility form, mu (3N) for the traction form, x of
                        bie_solve), or NULL for x0 = 0.  The first true residual is
                        b - A x0, so passing a converged solution back returns after
                        that one float64 matvec with iters = 0 (a restart = resume).
                        Read only; may alias no output                                   */
  double* res_hist;  /* optional host buffer of res_hist_cap doubles (NULL: none): the
                        GMRES residual estimate ||r_k|| / ||b|| after every iteration
                        k (all cycles, refinement steps and a fallback, in order);
                        bie_solve_info.res_hist_len reports how many were written        */
  int res_hist_cap;
} bie_solve_opts;

/* Indices of bie_solve_info.t_stage_s: device time of each step of the hot path summed
 * over one solve, from HIP events recorded on the context's stream around every launch
 * of that step (only while a solve runs with info != NULL). */
#define BIE_T_TRANSFORM 0  /* forward transform, self term, inverse (Section 2.1, Theorem 2; one fused launch) */
#define BIE_T_NEAR      1  /* near-pair series (Section 4.1, Eqs. 3.6-3.11)                                    */
#define BIE_T_FAR       2  /* far-field smooth quadrature (Eq. 4.4) with the completion flow (Eqs. 5.18-5.19) */
#define BIE_T_PRECOND   3  /* preconditioner (M0 and the coarse corrections)                                  */
#define BIE_T_KRYLOV    4  /* GMRES: orthogonalisation, updates, residual norms                                */
#define BIE_T_OTHER     5  /* right-hand side, read-out and the local terms of the traction form              */

typedef struct {
  int iters;            /* GMRES iterations (all cycles, all refinement steps)          */
  int outer_steps;      /* refinement steps (1 for BIE_FP64)                            */
  int matvecs_fp64;
  int matvecs_mixed;
  int fallback_used;    /* 1 if the preconditioned solve stalled and was restarted plain */
  double rel_residual;  /* final true relative residual                                */
  double seconds;       /* wall time of the solve (device synchronised)                 */
  double t_stage_s[8];  /* device seconds per step, indexed by BIE_T_*; 6, 7 are 0      */
  long long pairs_evaluated; /* far-field node pairs (target node, source node on a
                                well-separated sphere) summed over every matvec        */
  long long near_evals;      /* near-series evaluations (target node, near source
                                sphere) summed over every matvec                       */
  int res_hist_len;     /* entries written to bie_solve_opts.res_hist                   */
} bie_solve_info;

/* Resistance problem (Problem 5, Eqs. 5.18-5.19): given rigid velocities v and angular
 * velocities omega (host, n_b x 3), solve (1/2 I + sum (D_k + N_k)) psi = v_i +
 * omega_i x (x - c_i) and return F_k = int psi, T_k = int (y - c_k) x psi (host,
 * n_b x 3): the force and torque each particle exerts on the fluid (6 pi v and 8 pi
 * omega for an isolated sphere).  psi: optional device output (3N), else NULL.
 * Synchronises the stream.  info may be NULL. */
int bie_solve_resistance(bie_ctx* ctx, const double* v, const double* omega, const bie_solve_opts* opts,
                         double* F, double* T, double* psi, bie_solve_info* info);

/* Mobility problem in the bordered second-kind form of Problem 4 (Eqs. 5.14-5.17) with
 * the force/torque conditions of Eq. 5.15 set to the applied F_k, T_k (host, n_b x 3):
 * unknowns mu, v_k, omega_k.  slip: optional device u_s (3N) of Eq. 5.14, else NULL.
 * Returns v, omega (host, n_b x 3); mu: optional device output (3N).  Synchronises the
 * stream.  info may be NULL. */
int bie_solve_mobility(bie_ctx* ctx, const double* F, const double* T, const double* slip,
                       const bie_solve_opts* opts, double* v, double* omega, double* mu, bie_solve_info* info);

/* Mobility problem in the paper's own formulation (Problem 2, Eqs. 5.7-5.8): with the
 * force density rho_k = F_k / (4 pi) + 3/(8 pi) T_k x (x - c_k) (int rho = F_k,
 * int (x - c_k) x rho = T_k; F, T host n_b x 3, the force and torque each particle
 * exerts on the fluid), solve (1/2 I + sum (K_k + L_k)) mu = -(1/2 I + sum K_k) rho, then
 * u = sum S_k[mu + rho] on the surfaces gives v_k = (1/4 pi) int_k u and
 * omega_k = 3/(8 pi) int_k (x - c_k) x u (host outputs, n_b x 3).  opts->precond:
 * BIE_PC_NONE or BIE_PC_M0 (isolated-sphere inverse of 1/2 + K_pv + L); precision as in
 * bie_solve (the right-hand side and the final single layer are float64).  mu: optional
 * device output (3N), the solved density without rho.  near_method must be 0.
 * Synchronises the stream.  info may be NULL. */
int bie_solve_mobility_traction(bie_ctx* ctx, const double* F, const double* T, const bie_solve_opts* opts,
                                double* v, double* omega, double* mu, bie_solve_info* info);

/* Generic solve of op (BIE_OP_DN_BIE, BIE_OP_MOBILITY, BIE_OP_SD_BIE or BIE_OP_KL_BIE) with a caller
 * right-hand side: b, x device float64 of length 3N (3N + 6 n_b for mobility).  With
 * BIE_OP_SD_BIE and b = -u_inf at the nodes this is the porous-media problem (Problem 1,
 * Eq. 5.4: spheres held fixed in an imposed flow u_inf); the flow is then
 * u_inf + bie_eval_field(BIE_OP_SD_BIE, x) off the surfaces (Eq. 5.3).  Same solver and
 * return codes as bie_solve_resistance.  Synchronises the stream. */
int bie_solve(bie_ctx* ctx, int op, const double* b, double* x, const bie_solve_opts* opts, bie_solve_info* info);

/* z = M r for the preconditioner precond (BIE_PC_*) of op (BIE_OP_DN_BIE,
 * BIE_OP_MOBILITY, BIE_OP_SD_BIE or BIE_OP_KL_BIE; for BIE_OP_SD_BIE, M0 inverts
 * 1/2 + S + D_pv of each isolated sphere and the corrections do not apply; for
 * BIE_OP_KL_BIE only BIE_PC_NONE and BIE_PC_M0 exist), in the given precision.
 * r, z: device float64, length 3N (3N + 6 n_b for mobility), must not alias. */
int bie_apply_precond(bie_ctx* ctx, int op, int precision, int precond, const double* r, double* z);

/* Velocity at fluid points (the representations of Eqs. 5.3, 5.13 and 5.18 evaluated off
 * the surfaces): the layer potential of op (BIE_OP_S, BIE_OP_D, BIE_OP_SD_BIE = S + D, or
 * BIE_OP_DN_BIE = D plus the completion flow of Eqs. 5.18-5.19; the identity term of
 * the second-kind forms is a surface term and is not added) of the node density mu
 * (device float64, 3N) at n_targets points (device float64, n_targets x 3, row-major)
 * -> u (device float64, n_targets x 3).  Per sphere k: |x - c_k| - a_k < near_gap a_k
 * (a_k = 1 for unit spheres) takes the exterior series of Eqs. 3.6-3.11 (Section 3),
 * otherwise the smooth quadrature of Eq. 4.4.  Float64.  A point inside or on a sphere gets NaN and the call returns BIE_EINVAL
 * after writing the others.  n_targets = 0 is a no-op.  Synchronises the stream. */
int bie_eval_field(bie_ctx* ctx, int op, const double* mu, int64_t n_targets, const double* targets, double* u);

/* ---- Laplace single layer and the magnetostatic problem (Problem 3) ---------------
 * S^L[q](x) = int q / (4 pi |x - y|) over all spheres, evaluated as the Stokes operators
 * are: the own sphere spectrally (Theorem 1: S^L[Y_n^m] = Y_n^m / (2n+1), normal
 * derivative K^L with principal value -1 / (2(2n+1)), both on the band-limited
 * projection), near spheres by Eq. 3.3 and its gradient, others by the smooth
 * quadrature of Eq. 4.4.  Float64.
 * kind 0: out (device, N) = (1/2 I + eta K^L)[q], the operator of Eq. 5.13;
 * kind 1: out (device, N x 3) = gradient of S^L[q] at every node, exterior side (eta
 *         unused).  q: device float64, N scalar node values. */
int bie_apply_laplace(bie_ctx* ctx, int kind, double eta, const double* q, double* out);

/* Problem 3 (Eqs. 5.9-5.13): paramagnetic spheres in the imposed field H0 (host, 3),
 * eta = (mu - mu0) / (mu + mu0) in (-1, 1).  Solves (1/2 I + eta K^L)[q] = eta H0 . n
 * with the library's GMRES (float64; opts->precision is ignored, BIE_PC_M0 selects the
 * isolated-sphere inverse, BIE_PC_RIGID / BIE_PC_MLP are ignored), then evaluates
 * H = H0 - grad S^L[q] on the fluid side of every node and the Maxwell traction
 * t = (H . n) H - |H|^2 n / 2 (mu0 = 1), and returns each sphere's force F = int t and
 * torque T = int (x - c) x t (host, n_b x 3).  The flow couples to the field only
 * through these loads (Section 5): bie_solve_mobility(F, T) gives the particle
 * velocities.  q: optional device output (N), else NULL.  Synchronises the stream. */
int bie_solve_magnetic(bie_ctx* ctx, const double* H0, double eta, const bie_solve_opts* opts, double* q, double* F,
                       double* T, bie_solve_info* info);

/* ---- learned close-pair coarse correction (no counterpart in the paper) -------------
 * Coarse space per sphere: the vector spherical harmonics of degree <= 2 (Definition
 * 2.2) in a Cartesian parametrisation of 25 coefficients (s; a; b; c; tV; tW; tX):
 *   s x,  a - 3 (a.x) x,  b,  c x x,  2 T x - 5 (x.T x) x,  2 T x,  2 x x (T x),
 * x the unit normal, T = sum_k t_k E_k over the Frobenius-orthonormal symmetric
 * traceless basis (xy, yz, xz, xx - yy, 2zz - xx - yy).  BIE_PC_MLP applies
 *   z = M0 r + P zeta,  zeta_i = sum_{j close to i} rot_ij^T [K_off rot_ij rho_j + K_self rot_ij rho_i],
 * rho = R r (weighted projection with the Eq. 4.4 weights), P = synthesis, rot_ij the
 * rotation into the frame whose z axis points from c_i to c_j, and K(theta) 25 x 25
 * maps commuting with rotations about that axis (139 parameters each) produced per
 * directed close pair by an MLP (8 -> 64 -> 64 -> 278, tanh, float32) of the pair's
 * features: gap g, log(g + 0.01), 0.1/(g + 0.1), close counts of i and j / 8, smallest
 * other gap of i and of j (1 if none), sum_{k close to i} 0.1/(g_ik + 0.1).  Close pairs
 * are those with surface gap |c_i - c_j| - 2 < 1, the gap the network was trained
 * with; they do not depend on the context's d*.
 * The correction acts on the density part of the resistance and mobility forms (the
 * network is trained per form: weights/precond_dn*.npz, weights/precond_mob.npz); for
 * BIE_OP_SD_BIE BIE_PC_MLP is M0. */

/* rho = R f: f device 3N float64 -> rho device n_b x 25 float64. */
int bie_lowmodes(bie_ctx* ctx, const double* f, double* rho);
/* f = P rho (overwrites f). */
int bie_lowmodes_synth(bie_ctx* ctx, const double* rho, double* f);

/* Directed close pairs (surface gap < 1) in CSR order (grouped by target sphere i), with features and
 * frames.  Host outputs, each optional: pair_i, pair_j (count), feats (count x 8),
 * frames (count x 34: Q row-major then D2 row-major, D2_kl = tr(E_k Q E_l Q^T)). */
int bie_pair_geometry(const bie_ctx* ctx, int64_t* count, int32_t* pair_i, int32_t* pair_j, float* feats,
                      double* frames);

/* One training sample of the learned correction: for a right-hand side b and the
 * solution x = A^-1 b of op (BIE_OP_DN_BIE or BIE_OP_MOBILITY; b, x device float64 of
 * the solve's length), writes target = R x - R B b, the part of the low-mode response
 * that the base preconditioner B misses, and the network's input xi = R b, or
 * R (b - A_loc B b) when precond has BIE_PC_LOCAL (the composition the weights are
 * trained for).  precond: BIE_PC_M0 (| BIE_PC_RIGID) (| BIE_PC_MLP, ignored)
 * (| BIE_PC_LOCAL); with BIE_PC_RIGID (resistance form) the rigid components (b, c) of
 * xi and target are zero.  xi, target: device float64, n_b x 25.  Unit spheres only.  Float64.
 * Synchronises the stream. */
int bie_precond_sample(bie_ctx* ctx, int op, int precond, const double* b, const double* x, double* xi,
                       double* target);

/* Number of MLP weights (flattened W1 8x64, b1, W2 64x64, b2, W3 64x278, b3). */
int64_t bie_mlp_n_weights(void);

/* Loads MLP weights (host, float32) into the context and evaluates theta for every
 * directed close pair on the device; enables BIE_PC_MLP.  Rejects non-finite weights. */
int bie_precond_load(bie_ctx* ctx, const float* weights, int64_t n_weights);

/* Training set for the MLP: n_configs configurations concatenated; spheres and pairs
 * are numbered globally, pairs grouped by target sphere (sph_ptr CSR) and by
 * configuration (cfg_sph, cfg_pair offsets, n_configs + 1 each).  For each sphere and
 * each of n_rhs samples: xi (n_spheres x n_rhs x 25) = R b of a right-hand side b = P xi,
 * target (same layout) = R x - R M0 b for the solution of A x = b.  All host arrays. */
typedef struct {
  int64_t n_pairs, n_spheres, n_configs;
  int32_t n_rhs;
  const float* feats;      /* n_pairs x 8 */
  const float* frames;     /* n_pairs x 34 */
  const int32_t* pair_i;   /* n_pairs */
  const int32_t* pair_j;   /* n_pairs */
  const int32_t* sph_ptr;  /* n_spheres + 1 */
  const int32_t* cfg_sph;  /* n_configs + 1 */
  const int32_t* cfg_pair; /* n_configs + 1 */
  const float* xi;
  const float* target;
} bie_mlp_data;

/* Loss L = sum |target - zeta(xi)|^2 / sum |target|^2 and its gradient with respect to
 * the weights (host float32, length bie_mlp_n_weights()) on the device of the calling
 * thread, one forward and one backward pass over the whole set. */
int bie_mlp_eval(const bie_mlp_data* data, const float* weights, double* loss, float* grad);

/* Adam training (beta 0.9 / 0.999) for `epochs` passes over the set in batches of
 * cfg_per_batch configurations; weights in: initial, out: trained; loss_hist (epochs,
 * optional) receives the summed batch losses per epoch. */
int bie_mlp_train(const bie_mlp_data* data, float* weights, int epochs, int cfg_per_batch, double lr,
                  double* loss_hist);

/* ---- Operator application without device allocation ------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, operators, stages,
 * precisions and results as bie_apply_bio (up to the rounding order of the far-field
 * partial sums), for op BIE_OP_S, _D, _SD_BIE, _DN_BIE or _MOBILITY (optionally with
 * BIE_STAGE_* bits) on a context built with near_method 0.  The call's work buffers (far-
 * field source strengths, transform coefficients, near-series tables, sphere moments and
 * far-field partial sums) live in one file-scope device array of
 * BIE_NOALLOC_SCRATCH_BYTES (96 MiB) instead of the context's buffers: every device the
 * library runs this on holds its own copy until the process ends, and the call performs
 * no device allocation or free.  The array holds the work of about 900,000 nodes at
 * p = 12 (e.g. 2048 spheres, 638,976 nodes); a context whose work buffers do not fit
 * returns BIE_EINVAL before any device work.  All calls on one device share that
 * device's array, which keeps the last call's contents: calls that overlap in time on
 * one device (several host threads, or streams not ordered with each other) race and
 * give wrong results; order them.  Errors as bie_apply_bio. */
#define BIE_NOALLOC_SCRATCH_BYTES 100663296ULL
int bie_apply_bio_noalloc(bie_ctx* ctx, int op, int precision, const double* mu, double* u);

/* Thread-local message of the last error on this thread ("" if none). */
const char* bie_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIE_H */
