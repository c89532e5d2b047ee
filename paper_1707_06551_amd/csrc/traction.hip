// Traction of the Stokes single layer, K (Eq. 2.22, Section 3.3), on the near pairs, and
// the per-sphere rank-six operator L of Eq. 5.8 (plus the force density rho of Eq. 5.7,
// which has the same form).
//
// Near pairs.  For a directed near pair (source s, target t) and a node x of sphere t
// with outward unit normal n (the target's normal, which has tangential components in
// the source frame: the general case of Eq. 3.18), the traction
// (grad u + grad u^T - p I) n of the exterior flow u = S_s[mu] (Eqs. 3.6-3.8) is
// evaluated at the node.  The paper maps the terms of Eq. 3.18 to vector harmonics with
// precomputed matrices (Fig. 1); here the flow is written through decaying harmonic
// potentials, Phi_nm = r^{-n-1} Y_n^m with d = x - c_s, r = |d|:
//   u = grad Psi_A + r^2 grad Psi_B + d Psi_C + d x grad Psi_X,   p = Psi_P,
//   Psi_A = sum (s_V mu^V + s_WV mu^W) Phi,  Psi_B = -(n-2)/(2(2n-1)) mu^W Phi,
//   Psi_C = (n+1)/(2n-1) mu^W Phi,  Psi_X = mu^X/(2n+1) Phi,  Psi_P = n mu^W Phi,
// (s_V = n/((2n+1)(2n+3)), s_WV = n/(2(2n+1)) of Eqs. 3.6-3.7; grad Phi = r^{-n-2} V,
// d x grad Phi = r^{-n-1} X, r^{-n} W = r^2 grad Phi + (2n+1) d Phi).  The antisymmetric
// parts cancel in G + G^T and the traction becomes
//   t = 2 H_{A + r^2 B} n + d x (H_X n) + H_X (n x d) + (d.n) g + d (n.g) + s n,
// H the Hessians (at the fixed target, r^2 is a constant), g = grad Psi_G with
// Psi_G = 3/(2n-1) mu^W Phi, s = Psi_S with Psi_S = (2(n+1)/(2n-1) - n) mu^W Phi.  A
// Hessian times a vector v is the gradient of v . grad Psi, and the derivatives of a
// potential are potentials of one degree more, by the ladder relations of the
// irregular solid harmonics (orthonormal Y without the Condon-Shortley phase, as in
// Eq. 2.1; kappa = sqrt((2n+1)/(2n+3))):
//   d_z Phi_nm           = -kappa sqrt((n+1)^2 - m^2)     Phi_{n+1,m},
//   (d_x + i d_y) Phi_nm = -kappa sqrt((n+m+1)(n+m+2))    Phi_{n+1,m+1},
//   (d_x - i d_y) Phi_nm =  kappa sqrt((n-m+1)(n-m+2))    Phi_{n+1,m-1}   (m >= 1).
// Each work-group builds, per near source, the x, y, z derivative coefficients of
// Psi_A, Psi_B, Psi_X (degree <= p+1, stored like a real field: m >= 0) and those of
// Psi_G, Psi_S in LDS; each thread then sums, for its target node, the five series
// (four gradients sum c r^{-n-2} V_n^m with coefficients combined on the fly with the
// node's n, n x d and r^2, and one value sum c r^{-n-1} Y_n^m) over one shared Legendre
// recursion.  Float64 throughout (the near field is the accuracy-critical part).
#include <cmath>
#include <vector>

#include "bie_internal.h"

namespace bie {

std::vector<double> recurrence_table(int p, int mmax);

namespace {

constexpr int TR_NARR = 11;   // A_x A_y A_z, B_x B_y B_z, X_x X_y X_z, G, S

struct TracParams {
  const double* coef;      // nb x 3 x ncoef x 2: V, W, X coefficients (degree <= p)
  const double* centres4;  // nb x 4
  const int* near_ptr;
  const int* near_idx;
  const double* otab;      // P x 4 unit offsets (= outward normals) of the nodes
  const double* rec2;      // ncoef2 x 6 recurrence constants, degree <= p+1, m <= mm2
  const double* radius;    // nb radii, or null for unit spheres
  double* u;
  int p, mmax, P, ncoef, p2, mm2, ncoef2;
};

__device__ __forceinline__ int slot_of(int p, int m, int n) { return m * (p + 1) - (m * (m - 1)) / 2 + (n - m); }

// (re, im) of potential `fam` (0: Psi_A, 1: Psi_B, 2: Psi_X) at (n, m) of source s;
// zero outside n in [0, p], 0 <= m <= min(n, mmax).
__device__ __forceinline__ void pot_coef(const TracParams& a, int s, int fam, int n, int m, double& re, double& im) {
  re = im = 0.0;
  if (n < 0 || n > a.p || m < 0 || m > n || m > a.mmax) return;
  const double* cb = a.coef + ((size_t)s * 3 * a.ncoef) * 2;
  const int i = slot_of(a.p, m, n);
  const double dn = n;
  if (fam == 0) {
    const double sv = dn / ((2 * dn + 1) * (2 * dn + 3)), swv = dn / (2 * (2 * dn + 1));
    const double* cv = cb + 2 * i;
    const double* cw = cb + 2 * (a.ncoef + i);
    re = sv * cv[0] + swv * cw[0];
    im = sv * cv[1] + swv * cw[1];
  } else if (n >= 1) {
    const double* c = cb + 2 * ((fam == 1 ? 1 : 2) * a.ncoef + i);
    const double f = (fam == 1) ? -(dn - 2) / (2 * (2 * dn - 1)) : 1.0 / (2 * dn + 1);
    re = f * c[0];
    im = f * c[1];
  }
}

// Coefficients of source s in the degree-(p+1) slot layout: derivative potentials and
// the two W-family potentials.  Arrays k * ncoef2 * 2 in `cs`.
__device__ void build_slots(const TracParams& a, int s, double* cs) {
  for (int i = threadIdx.x; i < a.ncoef2; i += blockDim.x) {
    int m = 0, off = 0;
    while (m < a.mm2 && i >= off + (a.p2 + 1 - m)) {
      off += a.p2 + 1 - m;
      ++m;
    }
    const int n2 = m + (i - off);
    const int n = n2 - 1;  // degree of the potential being differentiated
    double v[TR_NARR][2];
    for (int k = 0; k < TR_NARR; ++k) v[k][0] = v[k][1] = 0.0;
    if (n >= 0) {
      const double kap = sqrt((2.0 * n + 1.0) / (2.0 * n + 3.0));
      const double fz = -kap * sqrt((n + 1.0) * (n + 1.0) - (double)m * m);
      const double fb = kap * sqrt((double)(n - m) * (n - m + 1.0));
      const double fa = -kap * sqrt((n + (double)m) * (n + m + 1.0));
      for (int fam = 0; fam < 3; ++fam) {
        double zr, zi, br, bi, ar, ai;
        pot_coef(a, s, fam, n, m, zr, zi);
        pot_coef(a, s, fam, n, m + 1, br, bi);
        br *= fb;
        bi *= fb;
        if (m >= 1) {
          pot_coef(a, s, fam, n, m - 1, ar, ai);
          ar *= fa;
          ai *= fa;
        } else {
          ar = br;   // (d_x + i d_y) coefficient at m = 0 of a real potential: conj of the other
          ai = -bi;
        }
        v[3 * fam + 0][0] = 0.5 * (ar + br);
        v[3 * fam + 0][1] = 0.5 * (ai + bi);
        v[3 * fam + 1][0] = 0.5 * (ai - bi);
        v[3 * fam + 1][1] = -0.5 * (ar - br);
        v[3 * fam + 2][0] = fz * zr;
        v[3 * fam + 2][1] = fz * zi;
      }
    }
    if (n2 >= 1 && n2 <= a.p && m <= n2 && m <= a.mmax) {
      const double* cw = a.coef + (((size_t)s * 3 + 1) * a.ncoef + slot_of(a.p, m, n2)) * 2;
      const double d2 = n2;
      const double fg = 3.0 / (2 * d2 - 1), fsc = 2 * (d2 + 1) / (2 * d2 - 1) - d2;
      v[9][0] = fg * cw[0];
      v[9][1] = fg * cw[1];
      v[10][0] = fsc * cw[0];
      v[10][1] = fsc * cw[1];
    }
    for (int k = 0; k < TR_NARR; ++k) {
      cs[(k * a.ncoef2 + i) * 2 + 0] = v[k][0];
      cs[(k * a.ncoef2 + i) * 2 + 1] = v[k][1];
    }
  }
}

// Traction at one target point d (relative to the source centre) with unit normal nv.
__device__ void traction_point(const TracParams& a, const double* cs, const double* rec, const double d[3],
                               const double nv[3], double t[3]) {
  const int nc2 = a.ncoef2;
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double r = sqrt(r2);
  const double ir = 1.0 / r, ir2 = ir * ir;
  const double ct = d[2] * ir;
  const double rho = sqrt(d[0] * d[0] + d[1] * d[1]);
  const double st = rho * ir;
  double cph = 1.0, sph = 0.0;
  if (rho > 0.0) {
    cph = d[0] / rho;
    sph = d[1] / rho;
  }
  const double w[3] = {nv[1] * d[2] - nv[2] * d[1], nv[2] * d[0] - nv[0] * d[2], nv[0] * d[1] - nv[1] * d[0]};
  // spherical components (r, theta, phi) of the four gradient series, and the value series
  double gs[4][3] = {};
  double sval = 0.0;
  double cm = 1.0, sm_ = 0.0;
  double pmm = 0.28209479177387814, qmm = 0.0, irm = 1.0;
  const auto C = [cs, nc2](int k, int i) { return cs + 2 * (k * nc2 + i); };
  for (int m = 0; m <= a.mm2; ++m) {
    const int off = m * (a.p2 + 1) - (m * (m - 1)) / 2;
    if (m > 0) {
      const double fm = rec[6 * off + 5];
      qmm = fm * pmm;
      pmm = fm * st * pmm;
      const double c2 = cm * cph - sm_ * sph;
      sm_ = sm_ * cph + cm * sph;
      cm = c2;
      irm *= ir;
    }
    double acc[4][6] = {};
    double vr = 0.0, vi = 0.0;
    double rp = irm;  // r^{-n}
    // one (n, m) term given Pbar (Pb), dPbar/dtheta (D) and m Pbar / sin (mQ)
    const auto term = [&](int n, int i, double Pb, double D, double mQ) {
      const double f = rp * ir2, fs = rp * ir;
      double e[4][2];
      const double* A0 = C(0, i);
      const double* A1 = C(1, i);
      const double* A2 = C(2, i);
      const double* B0 = C(3, i);
      const double* B1 = C(4, i);
      const double* B2 = C(5, i);
      const double* X0 = C(6, i);
      const double* X1 = C(7, i);
      const double* X2 = C(8, i);
      for (int q = 0; q < 2; ++q) {
        e[0][q] = nv[0] * fma(r2, B0[q], A0[q]) + nv[1] * fma(r2, B1[q], A1[q]) + nv[2] * fma(r2, B2[q], A2[q]);
        e[1][q] = nv[0] * X0[q] + nv[1] * X1[q] + nv[2] * X2[q];
        e[2][q] = w[0] * X0[q] + w[1] * X1[q] + w[2] * X2[q];
        e[3][q] = C(9, i)[q];
      }
      const double* S = C(10, i);
      const double yr = -(n + 1.0) * Pb;
      for (int k = 0; k < 4; ++k) {
        const double alr = f * e[k][0], ali = f * e[k][1];
        acc[k][0] = fma(yr, alr, acc[k][0]);
        acc[k][1] = fma(yr, ali, acc[k][1]);
        acc[k][2] = fma(D, alr, acc[k][2]);
        acc[k][3] = fma(D, ali, acc[k][3]);
        acc[k][4] = fma(-mQ, ali, acc[k][4]);
        acc[k][5] = fma(mQ, alr, acc[k][5]);
      }
      vr = fma(fs * Pb, S[0], vr);
      vi = fma(fs * Pb, S[1], vi);
    };
    if (m == 0) {
      double pm1 = 0.0, p0 = pmm;
      double z0 = 0.0, z1 = 1.2247448713915890 * pmm;  // Q_n^1, Q_{n+1}^1
      for (int n = 0; n <= a.p2; ++n) {
        const double* rc = rec + 6 * n;
        term(n, n, p0, rc[2] * st * z0, 0.0);
        const double pn1 = rc[0] * (ct * p0 - rc[1] * pm1);
        pm1 = p0;
        p0 = pn1;
        const double z2 = rc[4] * (ct * z1 - rc[5] * z0);
        z0 = z1;
        z1 = z2;
        rp *= ir;
      }
    } else {
      double qm1 = 0.0, q0 = qmm, q1 = rec[6 * off + 4] * ct * qmm;
      for (int n = m; n <= a.p2; ++n) {
        const int i = off + (n - m);
        const double* rc = rec + 6 * i;
        term(n, i, st * q0, rc[2] * q1 - rc[3] * qm1, m * q0);
        const double q2 = rc[0] * (ct * q1 - rc[1] * q0);
        qm1 = q0;
        q0 = q1;
        q1 = q2;
        rp *= ir;
      }
    }
    const double fac = (m == 0) ? 1.0 : 2.0;
    for (int k = 0; k < 4; ++k)
      for (int c3 = 0; c3 < 3; ++c3) gs[k][c3] += fac * (acc[k][2 * c3] * cm - acc[k][2 * c3 + 1] * sm_);
    sval += fac * (vr * cm - vi * sm_);
  }
  const double er[3] = {st * cph, st * sph, ct};
  const double et[3] = {ct * cph, ct * sph, -st};
  const double ep[3] = {-sph, cph, 0.0};
  double g[4][3];
  for (int k = 0; k < 4; ++k)
    for (int c3 = 0; c3 < 3; ++c3) g[k][c3] = gs[k][0] * er[c3] + gs[k][1] * et[c3] + gs[k][2] * ep[c3];
  const double dn = d[0] * nv[0] + d[1] * nv[1] + d[2] * nv[2];
  const double ng = nv[0] * g[3][0] + nv[1] * g[3][1] + nv[2] * g[3][2];
  const double dxg[3] = {d[1] * g[1][2] - d[2] * g[1][1], d[2] * g[1][0] - d[0] * g[1][2],
                         d[0] * g[1][1] - d[1] * g[1][0]};
  for (int c3 = 0; c3 < 3; ++c3)
    t[c3] = 2.0 * g[0][c3] + dxg[c3] + g[2][c3] + dn * g[3][c3] + d[c3] * ng + sval * nv[c3];
}

// grid (n_b, ceil(P / 256)); one thread per target node, the group walks the near list
// of its sphere.
__global__ __launch_bounds__(256) void near_traction_kernel(TracParams a) {
  extern __shared__ __align__(16) double sm[];
  const int t = blockIdx.x;
  const int s0 = a.near_ptr[t], s1 = a.near_ptr[t + 1];
  if (s0 == s1) return;
  double* cs = sm;                               // TR_NARR x ncoef2 x 2
  double* rec = sm + 2 * TR_NARR * a.ncoef2;     // ncoef2 x 6
  for (int i = threadIdx.x; i < 6 * a.ncoef2; i += blockDim.x) rec[i] = a.rec2[i];
  const int g = blockIdx.y * blockDim.x + threadIdx.x;
  const bool active = g < a.P;
  double o[3] = {0.0, 0.0, 1.0};
  if (active) {
    o[0] = a.otab[4 * g];
    o[1] = a.otab[4 * g + 1];
    o[2] = a.otab[4 * g + 2];
  }
  const double* ctp = a.centres4 + 4 * t;
  // spheres of radius a: the node is c_t + a_t o; the traction is scale invariant, so the
  // series is evaluated at (x - c_s) / a_s with no further factor
  const double at = a.radius ? a.radius[t] : 1.0;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = s0; e < s1; ++e) {
    const int s = a.near_idx[e];
    __syncthreads();
    build_slots(a, s, cs);
    __syncthreads();
    if (!active) continue;
    const double* csp = a.centres4 + 4 * s;
    double d[3] = {(ctp[0] - csp[0]) + at * o[0], (ctp[1] - csp[1]) + at * o[1], (ctp[2] - csp[2]) + at * o[2]};
    if (a.radius) {
      const double ias = 1.0 / a.radius[s];
      d[0] *= ias;
      d[1] *= ias;
      d[2] *= ias;
    }
    double tv[3];
    traction_point(a, cs, rec, d, o, tv);
    acc[0] += tv[0];
    acc[1] += tv[1];
    acc[2] += tv[2];
  }
  if (active) {
    double* uo = a.u + 3 * ((int64_t)t * a.P + g);
    uo[0] += acc[0];
    uo[1] += acc[1];
    uo[2] += acc[2];
  }
}

// u += a_k + b_k x (x - c_k) at every node of sphere k, ab = nb x 6 (a, b); x - c_k = r_k o
// (r_k = 1 without radii).
__global__ void k_add_rigid(const double* ab, const double* otab, const double* radius, int P, int64_t N,
                            double* u) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / P;
    const int li = (int)(g - k * P);
    const double r = radius ? radius[k] : 1.0;
    const double o[3] = {r * otab[4 * li], r * otab[4 * li + 1], r * otab[4 * li + 2]};
    const double* v = ab + 6 * k;
    u[3 * g + 0] += v[0] + (v[4] * o[2] - v[5] * o[1]);
    u[3 * g + 1] += v[1] + (v[5] * o[0] - v[3] * o[2]);
    u[3 * g + 2] += v[2] + (v[3] * o[1] - v[4] * o[0]);
  }
}

}  // namespace

void launch_near_traction(bie_ctx* c, double* u) {
  if (c->near_idx.empty()) return;
  if (c->ncoef2 == 0) {
    const int mm2 = std::min(c->mmax + 1, c->p + 1);
    std::vector<double> rec2 = recurrence_table(c->p + 1, mm2);
    c->rec2.alloc(rec2.size() * sizeof(double));
    BIE_HIP(hipMemcpy(c->rec2.ptr, rec2.data(), rec2.size() * sizeof(double), hipMemcpyHostToDevice));
    c->mm2 = mm2;
    c->ncoef2 = (int)(rec2.size() / 6);
  }
  TracParams a{};
  a.coef = c->coef.as<double>();
  a.centres4 = c->centres4.as<double>();
  a.near_ptr = c->dnear_ptr.as<int>();
  a.near_idx = c->dnear_idx.as<int>();
  a.otab = c->otab.as<double>();
  a.rec2 = c->rec2.as<double>();
  a.radius = c->poly ? c->radius_d.as<double>() : nullptr;
  a.u = u;
  a.p = c->p;
  a.mmax = c->mmax;
  a.P = c->P;
  a.ncoef = c->ncoef;
  a.p2 = c->p + 1;
  a.mm2 = c->mm2;
  a.ncoef2 = c->ncoef2;
  const size_t smem = (size_t)(2 * TR_NARR + 6) * c->ncoef2 * sizeof(double);
  const dim3 grid((unsigned)c->nb, (unsigned)((c->P + 255) / 256));
  near_traction_kernel<<<grid, dim3(256), smem, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

void add_rigid_local(bie_ctx* c, const double* ab, double* u, const double* radius) {
  const int blocks = (int)std::min<int64_t>((c->N + 255) / 256, 4096);
  k_add_rigid<<<dim3(blocks), dim3(256), 0, c->stream>>>(ab, c->otab.as<double>(), radius, c->P, c->N, u);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
