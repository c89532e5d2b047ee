// Near-pair correction (Section 4.1, near-singular integrands; Eqs. 3.6-3.11 exterior).
//
// For every directed near pair (source s, target t) and every node x of sphere t, the
// layer potential a_S S[mu_s] + a_D D[mu_s] is evaluated from the V, W, X coefficients of
// the density of sphere s by the exterior formulas, in float64.  With (r, theta, phi) the
// spherical coordinates of x - c_s, Q_n^m = Pbar_n^m / sin(theta) and the radial powers of
// the formulas, the series of one azimuthal order m >= 1 is
//   u_r = sum_n y_n Pbar_n,   u_theta = sum_n g_n dPbar_n - i m Q_n gamma_n,
//   u_phi = sum_n i m Q_n g_n + dPbar_n gamma_n,
// with alpha = f_VV V^ + f_WV W^, beta = f_WW W^, gamma = f_XX X^, y = -(n+1) alpha + n
// beta, g = alpha + beta and dPbar_n = a_n^m Q_{n+1} - b_n^m Q_{n-1} (the recurrence of
// Eq. 2.9).  Two rewrites make the per-target work small:
//  - every radial factor is r^-n times one of 1, r^-1, r^-2, so the Legendre values are
//    carried pre-scaled, q_n = r^-n Q_n e^{i m phi} (the recurrence absorbs 1/r), and
//    the remaining factors r, 1/r, 1/r^2, 1/r^3, sin(theta) are applied once per target
//    and source at the end;
//  - the shifted terms of dPbar are re-indexed onto q_n, so that each (n, m) contributes
//    Re(C q_n) to seven real accumulators, one per remaining factor, with complex
//    constants C that depend only on the source's coefficients.
// The constants (16 float64 per (n, m): seven complex C and the two recurrence
// coefficients) are formed once per source and matvec by near_table_kernel; the target
// kernel reads them through the scalar data cache (wave-uniform addresses, SGPR operands:
// float64 VALU instructions issue at full rate with one), so a term costs 14 FMAs into the
// accumulators and 6 operations of recurrence.  Order m = 0 (real parts only) has its own
// five accumulators.
//
// One work-group per target sphere with near neighbours, blocks ordered by decreasing
// near count (longest first), one thread per target node (the nodes in chunks of the
// block size); each thread walks the sphere's near list in order, so every target is
// written by exactly one thread (no atomics, deterministic order).
#include <algorithm>
#include <numeric>

#include "bie_internal.h"

namespace bie {

constexpr int NEAR_SLOT = 16;  // float64 per (n, m) table slot

// Table of one source sphere, slot order: m = 0, n = 0..p; then m = 1..mmax, n = m..p+1.
//  m = 0:  [0] Y1, [1] Y0, [2] G1 a, [3] G0 a, [4] X0 a, [5] A0, [6] A0 B0, [7] A1, [8] A1 B1
//          (real parts; a = -sqrt(n (n+1)) of dPbar_n^0 = a sin(theta) Q_n^1, A0 B0 the
//          order-0 recurrence producing degree n+1, A1 B1 the order-1 one producing n+2)
//  m >= 1: seven (Re, -Im) pairs of 2 C, the constants of Re(C q_n) for the factors
//          [0] sin(theta)/r^2, [2] sin(theta), [4] 1/r, [6] r, [8] -1/r^3 (u_theta),
//          [10] 1/r^2, [12] 1 (u_phi); [14] A, [15] A B of the recurrence of slot n,
//          q_{n+2} = A (cos(theta)/r q_{n+1} - B q_n / r^2)
// with (per degree n; c0, c1, c2 the V, W, X coefficients; k the radial constants)
//   a1 = kvv c0 + kwv c1, a0 = -kwv c1, b0 = kww c1, X0 = kxx c2,
//   Y1 = -(n+1) a1, Y0 = -(n+1) a0 + n b0, G1 = a1, G0 = a0 + b0.
struct NearTableParams {
  const double* coef;      // nb x 3 x ncoef x 2
  const double* rec;       // ncoef x 6 recurrence table (setup.cpp)
  const double* radius;    // nb radii or nullptr (unit spheres)
  double* table;           // nb x nslot x 16
  int p, mmax, ncoef, nslot;
  double kvv[33], kww[33], kwv[33], kxx[33];  // a_D D (+ a_S S for unit spheres)
  double sv[33], sw[33], swv[33], sx[33];     // a_S S, scaled by the source radius (radii only)
};

__global__ void near_table_kernel(NearTableParams a) {
  const int64_t s = blockIdx.y;
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= a.nslot) return;
  const int nc = a.ncoef;
  const double* cs = a.coef + s * 6 * nc;
  const double as = a.radius ? a.radius[s] : 1.0;
  double* out = a.table + (s * a.nslot + slot) * NEAR_SLOT;
  // slot -> (m, n)
  int m = 0, n = slot;
  if (slot > a.p) {
    int rem = slot - (a.p + 1);
    m = 1;
    while (rem >= a.p + 2 - m) {
      rem -= a.p + 2 - m;
      ++m;
    }
    n = m + rem;
  }
  const int off = m * (a.p + 1) - (m * (m - 1)) / 2;  // coefficient slot of (m, m)
  // the four complex combinations of degree k (zero outside m <= k <= p)
  auto combos = [&](int k, double* y1, double* y0, double* g1, double* g0, double* x0) {
    for (int j = 0; j < 2; ++j) y1[j] = y0[j] = g1[j] = g0[j] = x0[j] = 0.0;
    if (k < m || k > a.p) return;
    const int i = off + (k - m);
    const double kvv = a.radius ? fma(as, a.sv[k], a.kvv[k]) : a.kvv[k];
    const double kww = a.radius ? fma(as, a.sw[k], a.kww[k]) : a.kww[k];
    const double kwv = a.radius ? fma(as, a.swv[k], a.kwv[k]) : a.kwv[k];
    const double kxx = a.radius ? fma(as, a.sx[k], a.kxx[k]) : a.kxx[k];
    for (int j = 0; j < 2; ++j) {
      const double c0 = cs[2 * i + j], c1 = cs[2 * (nc + i) + j], c2 = cs[2 * (2 * nc + i) + j];
      const double a1 = kvv * c0 + kwv * c1, a0 = -kwv * c1, b0 = kww * c1;
      y1[j] = -(k + 1.0) * a1;
      y0[j] = -(k + 1.0) * a0 + k * b0;
      g1[j] = a1;
      g0[j] = a0 + b0;
      x0[j] = kxx * c2;
    }
  };
  double y1[2], y0[2], g1[2], g0[2], x0[2];
  if (m == 0) {
    combos(n, y1, y0, g1, g0, x0);
    const double* rc = a.rec + 6 * n;
    out[0] = y1[0];
    out[1] = y0[0];
    out[2] = g1[0] * rc[2];
    out[3] = g0[0] * rc[2];
    out[4] = x0[0] * rc[2];
    out[5] = rc[0];
    out[6] = rc[0] * rc[1];
    out[7] = rc[4];
    out[8] = rc[4] * rc[5];
    for (int j = 9; j < NEAR_SLOT; ++j) out[j] = 0.0;
    return;
  }
  double ym1[2], yp1[2], g1m[2], g0m[2], g1p[2], g0p[2], xm[2], xp[2], dum[2], dum2[2];
  combos(n, y1, y0, g1, g0, x0);
  combos(n - 1, ym1, dum, g1m, g0m, xm);
  combos(n + 1, yp1, dum2, g1p, g0p, xp);
  // a_k^m (coefficient of Q_{k+1} in dPbar_k) of degree n - 1, b_k^m (of Q_{k-1}) of degree n + 1
  const double am = (n - 1 >= m && n - 1 <= a.p) ? a.rec[6 * (off + n - 1 - m) + 2] : 0.0;
  const double bp = (n + 1 <= a.p) ? a.rec[6 * (off + n + 1 - m) + 3] : 0.0;
  const double fm = (double)m;
  double C[7][2];
  for (int j = 0; j < 2; ++j) {
    // i m Z = m (-Z_im, Z_re)
    const double imx = (j == 0) ? -fm * x0[1] : fm * x0[0];
    const double img1 = (j == 0) ? -fm * g1[1] : fm * g1[0];
    const double img0 = (j == 0) ? -fm * g0[1] : fm * g0[0];
    C[0][j] = y1[j];
    C[1][j] = y0[j];
    C[2][j] = am * g1m[j] - bp * g0p[j] - imx;
    C[3][j] = am * g0m[j];
    C[4][j] = bp * g1p[j];
    C[5][j] = img1 - bp * xp[j];
    C[6][j] = img0 + am * xm[j];
  }
  // factor 2 of the orders +-m of a real field; (Re, -Im) so that Re(C q) is two FMAs
  for (int k = 0; k < 7; ++k) {
    out[2 * k] = 2.0 * C[k][0];
    out[2 * k + 1] = -2.0 * C[k][1];
  }
  if (n <= a.p) {
    const double* rc = a.rec + 6 * (off + n - m);
    out[14] = rc[0];
    out[15] = rc[0] * rc[1];
  } else {
    out[14] = out[15] = 0.0;
  }
}

struct NearParams {
  const double* table;      // nb x nslot x 16 (near_table_kernel)
  const double* centres4;   // nb x 4
  const double* radius;     // nb radii or nullptr
  const int* near_ptr;
  const int* near_idx;
  const int* order;         // target spheres with near neighbours, longest list first
  const double* otab;       // P x 4
  double* u;
  int p, mmax, P, nslot;
  double fm[33];            // sqrt((2m+1)/(2m)): Pbar_m^m = fm sin(theta) Pbar_{m-1}^{m-1}
  double g4[33];            // sqrt(2m+3): Q_{m+1}^m = g4 cos(theta) Q_m^m
};

typedef __attribute__((address_space(4))) const double CDouble;

__global__ __launch_bounds__(1024) void near_kernel(NearParams a) {
  const int t = a.order[blockIdx.x];
  const int e0 = a.near_ptr[t], e1 = a.near_ptr[t + 1];
  const double ctx = a.centres4[4 * t], cty = a.centres4[4 * t + 1], ctz = a.centres4[4 * t + 2];
  const double at = a.radius ? a.radius[t] : 1.0;
  const int stride = (a.p + 1) * NEAR_SLOT;  // m = 0 block of a table
  for (int g = threadIdx.x; g < a.P; g += blockDim.x) {
    const double ox = at * a.otab[4 * g], oy = at * a.otab[4 * g + 1], oz = at * a.otab[4 * g + 2];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int s = ((const __attribute__((address_space(4))) int*)a.near_idx)[e];
      const CDouble* tab = (const CDouble*)(a.table + (int64_t)s * a.nslot * NEAR_SLOT);
      const double ias = a.radius ? 1.0 / a.radius[s] : 1.0;
      const double dx = ((ctx - a.centres4[4 * s]) + ox) * ias;
      const double dy = ((cty - a.centres4[4 * s + 1]) + oy) * ias;
      const double dz = ((ctz - a.centres4[4 * s + 2]) + oz) * ias;
      const double rho2 = fma(dx, dx, dy * dy);
      const double r = sqrt(fma(dz, dz, rho2));
      const double ir = 1.0 / r;
      const double ct = dz * ir;
      const double rho = sqrt(rho2);
      const double st = rho * ir;
      double cph = 1.0, sph = 0.0;
      if (rho > 0.0) {
        const double irho = 1.0 / rho;
        cph = dx * irho;
        sph = dy * irho;
      }
      const double ir2 = ir * ir, ctir = ct * ir;
      // ---- order 0 ----
      double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0;
      {
        double pm = 0.0, p0 = 0.28209479177387814;  // r^-n Pbar_n^0: degrees n-1, n
        double z0 = 0.0, z1 = 1.2247448713915890 * 0.28209479177387814 * ir;  // r^-n Q_n^1: n, n+1
#pragma unroll 2
        for (int n = 0; n <= a.p; ++n) {
          const CDouble* c = tab + n * NEAR_SLOT;
          A0 = fma(c[0], p0, A0);
          A1 = fma(c[1], p0, A1);
          A2 = fma(c[2], z0, A2);
          A3 = fma(c[3], z0, A3);
          A4 = fma(c[4], z0, A4);
          const double pn = fma(c[5] * ctir, p0, -(c[6] * ir2) * pm);
          pm = p0;
          p0 = pn;
          const double z2 = fma(c[7] * ctir, z1, -(c[8] * ir2) * z0);
          z0 = z1;
          z1 = z2;
        }
      }
      // ---- orders m >= 1 ----
      double R2 = 0, R0 = 0, T1 = 0, Tp = 0, T3 = 0, P2 = 0, P0 = 0;
      {
        double pmm = 0.28209479177387814, cm = 1.0, sm = 0.0, irm = 1.0;
        const CDouble* c = tab + stride;
        for (int m = 1; m <= a.mmax; ++m) {
          const double qmm = a.fm[m] * pmm;
          pmm = a.fm[m] * st * pmm;
          const double c2 = cm * cph - sm * sph;
          sm = fma(sm, cph, cm * sph);
          cm = c2;
          irm *= ir;
          // q_m and q_{m+1} = r^-n Q_n^m e^{i m phi}
          const double qm = irm * qmm;
          double q0r = qm * cm, q0i = qm * sm;
          const double f1 = a.g4[m] * ctir;
          double q1r = f1 * q0r, q1i = f1 * q0i;
#pragma unroll 2
          for (int n = m; n <= a.p + 1; ++n, c += NEAR_SLOT) {
            R2 = fma(c[1], q0i, fma(c[0], q0r, R2));
            R0 = fma(c[3], q0i, fma(c[2], q0r, R0));
            T1 = fma(c[5], q0i, fma(c[4], q0r, T1));
            Tp = fma(c[7], q0i, fma(c[6], q0r, Tp));
            T3 = fma(c[9], q0i, fma(c[8], q0r, T3));
            P2 = fma(c[11], q0i, fma(c[10], q0r, P2));
            P0 = fma(c[13], q0i, fma(c[12], q0r, P0));
            const double ea = c[14] * ctir, fb = c[15] * ir2;
            const double q2r = fma(ea, q1r, -fb * q0r);
            const double q2i = fma(ea, q1i, -fb * q0i);
            q0r = q1r;
            q0i = q1i;
            q1r = q2r;
            q1i = q2i;
          }
        }
      }
      const double ur = fma(ir2, A0, A1) + st * fma(ir2, R2, R0);
      const double ut = st * fma(ir2, A2, A3) + fma(ir, T1, fma(r, Tp, -(ir * ir2) * T3));
      const double up = st * ir * A4 + fma(ir2, P2, P0);
      // spherical (about c_s) -> Cartesian
      const double erx = st * cph, ery = st * sph, erz = ct;
      const double etx = ct * cph, ety = ct * sph, etz = -st;
      ax += ur * erx + ut * etx - up * sph;
      ay += ur * ery + ut * ety + up * cph;
      az += ur * erz + ut * etz;
    }
    double* uo = a.u + 3 * ((int64_t)t * a.P + g);
    uo[0] += ax;
    uo[1] += ay;
    uo[2] += az;
  }
}

// Radial constants of the exterior series (Eqs. 3.6-3.11, exterior branches) of
// a_S S + a_D D for n = 0..p.
void series_radial(double a_s, double a_d, int p, double* kvv, double* kww, double* kwv, double* kxx) {
  for (int n = 0; n <= p; ++n) {
    const double dn = n;
    kvv[n] = a_s * dn / ((2 * dn + 1) * (2 * dn + 3)) + a_d * (2 * dn * dn + 4 * dn + 3) / ((2 * dn + 1) * (2 * dn + 3));
    if (n == 0) {
      kww[n] = kwv[n] = kxx[n] = 0.0;
      continue;
    }
    kww[n] = a_s * (dn + 1) / ((2 * dn + 1) * (2 * dn - 1)) + a_d * 2.0 * (dn + 1) * (dn - 1) / ((2 * dn + 1) * (2 * dn - 1));
    kwv[n] = a_s * dn / (4 * dn + 2) + a_d * 2.0 * dn * (dn - 1) / (4 * dn + 2);
    kxx[n] = a_s / (2 * dn + 1) + a_d * (dn - 1) / (2 * dn + 1);
  }
}

int near_table_slots(int p, int mmax) {
  int n = p + 1;
  for (int m = 1; m <= mmax; ++m) n += p + 2 - m;
  return n;
}

// Target spheres with near neighbours, longest near list first (ties by index).
std::vector<int> near_launch_order(const std::vector<int>& near_ptr, int64_t nb) {
  std::vector<int> order;
  for (int64_t t = 0; t < nb; ++t)
    if (near_ptr[t + 1] > near_ptr[t]) order.push_back((int)t);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return near_ptr[x + 1] - near_ptr[x] > near_ptr[y + 1] - near_ptr[y];
  });
  return order;
}

void launch_near(bie_ctx* c, const OpSpec& spec, double* u) {
  if (c->near_idx.empty()) return;
  if (c->near_method == 1) {
    launch_near_rot(c, spec, u);
    return;
  }
  NearTableParams tp{};
  tp.coef = c->coef.as<double>();
  tp.rec = c->rec.as<double>();
  tp.radius = c->poly ? c->radius_d.as<double>() : nullptr;
  tp.table = c->neartab.as<double>();
  tp.p = c->p;
  tp.mmax = c->mmax;
  tp.ncoef = c->ncoef;
  tp.nslot = c->near_slots;
  if (c->poly) {
    series_radial(0.0, spec.a_d, c->p, tp.kvv, tp.kww, tp.kwv, tp.kxx);
    series_radial(spec.a_s, 0.0, c->p, tp.sv, tp.sw, tp.swv, tp.sx);
  } else {
    series_radial(spec.a_s, spec.a_d, c->p, tp.kvv, tp.kww, tp.kwv, tp.kxx);
  }
  near_table_kernel<<<dim3((unsigned)((tp.nslot + 63) / 64), (unsigned)c->nb), dim3(64), 0, c->stream>>>(tp);
  BIE_HIP(hipGetLastError());

  NearParams a{};
  a.table = tp.table;
  a.centres4 = c->centres4.as<double>();
  a.radius = tp.radius;
  a.near_ptr = c->dnear_ptr.as<int>();
  a.near_idx = c->dnear_idx.as<int>();
  a.order = c->dnear_order.as<int>();
  a.otab = c->otab.as<double>();
  a.u = u;
  a.p = c->p;
  a.mmax = c->mmax;
  a.P = c->P;
  a.nslot = c->near_slots;
  for (int m = 1; m <= c->mmax; ++m) {
    a.fm[m] = std::sqrt((2.0 * m + 1.0) / (2.0 * m));
    a.g4[m] = std::sqrt(2.0 * m + 3.0);
  }
  const int threads = std::min(1024, ((c->P + 63) / 64) * 64);
  near_kernel<<<dim3((unsigned)c->n_near_targets), dim3(threads), 0, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
