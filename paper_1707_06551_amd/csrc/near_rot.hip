// Near-pair correction by pole rotation and delayed evaluation (Section 4.2, Fig. 2), the
// alternative to the direct series at the target nodes (near.hip).
//
// For a directed near pair (source s, target t), d = c_t - c_s = L (sin b cos a,
// sin b sin a, cos b):
//  1. rotate the source coefficients into the frame whose pole points at c_t:
//     c^R = D(Q) c, Q = R_y(-b) R_z(-a), D(Q) = E diag(e^{i m b}) E^H diag(e^{i m a}) per
//     degree, with E = D(R_x(-pi/2)) (a rotation about y is the rotation about z
//     conjugated by R_x(-pi/2)) tabulated once at set-up; D is defined by
//     Y_n^m(Q^T x) = sum_m' D_m'm Y_n^m'(x), and one matrix per degree serves V, W and X
//     (they are built from Y_n^m by rotation-covariant operations, Eqs. 2.4-2.6);
//  2. evaluate the exterior series on the target grid translated to (0, 0, L): its nodes
//     have fixed (r, theta) per latitude and the grid's own phi_l, so each azimuthal
//     order m of the series is directly the order-m Fourier coefficient of the samples
//     (for |m| <= mmax no order |m| <= p aliases onto it); the source-frame spherical
//     components become the target's by the meridional rotation of angle
//     theta_s - theta_j, which does not depend on m;
//  3. project onto the target's V, W, X (the forward transform's Legendre stage, Eq. 4.4
//     weights), rotate back with D(Q^T) = diag(e^{-i m a}) E diag(e^{-i m b}) E^H and sum
//     over the target's near sources; one inverse transform per target sphere (the
//     transform kernel, accumulating into u) evaluates the sum (delayed evaluation).
// The result is the band-limited projection of the near field on the target sphere, not
// its values at the nodes.  One work-group per target sphere, float64, vectors and
// per-pair Fourier coefficients in LDS, deterministic order, no atomics.
// Spheres of radii a_s (source) and a_t (target): steps 1-3 run in units of a_s, where
// the source is a unit sphere: the translated grid sits at (0, 0, L / a_s) + (a_t / a_s) x
// (still a fixed (r, theta) per latitude) and the single layer's radial constants carry
// the factor a_s; rotations and the projection are angular and do not see the radii.
// The constants of the current pair are formed in LDS (for unit spheres they are the
// operator's own: a_s = 1 and no separate single-layer part).
#include "bie_internal.h"
#include "series.h"

namespace bie {

namespace {

struct RotParams {
  const double* coef;      // nb x 3 x ncoef x 2 source coefficients
  const double* centres4;  // nb x 4
  const int* near_ptr;
  const int* near_idx;
  const int* modes;        // ncoef x 2: (m, n) of each slot
  const double* rec;       // ncoef x 6 recurrence constants
  const double* leg;       // 3 x ncoef x nlat: Pbar, dPbar/dtheta, m Pbar/sin at the target latitudes
  const double* wlat;      // nlat latitude weights 2 pi lambda_j / n_phi
  const double* tlat;      // nlat cos(theta_j)
  const double* wig;       // per n, (2n+1)^2 complex (re, im): row m' + n, column m + n holds E_n[m', m]
  double* out;             // nb x 3 x ncoef x 2 accumulated target coefficients
  const double* radius;    // nb radii, or NULL for unit spheres
  int p, mmax, ncoef, nlat, nphi;
  double kvv[33], kww[33], kwv[33], kxx[33];   // a_S S + a_D D (unit) or a_D D (radii)
  double sv[33], sw[33], swv[33], sx[33];      // a_S S (radii; zero for unit spheres)
};

// radial constants of the current pair (LDS), read by series_order
struct RotK {
  int p, mmax, ncoef;
  const double *kvv, *kww, *kwv, *kxx;
};

__device__ inline int wig_off(int n) { return n * (2 * n - 1) * (2 * n + 1) / 3; }

// entry m (-n..n) of the full-order vector of a real field stored for m >= 0 in slots
__device__ inline void full_entry(const double* slots, int nc, int p, int mmax, int f, int n, int m, double& re,
                                  double& im) {
  const int am = m < 0 ? -m : m;
  if (am > mmax) {
    re = im = 0.0;
    return;
  }
  const double* c = slots + 2 * (f * nc + am * (p + 1) - (am * (am - 1)) / 2 + (n - am));
  re = c[0];
  im = m < 0 ? -c[1] : c[1];
}

// e^{i s m x} for m in -p..p from the tabulated cos / sin of |m| x (s = +1 or -1)
__device__ inline void phase(const double* cosv, const double* sinv, int m, double sgn, double& c, double& s) {
  const int am = m < 0 ? -m : m;
  c = cosv[am];
  s = (m < 0 ? -sgn : sgn) * sinv[am];
}

__global__ __launch_bounds__(256) void near_rot_kernel(RotParams a) {
  extern __shared__ __align__(16) double sm[];
  const int t = blockIdx.x;
  const int p = a.p, mmax = a.mmax, nc = a.ncoef, nl = a.nlat, M1 = mmax + 1;
  const int nfull = (p + 1) * (p + 1);
  // F (written in step 2, read in 3a) shares B's space (read last in 1c, written again
  // in 3c); barriers separate those phases
  const int fb = 6 * nfull > 6 * nl * M1 ? 6 * nfull : 6 * nl * M1;
  double* A = sm;                      // 3 x nfull x 2, order k = n^2 + m + n
  double* B = A + 6 * nfull;           // 3 x nfull x 2
  double* F = B;                       // 3 x nl x M1 x 2
  double* U = B + fb;                  // 3 x nc x 2, slot layout
  double* ACC = U + 6 * nc;            // 3 x nc x 2
  double* rec = ACC + 6 * nc;          // nc x 6
  double* ca = rec + 6 * nc;           // cos(m a), sin(m a), cos(m b), sin(m b), m = 0..p
  double* sa = ca + (p + 1);
  double* cb = sa + (p + 1);
  double* sb = cb + (p + 1);
  double* kc = sb + (p + 1);           // 4 x 33 radial constants of the current pair
  const RotK kr{p, mmax, nc, kc, kc + 33, kc + 66, kc + 99};
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < 6 * nc; i += nt) {
    rec[i] = a.rec[i];
    ACC[i] = 0.0;
  }
  const int s0 = a.near_ptr[t], s1 = a.near_ptr[t + 1];
  const double ctx = a.centres4[4 * t], cty = a.centres4[4 * t + 1], ctz = a.centres4[4 * t + 2];
  const double rt = a.radius ? a.radius[t] : 1.0;
  const auto Ucoef = [U, nc](int f, int i) { return U + 2 * (f * nc + i); };
  for (int e = s0; e < s1; ++e) {
    const int s = a.near_idx[e];
    const double dx = ctx - a.centres4[4 * s], dy = cty - a.centres4[4 * s + 1], dz = ctz - a.centres4[4 * s + 2];
    const double L = sqrt(dx * dx + dy * dy + dz * dz);
    const double al = atan2(dy, dx);
    const double be = acos(fmin(1.0, fmax(-1.0, dz / L)));
    const double* cs = a.coef + (size_t)s * 6 * nc;
    const double rs = a.radius ? a.radius[s] : 1.0;
    const double Ls = L / rs, rho = rt / rs;   // in units of the source radius
    __syncthreads();
    for (int m = tid; m <= p; m += nt) {
      sincos(m * al, &sa[m], &ca[m]);
      sincos(m * be, &sb[m], &cb[m]);
      kc[m] = fma(rs, a.sv[m], a.kvv[m]);
      kc[33 + m] = fma(rs, a.sw[m], a.kww[m]);
      kc[66 + m] = fma(rs, a.swv[m], a.kwv[m]);
      kc[99 + m] = fma(rs, a.sx[m], a.kxx[m]);
    }
    __syncthreads();
    // 1a. A = diag(e^{i m a}) c
    for (int it = tid; it < 3 * nfull; it += nt) {
      const int f = it / nfull, k = it - f * nfull;
      const int n = (int)sqrt((double)k + 0.5), m = k - n * n - n;
      double re, im, c, sn;
      full_entry(cs, nc, p, mmax, f, n, m, re, im);
      phase(ca, sa, m, 1.0, c, sn);
      A[2 * it] = re * c - im * sn;
      A[2 * it + 1] = re * sn + im * c;
    }
    __syncthreads();
    // 1b. B = E^H A
    for (int it = tid; it < 3 * nfull; it += nt) {
      const int f = it / nfull, k = it - f * nfull;
      const int n = (int)sqrt((double)k + 0.5), mp = k - n * n - n;
      const double* E = a.wig + 2 * wig_off(n);
      const double* v = A + 2 * (f * nfull + n * n);
      const int w = 2 * n + 1;
      double re = 0, im = 0;
      for (int j = 0; j < w; ++j) {
        const double er = E[2 * (j * w + mp + n)], ei = -E[2 * (j * w + mp + n) + 1];
        re += er * v[2 * j] - ei * v[2 * j + 1];
        im += er * v[2 * j + 1] + ei * v[2 * j];
      }
      B[2 * it] = re;
      B[2 * it + 1] = im;
    }
    __syncthreads();
    // 1c. U = E diag(e^{i m b}) B, orders m' = 0..mmax only
    for (int it = tid; it < 3 * nc; it += nt) {
      const int f = it / nc, i = it - f * nc;
      const int mp = a.modes[2 * i], n = a.modes[2 * i + 1];
      const double* E = a.wig + 2 * (wig_off(n) + (mp + n) * (2 * n + 1));
      const double* v = B + 2 * (f * nfull + n * n);
      double re = 0, im = 0;
      for (int j = 0; j < 2 * n + 1; ++j) {
        double c, sn;
        phase(cb, sb, j - n, 1.0, c, sn);
        const double vr = v[2 * j] * c - v[2 * j + 1] * sn, vi = v[2 * j] * sn + v[2 * j + 1] * c;
        re += E[2 * j] * vr - E[2 * j + 1] * vi;
        im += E[2 * j] * vi + E[2 * j + 1] * vr;
      }
      U[2 * it] = re;
      U[2 * it + 1] = im;
    }
    __syncthreads();
    // 2. order-m Fourier coefficients of the series on the translated target grid, in the
    //    target's spherical components, times n_phi (the forward DFT's normalisation)
    for (int it = tid; it < nl * M1; it += nt) {
      const int j = it / M1, m = it - j * M1;
      const double tj = a.tlat[j], sj = sqrt(fmax(0.0, 1.0 - tj * tj));
      const double z = Ls + rho * tj, h = rho * sj;
      const double r = sqrt(h * h + z * z);
      const double ir = 1.0 / r, ir2 = ir * ir;
      const double ct = z * ir, st = h * ir;
      double pmm = 0.28209479177387814, qmm = 0.0, irm = 1.0;
      for (int q = 1; q <= m; ++q) {
        const double fq = rec[6 * (q * (p + 1) - (q * (q - 1)) / 2) + 5];
        qmm = fq * pmm;
        pmm = fq * st * pmm;
        irm *= ir;
      }
      double sv[6];
      series_order(kr, Ucoef, rec, m, ct, st, ir, ir2, irm, pmm, qmm, sv);
      const double cd = ct * tj + st * sj, sd = st * tj - ct * sj;   // cos, sin (theta_s - theta_j)
      const double g = (double)a.nphi;
      double* Fr = F + 2 * ((0 * nl + j) * M1 + m);
      double* Ft = F + 2 * ((1 * nl + j) * M1 + m);
      double* Fp = F + 2 * ((2 * nl + j) * M1 + m);
      Fr[0] = g * (sv[0] * cd - sv[2] * sd);
      Fr[1] = g * (sv[1] * cd - sv[3] * sd);
      Ft[0] = g * (sv[0] * sd + sv[2] * cd);
      Ft[1] = g * (sv[1] * sd + sv[3] * cd);
      Fp[0] = g * sv[4];
      Fp[1] = g * sv[5];
    }
    __syncthreads();
    // 3a. projection onto the target's V, W, X (as the forward transform)
    for (int i = tid; i < nc; i += nt) {
      const int m = a.modes[2 * i], n = a.modes[2 * i + 1];
      const double* Lp = a.leg + ((size_t)0 * nc + i) * nl;
      const double* Ld = a.leg + ((size_t)1 * nc + i) * nl;
      const double* Lq = a.leg + ((size_t)2 * nc + i) * nl;
      double ar = 0, ai = 0, btr = 0, bti = 0, bpr = 0, bpi = 0, ctr = 0, cti = 0, cpr = 0, cpi = 0;
      for (int j = 0; j < nl; ++j) {
        const double w = a.wlat[j];
        const double pw = w * Lp[j], dw = w * Ld[j], qw = w * Lq[j];
        const double* Fr = F + 2 * ((0 * nl + j) * M1 + m);
        const double* Ft = F + 2 * ((1 * nl + j) * M1 + m);
        const double* Fp = F + 2 * ((2 * nl + j) * M1 + m);
        ar += pw * Fr[0];
        ai += pw * Fr[1];
        btr += dw * Ft[0];
        bti += dw * Ft[1];
        bpr += dw * Fp[0];
        bpi += dw * Fp[1];
        ctr += qw * Ft[0];
        cti += qw * Ft[1];
        cpr += qw * Fp[0];
        cpi += qw * Fp[1];
      }
      const double gr = btr + cpi, gi = bti - cpr;
      const double nn = n;
      double* u0 = U + 2 * i;
      double* u1 = U + 2 * (nc + i);
      double* u2 = U + 2 * (2 * nc + i);
      u0[0] = (gr - (nn + 1) * ar) / ((nn + 1) * (2 * nn + 1));
      u0[1] = (gi - (nn + 1) * ai) / ((nn + 1) * (2 * nn + 1));
      if (n >= 1) {
        u1[0] = (gr + nn * ar) / (nn * (2 * nn + 1));
        u1[1] = (gi + nn * ai) / (nn * (2 * nn + 1));
        u2[0] = (bpr - cti) / (nn * (nn + 1));
        u2[1] = (bpi + ctr) / (nn * (nn + 1));
      } else {
        u1[0] = u1[1] = u2[0] = u2[1] = 0.0;
      }
    }
    __syncthreads();
    // 3b. A = full-order vectors of U
    for (int it = tid; it < 3 * nfull; it += nt) {
      const int f = it / nfull, k = it - f * nfull;
      const int n = (int)sqrt((double)k + 0.5), m = k - n * n - n;
      full_entry(U, nc, p, mmax, f, n, m, A[2 * it], A[2 * it + 1]);
    }
    __syncthreads();
    // 3c. B = E^H A
    for (int it = tid; it < 3 * nfull; it += nt) {
      const int f = it / nfull, k = it - f * nfull;
      const int n = (int)sqrt((double)k + 0.5), mp = k - n * n - n;
      const double* E = a.wig + 2 * wig_off(n);
      const double* v = A + 2 * (f * nfull + n * n);
      const int w = 2 * n + 1;
      double re = 0, im = 0;
      for (int j = 0; j < w; ++j) {
        const double er = E[2 * (j * w + mp + n)], ei = -E[2 * (j * w + mp + n) + 1];
        re += er * v[2 * j] - ei * v[2 * j + 1];
        im += er * v[2 * j + 1] + ei * v[2 * j];
      }
      B[2 * it] = re;
      B[2 * it + 1] = im;
    }
    __syncthreads();
    // 3d. ACC += diag(e^{-i m a}) E diag(e^{-i m b}) B, orders m' = 0..mmax
    for (int it = tid; it < 3 * nc; it += nt) {
      const int f = it / nc, i = it - f * nc;
      const int mp = a.modes[2 * i], n = a.modes[2 * i + 1];
      const double* E = a.wig + 2 * (wig_off(n) + (mp + n) * (2 * n + 1));
      const double* v = B + 2 * (f * nfull + n * n);
      double re = 0, im = 0;
      for (int j = 0; j < 2 * n + 1; ++j) {
        double c, sn;
        phase(cb, sb, j - n, -1.0, c, sn);
        const double vr = v[2 * j] * c - v[2 * j + 1] * sn, vi = v[2 * j] * sn + v[2 * j + 1] * c;
        re += E[2 * j] * vr - E[2 * j + 1] * vi;
        im += E[2 * j] * vi + E[2 * j + 1] * vr;
      }
      double c, sn;
      phase(ca, sa, mp, -1.0, c, sn);
      ACC[2 * it] += re * c - im * sn;
      ACC[2 * it + 1] += re * sn + im * c;
    }
  }
  __syncthreads();
  double* o = a.out + (size_t)t * 6 * nc;
  for (int i = tid; i < 6 * nc; i += nt) o[i] = ACC[i];
}

}  // namespace

static size_t rot_smem(const bie_ctx* c) {
  const size_t nfull = (size_t)(c->p + 1) * (c->p + 1);
  const size_t fb = std::max(6 * nfull, 6 * (size_t)c->nlat * (c->mmax + 1));   // B and F share it
  return sizeof(double) * (6 * nfull + fb + 18 * (size_t)c->ncoef + 4 * (c->p + 1) + 4 * 33);
}

void launch_near_rot(bie_ctx* c, const OpSpec& spec, double* u) {
  if (c->near_idx.empty()) return;
  RotParams a{};
  a.coef = c->coef.as<double>();
  a.centres4 = c->centres4.as<double>();
  a.near_ptr = c->dnear_ptr.as<int>();
  a.near_idx = c->dnear_idx.as<int>();
  a.modes = c->modes.as<int>();
  a.rec = c->rec.as<double>();
  a.leg = c->leg.as<double>();
  a.wlat = c->wlat_d.as<double>();
  a.tlat = c->tlat_d.as<double>();
  a.wig = c->wig.as<double>();
  a.out = c->nearcoef.as<double>();
  a.p = c->p;
  a.mmax = c->mmax;
  a.ncoef = c->ncoef;
  a.nlat = c->nlat;
  a.nphi = c->n_phi;
  if (c->poly) {
    a.radius = c->radius_d.as<double>();
    series_radial(0.0, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);
    series_radial(spec.a_s, 0.0, c->p, a.sv, a.sw, a.swv, a.sx);
  } else {
    series_radial(spec.a_s, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);   // a.sv... stay zero
  }
  const size_t sm = rot_smem(c);
  BIE_HIP(hipFuncSetAttribute((const void*)near_rot_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
  near_rot_kernel<<<dim3((unsigned)c->nb), dim3(256), sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
  // delayed evaluation: one synthesis per target sphere, added to u
  VshCall v;
  v.coef_in = c->nearcoef.as<double>();
  v.u = u;
  v.coef_is_input = true;
  v.accumulate = true;
  launch_vsh(c, BIE_FP64, v);
}

}  // namespace bie
