// Near-pair correction (Section 4.1, near-singular integrands; Eqs. 3.6-3.11 exterior).
//
// For every directed near pair (source s, target t) and every node x of sphere t, the
// layer potential a_S S[mu_s] + a_D D[mu_s] is evaluated from the V, W, X coefficients of
// the density of sphere s by the exterior formulas, in float64 (series.h).  One
// work-group per target sphere (one thread per target node); the group walks the near
// list of its sphere, staging each source's coefficients in LDS, so every target is
// written by exactly one thread (no atomics, deterministic order).
#include "bie_internal.h"
#include "series.h"

namespace bie {

struct NearParams {
  const double* coef;      // nb x 3 x ncoef x 2
  const double* centres4;  // nb x 4
  const int* near_ptr;
  const int* near_idx;
  const double* otab;      // P x 4
  const double* rec;       // ncoef x 6 recurrence table
  double* u;
  int p, mmax, P, ncoef;
  double kvv[33], kww[33], kwv[33], kxx[33];
};

__global__ __launch_bounds__(1024) void near_kernel(NearParams a) {
  extern __shared__ __align__(16) double sm[];
  const int t = blockIdx.x;
  const int s0 = a.near_ptr[t], s1 = a.near_ptr[t + 1];
  if (s0 == s1) return;
  const int nc = a.ncoef;
  double* cs = sm;               // 3 x nc x 2 coefficients of the current source
  double* rec = sm + 6 * nc;     // nc x 6
  for (int i = threadIdx.x; i < 6 * nc; i += blockDim.x) rec[i] = a.rec[i];
  const int g = threadIdx.x;
  const bool active = g < a.P;
  const double ctx = a.centres4[4 * t], cty = a.centres4[4 * t + 1], ctz = a.centres4[4 * t + 2];
  double ox = 0, oy = 0, oz = 0;
  if (active) {
    ox = a.otab[4 * g];
    oy = a.otab[4 * g + 1];
    oz = a.otab[4 * g + 2];
  }
  double acc0 = 0, acc1 = 0, acc2 = 0;
  for (int e = s0; e < s1; ++e) {
    const int s = a.near_idx[e];
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * nc; i += blockDim.x) cs[i] = a.coef[(size_t)s * 6 * nc + i];
    __syncthreads();
    if (!active) continue;
    const double dx = (ctx - a.centres4[4 * s]) + ox;
    const double dy = (cty - a.centres4[4 * s + 1]) + oy;
    const double dz = (ctz - a.centres4[4 * s + 2]) + oz;
    exterior_series(a, cs, rec, dx, dy, dz, acc0, acc1, acc2);
  }
  if (active) {
    double* uo = a.u + 3 * ((int64_t)t * a.P + g);
    uo[0] += acc0;
    uo[1] += acc1;
    uo[2] += acc2;
  }
}

// Spheres of radius a: the exterior series of source s is evaluated at (x - c_s) / a_s
// with its single-layer constants scaled by a_s (the single layer is homogeneous of
// degree 1 in the length scale, the double layer of degree 0); the per-source constants
// are formed in LDS.  Same structure as near_kernel otherwise.
struct NearRadParams {
  NearParams b;
  const double* radius;                    // nb radii
  double sv[33], sw[33], swv[33], sx[33];  // single-layer part of the constants (a_S S)
};

struct NearK {
  int p, mmax, ncoef;
  const double *kvv, *kww, *kwv, *kxx;
};

__global__ __launch_bounds__(1024) void near_kernel_radii(NearRadParams ar) {
  extern __shared__ __align__(16) double sm[];
  const NearParams& a = ar.b;
  const int t = blockIdx.x;
  const int s0 = a.near_ptr[t], s1 = a.near_ptr[t + 1];
  if (s0 == s1) return;
  const int nc = a.ncoef;
  double* cs = sm;               // 3 x nc x 2
  double* rec = sm + 6 * nc;     // nc x 6
  double* kc = sm + 12 * nc;     // 4 x 33 constants of the current source
  for (int i = threadIdx.x; i < 6 * nc; i += blockDim.x) rec[i] = a.rec[i];
  const int g = threadIdx.x;
  const bool active = g < a.P;
  const double at = ar.radius[t];
  const double ctx = a.centres4[4 * t], cty = a.centres4[4 * t + 1], ctz = a.centres4[4 * t + 2];
  double ox = 0, oy = 0, oz = 0;
  if (active) {
    ox = at * a.otab[4 * g];
    oy = at * a.otab[4 * g + 1];
    oz = at * a.otab[4 * g + 2];
  }
  const NearK k{a.p, a.mmax, nc, kc, kc + 33, kc + 66, kc + 99};
  double acc0 = 0, acc1 = 0, acc2 = 0;
  for (int e = s0; e < s1; ++e) {
    const int s = a.near_idx[e];
    const double as = ar.radius[s];
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * nc; i += blockDim.x) cs[i] = a.coef[(size_t)s * 6 * nc + i];
    for (int n = threadIdx.x; n <= a.p; n += blockDim.x) {
      kc[n] = fma(as, ar.sv[n], a.kvv[n]);
      kc[33 + n] = fma(as, ar.sw[n], a.kww[n]);
      kc[66 + n] = fma(as, ar.swv[n], a.kwv[n]);
      kc[99 + n] = fma(as, ar.sx[n], a.kxx[n]);
    }
    __syncthreads();
    if (!active) continue;
    const double ias = 1.0 / as;
    const double dx = ((ctx - a.centres4[4 * s]) + ox) * ias;
    const double dy = ((cty - a.centres4[4 * s + 1]) + oy) * ias;
    const double dz = ((ctz - a.centres4[4 * s + 2]) + oz) * ias;
    exterior_series(k, cs, rec, dx, dy, dz, acc0, acc1, acc2);
  }
  if (active) {
    double* uo = a.u + 3 * ((int64_t)t * a.P + g);
    uo[0] += acc0;
    uo[1] += acc1;
    uo[2] += acc2;
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

void launch_near(bie_ctx* c, const OpSpec& spec, double* u) {
  if (c->near_idx.empty()) return;
  if (c->near_method == 1) {
    launch_near_rot(c, spec, u);
    return;
  }
  NearParams a{};
  a.coef = c->coef.as<double>();
  a.centres4 = c->centres4.as<double>();
  a.near_ptr = c->dnear_ptr.as<int>();
  a.near_idx = c->dnear_idx.as<int>();
  a.otab = c->otab.as<double>();
  a.rec = c->rec.as<double>();
  a.u = u;
  a.p = c->p;
  a.mmax = c->mmax;
  a.P = c->P;
  a.ncoef = c->ncoef;
  const int threads = std::min(1024, ((c->P + 63) / 64) * 64);
  if (c->poly) {
    NearRadParams ar{};
    ar.b = a;
    ar.radius = c->radius_d.as<double>();
    series_radial(0.0, spec.a_d, c->p, ar.b.kvv, ar.b.kww, ar.b.kwv, ar.b.kxx);
    series_radial(spec.a_s, 0.0, c->p, ar.sv, ar.sw, ar.swv, ar.sx);
    const size_t sm = (12 * (size_t)c->ncoef + 4 * 33) * sizeof(double);
    near_kernel_radii<<<dim3((unsigned)c->nb), dim3(threads), sm, c->stream>>>(ar);
    BIE_HIP(hipGetLastError());
    return;
  }
  series_radial(spec.a_s, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);
  const size_t sm = 12 * (size_t)c->ncoef * sizeof(double);
  near_kernel<<<dim3((unsigned)c->nb), dim3(threads), sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
