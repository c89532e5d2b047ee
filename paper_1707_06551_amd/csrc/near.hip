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
  series_radial(spec.a_s, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);
  const int threads = std::min(1024, ((c->P + 63) / 64) * 64);
  const size_t sm = 12 * (size_t)c->ncoef * sizeof(double);
  near_kernel<<<dim3((unsigned)c->nb), dim3(threads), sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
