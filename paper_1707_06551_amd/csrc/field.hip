// Velocity at arbitrary points of the fluid (the representations of Eqs. 5.3, 5.13 and
// 5.18 evaluated off the surfaces; Problem 1 adds the imposed flow).
//
// For a node density mu on the unit spheres, the layer potential a_S S + a_D D (and for
// the completed form the completion flow of Eqs. 5.18-5.19) is evaluated at each target
// point sphere by sphere, with the separation test of Eq. 4.5 measured from the point to
// the surface: |x - c_k| - 1 < d* takes the exterior series of the sphere's VSH
// coefficients (series.h, Eqs. 3.6-3.11), otherwise the smooth quadrature of Eq. 4.4
// over its nodes.  Float64 throughout.  One thread per target; a work-group stages the
// strengths w mu of one source sphere at a time in LDS (broadcast reads) and the
// Legendre recurrence table once.  A point inside or on a sphere gets NaN and raises
// a flag the host turns into BIE_EINVAL.  Spheres of radius a_k: the test reads
// |x - c_k| - a_k < d* a_k, the series is evaluated at (x - c_k)/a_k with its single-layer
// part scaled by a_k (constants staged per sphere), the quadrature uses the nodes
// c_k + a_k o and weights a_k^2 w.
#include "bie_internal.h"
#include "series.h"

namespace bie {

namespace {

struct FieldParams {
  const double* x;         // M x 3 targets
  const double* q;         // N x 4: w mu, w (o . mu)
  const double* otab;      // P x 4 unit offsets
  const double* coef;      // nb x 3 x ncoef x 2
  const double* centres4;  // nb x 4
  const double* moments;   // nb x 6: int mu, int o x mu
  const double* rec;       // ncoef x 6
  double* u;               // M x 3
  int* bad;                // set when a target lies inside or on a sphere
  const double* radius;    // nb radii, or null (unit spheres)
  int64_t M, nb;
  int P, p, mmax, ncoef, completion;
  double near_gap, a_s, a_d;
  double kvv[33], kww[33], kwv[33], kxx[33];  // series constants (double-layer part with radii)
  double sv[33], sw[33], swv[33], sx[33];     // single-layer part, scaled by a_k (radii only)
};

struct FieldK {
  int p, mmax, ncoef;
  const double *kvv, *kww, *kwv, *kxx;
};

__global__ __launch_bounds__(256) void field_kernel(FieldParams a) {
  extern __shared__ __align__(16) double sm[];
  double* qs = sm;                    // P x 4 strengths of the current sphere
  double* rec = sm + 4 * a.P;         // ncoef x 6
  double* kc = rec + 6 * a.ncoef;     // 4 x 33 series constants of the current sphere
  for (int i = threadIdx.x; i < 6 * a.ncoef; i += blockDim.x) rec[i] = a.rec[i];
  const FieldK kk{a.p, a.mmax, a.ncoef, kc, kc + 33, kc + 66, kc + 99};
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < a.M;
  double xx = 0, xy = 0, xz = 0;
  if (valid) {
    xx = a.x[3 * t];
    xy = a.x[3 * t + 1];
    xz = a.x[3 * t + 2];
  }
  const double cS = 1.0 / (8.0 * M_PI), cD = 3.0 / (4.0 * M_PI);
  double ux = 0, uy = 0, uz = 0;
  bool inside = false;
  for (int64_t k = 0; k < a.nb; ++k) {
    const double ak = a.radius ? a.radius[k] : 1.0;
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * a.P; i += blockDim.x) qs[i] = a.q[4 * k * a.P + i];
    for (int n = threadIdx.x; n <= a.p; n += blockDim.x) {
      const bool r = a.radius != nullptr;
      kc[n] = r ? fma(ak, a.sv[n], a.kvv[n]) : a.kvv[n];
      kc[33 + n] = r ? fma(ak, a.sw[n], a.kww[n]) : a.kww[n];
      kc[66 + n] = r ? fma(ak, a.swv[n], a.kwv[n]) : a.kwv[n];
      kc[99 + n] = r ? fma(ak, a.sx[n], a.kxx[n]) : a.kxx[n];
    }
    __syncthreads();
    if (!valid) continue;
    const double dx = xx - a.centres4[4 * k], dy = xy - a.centres4[4 * k + 1], dz = xz - a.centres4[4 * k + 2];
    const double dist = sqrt(dx * dx + dy * dy + dz * dz) - ak;
    if (!(dist > 0.0)) {
      inside = true;
      continue;
    }
    if (dist < a.near_gap * ak) {
      const double iak = 1.0 / ak;
      exterior_series(kk, a.coef + (size_t)k * 6 * a.ncoef, rec, dx * iak, dy * iak, dz * iak, ux, uy, uz);
      continue;
    }
    const double w2 = ak * ak;   // weights a^2 w (strengths q = w mu are per unit sphere)
    double sx = 0, sy = 0, sz = 0;
    for (int i = 0; i < a.P; ++i) {
      const double ox = a.otab[4 * i], oy = a.otab[4 * i + 1], oz = a.otab[4 * i + 2];
      const double* qi0 = qs + 4 * i;
      const double qi[3] = {w2 * qi0[0], w2 * qi0[1], w2 * qi0[2]};
      const double rx = dx - ak * ox, ry = dy - ak * oy, rz = dz - ak * oz;
      const double r2 = rx * rx + ry * ry + rz * rz;
      const double ir = 1.0 / sqrt(r2);
      const double ir2 = ir * ir;
      const double rq = rx * qi[0] + ry * qi[1] + rz * qi[2];
      // S: (q/r + r (r.q)/r^3) / 8pi;  D: 3/(4pi) r (r.q)(r.n)/r^5 with n = o
      const double rn = rx * ox + ry * oy + rz * oz;
      const double c = rq * ir * ir2 * (a.a_s * cS + a.a_d * cD * rn * ir2);
      const double s0 = a.a_s * cS * ir;
      sx += s0 * qi[0] + c * rx;
      sy += s0 * qi[1] + c * ry;
      sz += s0 * qi[2] + c * rz;
    }
    ux += sx;
    uy += sy;
    uz += sz;
  }
  if (!valid) return;
  if (a.completion) {
    for (int64_t k = 0; k < a.nb; ++k) {
      const double* mo = a.moments + 6 * k;
      const double rx = xx - a.centres4[4 * k], ry = xy - a.centres4[4 * k + 1], rz = xz - a.centres4[4 * k + 2];
      const double r2 = rx * rx + ry * ry + rz * rz;
      const double ir = 1.0 / sqrt(r2);
      const double ir3 = ir * ir * ir;
      const double rf = rx * mo[0] + ry * mo[1] + rz * mo[2];
      ux += cS * (mo[0] * ir + rx * rf * ir3 + (mo[4] * rz - mo[5] * ry) * ir3);
      uy += cS * (mo[1] * ir + ry * rf * ir3 + (mo[5] * rx - mo[3] * rz) * ir3);
      uz += cS * (mo[2] * ir + rz * rf * ir3 + (mo[3] * ry - mo[4] * rx) * ir3);
    }
  }
  if (inside) {
    ux = uy = uz = __builtin_nan("");
    *a.bad = 1;
  }
  a.u[3 * t] = ux;
  a.u[3 * t + 1] = uy;
  a.u[3 * t + 2] = uz;
}

}  // namespace

void eval_field(bie_ctx* c, int op_base, const double* mu, int64_t M, const double* x, double* u) {
  if (op_base != BIE_OP_S && op_base != BIE_OP_D && op_base != BIE_OP_SD_BIE && op_base != BIE_OP_DN_BIE)
    throw Error{BIE_EINVAL, "bie_eval_field: op must be BIE_OP_S, BIE_OP_D, BIE_OP_SD_BIE or BIE_OP_DN_BIE"};
  if (M < 0 || (M > 0 && (!x || !u)) || !mu) throw Error{BIE_EINVAL, "bie_eval_field: bad arguments"};
  if (M == 0) return;
  const OpSpec spec = op_spec(op_base);
  // coefficients (series), float64 strengths w mu (quadrature) and moments (completion)
  VshCall v;
  v.mu = mu;
  v.u = nullptr;
  v.write_q = true;
  v.write_coef = true;
  v.want_moments = spec.completion;
  if (c->poly) {
    v.radius = c->radius_d.as<double>();   // moments with a^2, a^3
    v.lam_mode = 1;
  }
  launch_vsh(c, BIE_FP64, v);
  int* bad = reinterpret_cast<int*>(c->scal.as<double>());
  BIE_HIP(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
  FieldParams a{};
  a.x = x;
  a.q = c->q.as<double>();
  a.otab = c->otab.as<double>();
  a.coef = c->coef.as<double>();
  a.centres4 = c->centres4.as<double>();
  a.moments = c->moments.as<double>();
  a.rec = c->rec.as<double>();
  a.u = u;
  a.bad = bad;
  a.M = M;
  a.nb = c->nb;
  a.P = c->P;
  a.p = c->p;
  a.mmax = c->mmax;
  a.ncoef = c->ncoef;
  a.completion = spec.completion ? 1 : 0;
  a.near_gap = c->near_gap;
  a.a_s = spec.a_s;
  a.a_d = spec.a_d;
  a.radius = c->poly ? c->radius_d.as<double>() : nullptr;
  if (c->poly) {
    series_radial(0.0, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);
    series_radial(spec.a_s, 0.0, c->p, a.sv, a.sw, a.swv, a.sx);
  } else {
    series_radial(spec.a_s, spec.a_d, c->p, a.kvv, a.kww, a.kwv, a.kxx);
  }
  const size_t sm = (4 * (size_t)c->P + 6 * (size_t)c->ncoef + 4 * 33) * sizeof(double);
  field_kernel<<<dim3((unsigned)((M + 255) / 256)), dim3(256), sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
  int hbad = 0;
  BIE_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  BIE_HIP(hipStreamSynchronize(c->stream));
  if (hbad) throw Error{BIE_EINVAL, "bie_eval_field: a target point lies inside or on a sphere (its value is NaN)"};
}

}  // namespace bie
