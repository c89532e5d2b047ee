// Laplace single layer on the unit spheres (Section 3.1, Theorem 1, Eq. 3.3) and the
// magnetostatic problem of Problem 3 (Eqs. 5.9-5.13), float64.
//
// Evaluation follows the Stokes operators: the own sphere through its scalar spherical
// harmonic coefficients (Theorem 1: S^L[Y_n^m] = Y_n^m / (2n+1); the normal derivative
// K^L has principal value -1 / (2(2n+1)); the exterior gradient of the own layer is
// sum c V_n^m / (2n+1)), near spheres (surface gap < d*) through the exterior series of
// Eq. 3.3 and its gradient (series.h), the others through the smooth quadrature of Eq.
// 4.4 with the kernels 1 / (4 pi r) and -r / (4 pi r^3).
//
// Problem 3: (1/2 I + eta K^L)[q] = eta H0 . n on all surfaces (Eq. 5.13) is solved by
// the library's GMRES; H = H0 - grad S^L[q] on the fluid side; the Maxwell traction
// t = (H . n) H - |H|^2 n / 2 (mu0 = 1) gives each sphere's force int t and torque
// int (x - c) x t, the loads through which the field moves the particles.
//
// Spheres of radius a: S^L of a sphere of radius a is a times the unit-sphere layer at
// (x - c)/a, so its gradient and K^L are scale-free.  The own-sphere terms (K_pv, the
// gradient, the block inverse) are unchanged; near and far sources are evaluated at the
// target node written in units of the source radius, (c_t + a_t o - c_s)/a_s, with the
// unit-sphere series and quadrature; force and torque carry a^2 (area) and a^3 (area
// and lever arm).
#include <algorithm>

#include "bie_internal.h"
#include "series.h"

namespace bie {

namespace {

__device__ inline double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct SelfParams {
  const double* f;       // N scalar input
  double* out;           // N: c_id f + scale * sum lam_n c Y   (or nullptr)
  double* grad;          // N x 3: sum c V_n^m / (2n+1)        (or nullptr)
  double* coef;          // nb x ncoef x 2 scalar coefficients (or nullptr)
  const double* dft;     // (mmax+1) x nphi x 2
  const double* leg;     // 3 x ncoef x nlat: Pbar, dPbar/dtheta, m Pbar / sin
  const double* wlat;    // nlat
  const double* frame;   // P x 9
  const int* modes;      // ncoef x 2 (m, n)
  int p, nphi, mmax, P, ncoef, nlat;
  double c_id, scale;
  double lam[33];
};

// One work-group per sphere: scalar transform (real DFT per latitude, Legendre
// projection with the Eq. 4.4 weights), multipliers per degree, synthesis.
__global__ __launch_bounds__(256) void lap_self_kernel(SelfParams a) {
  extern __shared__ __align__(16) double sm[];
  const int k = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int P = a.P, nphi = a.nphi, nl = a.nlat, M1 = a.mmax + 1, nc = a.ncoef;
  double* fs = sm;                  // P
  double* F = fs + P;               // nl x M1 x 2
  double* C = F + 2 * nl * M1;      // nc x 2
  double* G = C + 2 * nc;           // 3 x nl x M1 x 2 (synthesis in the latitude / order domain)
  const int64_t base = (int64_t)k * P;
  for (int g = tid; g < P; g += nt) fs[g] = a.f[base + g];
  __syncthreads();
  for (int e = tid; e < nl * M1; e += nt) {
    const int j = e / M1, m = e - j * M1;
    const double* tw = a.dft + (size_t)m * nphi * 2;
    double re = 0, im = 0;
    for (int l = 0; l < nphi; ++l) {
      re += fs[j * nphi + l] * tw[2 * l];
      im -= fs[j * nphi + l] * tw[2 * l + 1];
    }
    F[2 * e] = re;
    F[2 * e + 1] = im;
  }
  __syncthreads();
  for (int i = tid; i < nc; i += nt) {
    const int m = a.modes[2 * i];
    const double* Lp = a.leg + (size_t)i * nl;
    double re = 0, im = 0;
    for (int j = 0; j < nl; ++j) {
      const double w = a.wlat[j] * Lp[j];
      re += w * F[2 * (j * M1 + m)];
      im += w * F[2 * (j * M1 + m) + 1];
    }
    C[2 * i] = re;
    C[2 * i + 1] = im;
    if (a.coef) {
      a.coef[2 * ((size_t)k * nc + i)] = re;
      a.coef[2 * ((size_t)k * nc + i) + 1] = im;
    }
  }
  __syncthreads();
  if (!a.out && !a.grad) return;
  // latitude / order domain: value with lam_n; gradient components r, theta, phi
  for (int e = tid; e < nl * M1; e += nt) {
    const int j = e / M1, m = e - j * M1;
    const int off = m * (a.p + 1) - (m * (m - 1)) / 2;
    double vr = 0, vi = 0, rr = 0, ri = 0, tr = 0, ti = 0, pr = 0, pi = 0;
    for (int n = m; n <= a.p; ++n) {
      const int i = off + (n - m);
      const double lp = a.leg[((size_t)0 * nc + i) * nl + j];
      const double ld = a.leg[((size_t)1 * nc + i) * nl + j];
      const double lq = a.leg[((size_t)2 * nc + i) * nl + j];
      const double cr = C[2 * i], ci = C[2 * i + 1];
      vr += a.lam[n] * cr * lp;
      vi += a.lam[n] * ci * lp;
      const double g = 1.0 / (2 * n + 1.0);
      rr -= (n + 1.0) * g * cr * lp;
      ri -= (n + 1.0) * g * ci * lp;
      tr += g * cr * ld;
      ti += g * ci * ld;
      // (i m / sin) Y: i (m Pbar / sin) c
      pr -= g * lq * ci;
      pi += g * lq * cr;
    }
    double* Ge = G + 2 * e;
    const int S = 2 * nl * M1;
    Ge[0] = vr;
    Ge[1] = vi;
    Ge[S] = rr;
    Ge[S + 1] = ri;
    Ge[2 * S] = tr;
    Ge[2 * S + 1] = ti;
    Ge[3 * S] = pr;
    Ge[3 * S + 1] = pi;
  }
  __syncthreads();
  const int S = 2 * nl * M1;
  const double* tw1 = a.dft + 2 * nphi;  // order 1: cos, sin of 2 pi idx / n_phi
  for (int g = tid; g < P; g += nt) {
    const int j = g / nphi, l = g - j * nphi;
    double s[4];
    for (int c = 0; c < 4; ++c) {
      const double* Gc = G + c * S + 2 * j * M1;
      double acc = Gc[0];
      double acc2 = 0;
      for (int m = 1; m < M1; ++m) {
        const int idx = (m * l) % nphi;
        acc2 += Gc[2 * m] * tw1[2 * idx] - Gc[2 * m + 1] * tw1[2 * idx + 1];
      }
      s[c] = acc + 2 * acc2;
    }
    if (a.out) a.out[base + g] = a.c_id * fs[g] + a.scale * s[0];
    if (a.grad) {
      const double* fr = a.frame + 9 * g;
      for (int d = 0; d < 3; ++d) a.grad[3 * (base + g) + d] = s[1] * fr[d] + s[2] * fr[3 + d] + s[3] * fr[6 + d];
    }
  }
}

struct NearLapParams {
  const double* coef;      // nb x ncoef x 2
  const double* centres4;
  const int* near_ptr;
  const int* near_idx;
  const double* otab;      // P x 4
  const double* rec;       // ncoef x 6
  const double* radius;    // nb radii, or nullptr for unit spheres
  double* out;             // N: += scale * n . grad  (or nullptr)
  double* grad;            // N x 3: += grad          (or nullptr)
  int p, mmax, P, ncoef;
  double scale;
};

// One work-group per target sphere, one thread per node; the near sources' coefficients
// are staged in LDS one source at a time.
__global__ __launch_bounds__(1024) void lap_near_kernel(NearLapParams a) {
  extern __shared__ __align__(16) double sm[];
  const int t = blockIdx.x;
  const int s0 = a.near_ptr[t], s1 = a.near_ptr[t + 1];
  if (s0 == s1) return;
  const int nc = a.ncoef;
  double* cs = sm;
  double* rec = sm + 2 * nc;
  for (int i = threadIdx.x; i < 6 * nc; i += blockDim.x) rec[i] = a.rec[i];
  const double ctx = a.centres4[4 * t], cty = a.centres4[4 * t + 1], ctz = a.centres4[4 * t + 2];
  const double at = a.radius ? a.radius[t] : 1.0;
  // the target nodes in chunks of the block size (grids with more than 1024 nodes)
  for (int g0 = 0; g0 < a.P; g0 += blockDim.x) {
    const int g = g0 + threadIdx.x;
    const bool active = g < a.P;
    double ox = 0, oy = 0, oz = 0;
    if (active) {
      ox = a.otab[4 * g];
      oy = a.otab[4 * g + 1];
      oz = a.otab[4 * g + 2];
    }
    double v = 0, gx = 0, gy = 0, gz = 0;
    for (int e = s0; e < s1; ++e) {
      const int s = a.near_idx[e];
      __syncthreads();
      for (int i = threadIdx.x; i < 2 * nc; i += blockDim.x) cs[i] = a.coef[(size_t)s * 2 * nc + i];
      __syncthreads();
      if (!active) continue;
      const double ias = a.radius ? 1.0 / a.radius[s] : 1.0;
      laplace_series(a.p, a.mmax, cs, rec, ((ctx - a.centres4[4 * s]) + at * ox) * ias,
                     ((cty - a.centres4[4 * s + 1]) + at * oy) * ias, ((ctz - a.centres4[4 * s + 2]) + at * oz) * ias,
                     v, gx, gy, gz);
    }
    if (!active) continue;
    const int64_t node = (int64_t)t * a.P + g;
    if (a.out) a.out[node] += a.scale * (gx * ox + gy * oy + gz * oz);
    if (a.grad) {
      a.grad[3 * node] += gx;
      a.grad[3 * node + 1] += gy;
      a.grad[3 * node + 2] += gz;
    }
  }
}

struct FarLapParams {
  const double* f;         // N scalar density
  const double* wnode;     // P
  const double* otab;      // P x 4
  const double* centres4;
  const uint32_t* excl;    // nb x nwords
  const double* radius;    // nb radii, or nullptr for unit spheres
  double* out;             // N: += scale * n . grad   (or nullptr)
  double* grad;            // N x 3: += grad           (or nullptr)
  int64_t N, nb;
  int P, nwords;
  double scale;
};

// Smooth quadrature of grad S^L over every well-separated sphere (Eq. 4.4): one thread
// per target node, the strengths w q of one source sphere at a time in LDS.
__global__ __launch_bounds__(256) void lap_far_kernel(FarLapParams a) {
  extern __shared__ __align__(16) double sm[];
  double* qs = sm;   // P
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = x < a.N;
  const int64_t xx = valid ? x : 0;
  const int t = (int)(xx / a.P);
  const int li = (int)(xx - (int64_t)t * a.P);
  const double ox = a.otab[4 * li], oy = a.otab[4 * li + 1], oz = a.otab[4 * li + 2];
  const double at = a.radius ? a.radius[t] : 1.0;
  double gx = 0, gy = 0, gz = 0;
  for (int64_t s = 0; s < a.nb; ++s) {
    __syncthreads();
    for (int i = threadIdx.x; i < a.P; i += 256) qs[i] = a.f[s * a.P + i] * a.wnode[i];
    __syncthreads();
    const bool skip = !valid || ((a.excl[(int64_t)t * a.nwords + (s >> 5)] >> (s & 31)) & 1u);
    if (__any(skip ? 0 : 1) == 0) continue;
    if (skip) continue;
    // in units of the source radius (grad S^L is scale-free)
    const double ias = a.radius ? 1.0 / a.radius[s] : 1.0;
    const double px = ((a.centres4[4 * t] - a.centres4[4 * s]) + at * ox) * ias;
    const double py = ((a.centres4[4 * t + 1] - a.centres4[4 * s + 1]) + at * oy) * ias;
    const double pz = ((a.centres4[4 * t + 2] - a.centres4[4 * s + 2]) + at * oz) * ias;
    double sx = 0, sy = 0, sz = 0;
    for (int i = 0; i < a.P; ++i) {
      const double rx = px - a.otab[4 * i], ry = py - a.otab[4 * i + 1], rz = pz - a.otab[4 * i + 2];
      const double r2 = rx * rx + ry * ry + rz * rz;
      const double ir = 1.0 / sqrt(r2);
      const double c = qs[i] * ir * ir * ir;
      sx += c * rx;
      sy += c * ry;
      sz += c * rz;
    }
    gx -= sx;
    gy -= sy;
    gz -= sz;
  }
  if (!valid) return;
  const double k = 1.0 / (4.0 * M_PI);
  gx *= k;
  gy *= k;
  gz *= k;
  if (a.out) a.out[x] += a.scale * (gx * ox + gy * oy + gz * oz);
  if (a.grad) {
    a.grad[3 * x] += gx;
    a.grad[3 * x + 1] += gy;
    a.grad[3 * x + 2] += gz;
  }
}

// b = eta H0 . n at every node
__global__ void lap_rhs_kernel(const double* otab, int P, int64_t N, double hx, double hy, double hz, double* b) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int li = (int)(g % P);
    b[g] = hx * otab[4 * li] + hy * otab[4 * li + 1] + hz * otab[4 * li + 2];
  }
}

// Maxwell traction of H = H0 - grad on each sphere; force and torque (nb x 6); a sphere
// of radius a: area element a^2, lever arm a n.
__global__ __launch_bounds__(256) void lap_force_kernel(const double* grad, const double* otab, const double* wnode,
                                                        const double* radius, int P, double hx, double hy, double hz,
                                                        double* ft) {
  __shared__ double red[4];
  const int64_t k = blockIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int g = threadIdx.x; g < P; g += 256) {
    const double* gr = grad + 3 * (k * P + g);
    const double Hx = hx - gr[0], Hy = hy - gr[1], Hz = hz - gr[2];
    const double nx = otab[4 * g], ny = otab[4 * g + 1], nz = otab[4 * g + 2];
    const double Hn = Hx * nx + Hy * ny + Hz * nz;
    const double H2 = 0.5 * (Hx * Hx + Hy * Hy + Hz * Hz);
    const double w = wnode[g];
    const double tx = w * (Hn * Hx - H2 * nx), ty = w * (Hn * Hy - H2 * ny), tz = w * (Hn * Hz - H2 * nz);
    acc[0] += tx;
    acc[1] += ty;
    acc[2] += tz;
    acc[3] += ny * tz - nz * ty;
    acc[4] += nz * tx - nx * tz;
    acc[5] += nx * ty - ny * tx;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double rk = radius ? radius[k] : 1.0;
  for (int d = 0; d < 6; ++d) {
    const double v = wsum(acc[d]);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) ft[6 * k + d] = (d < 3 ? rk * rk : rk * rk * rk) * (red[0] + red[1] + red[2] + red[3]);
  }
}

void launch_self(bie_ctx* c, const double* f, double* out, double* grad, double c_id, double scale,
                 const double lam[33]) {
  SelfParams a{};
  a.f = f;
  a.out = out;
  a.grad = grad;
  a.coef = c->lapcoef.as<double>();
  a.dft = c->dft.as<double>();
  a.leg = c->leg.as<double>();
  a.wlat = c->wlat_d.as<double>();
  a.frame = c->frame.as<double>();
  a.modes = c->modes.as<int>();
  a.p = c->p;
  a.nphi = c->n_phi;
  a.mmax = c->mmax;
  a.P = c->P;
  a.ncoef = c->ncoef;
  a.nlat = c->nlat;
  a.c_id = c_id;
  a.scale = scale;
  for (int n = 0; n < 33; ++n) a.lam[n] = lam ? lam[n] : 0.0;
  const size_t sm = sizeof(double) * ((size_t)c->P + 2 * (size_t)c->nlat * (c->mmax + 1) + 2 * (size_t)c->ncoef +
                                      8 * (size_t)c->nlat * (c->mmax + 1));
  lap_self_kernel<<<dim3((unsigned)c->nb), dim3(256), sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

// near and far parts (coefficients in c->lapcoef must be current)
void launch_others(bie_ctx* c, const double* f, double* out, double* grad, double scale) {
  if (!c->near_idx.empty()) {
    NearLapParams a{};
    a.coef = c->lapcoef.as<double>();
    a.centres4 = c->centres4.as<double>();
    a.near_ptr = c->dnear_ptr.as<int>();
    a.near_idx = c->dnear_idx.as<int>();
    a.otab = c->otab.as<double>();
    a.rec = c->rec.as<double>();
    a.radius = c->poly ? c->radius_d.as<double>() : nullptr;
    a.out = out;
    a.grad = grad;
    a.p = c->p;
    a.mmax = c->mmax;
    a.P = c->P;
    a.ncoef = c->ncoef;
    a.scale = scale;
    const int threads = std::min(1024, ((c->P + 63) / 64) * 64);
    lap_near_kernel<<<dim3((unsigned)c->nb), dim3(threads), 8 * sizeof(double) * (size_t)c->ncoef, c->stream>>>(a);
    BIE_HIP(hipGetLastError());
  }
  FarLapParams b{};
  b.f = f;
  b.wnode = c->wnode.as<double>();
  b.otab = c->otab.as<double>();
  b.centres4 = c->centres4.as<double>();
  b.excl = c->excl.as<uint32_t>();
  b.radius = c->poly ? c->radius_d.as<double>() : nullptr;
  b.out = out;
  b.grad = grad;
  b.N = c->N;
  b.nb = c->nb;
  b.P = c->P;
  b.nwords = c->nwords;
  b.scale = scale;
  lap_far_kernel<<<dim3((unsigned)((c->N + 255) / 256)), dim3(256), sizeof(double) * (size_t)c->P, c->stream>>>(b);
  BIE_HIP(hipGetLastError());
}

void ensure_lap(bie_ctx* c) {
  if (!c->lapcoef.ptr) c->lapcoef.alloc((size_t)c->nb * c->ncoef * 2 * sizeof(double));
}

}  // namespace

// out = (1/2 I + eta K^L)[q] (Eq. 5.13), with eta = c->lap_eta
void lap_apply(bie_ctx* c, const double* q, double* out) {
  ensure_lap(c);
  double lam[33];
  for (int n = 0; n < 33; ++n) lam[n] = -0.5 / (2.0 * n + 1.0);   // K_pv on the own surface
  launch_self(c, q, out, nullptr, 0.5, c->lap_eta, lam);
  launch_others(c, q, out, nullptr, c->lap_eta);
}

// z = M0 r: per degree 1 / (1/2 + eta K_pv) on the band-limited part, 2 on the rest
void lap_precond(bie_ctx* c, const double* r, double* z) {
  ensure_lap(c);
  double lam[33];
  for (int n = 0; n < 33; ++n) lam[n] = 1.0 / (0.5 - c->lap_eta * 0.5 / (2.0 * n + 1.0)) - 2.0;
  launch_self(c, r, z, nullptr, 2.0, 1.0, lam);
}

// grad = exterior gradient of S^L[q] at every node (N x 3)
void lap_grad(bie_ctx* c, const double* q, double* grad) {
  ensure_lap(c);
  launch_self(c, q, nullptr, grad, 0.0, 0.0, nullptr);
  launch_others(c, q, nullptr, grad, 0.0);
}

void solve_magnetic(bie_ctx* c, const double H0[3], double eta, const bie_solve_opts* opts, double* q_dev,
                    double* ft_host, bie_solve_info* info, int* rc) {
  if (!(eta > -1.0 && eta < 1.0)) throw Error{BIE_EINVAL, "eta = (mu - mu0) / (mu + mu0) must lie in (-1, 1)"};
  ensure_lap(c);
  c->lap_eta = eta;
  const int64_t N = c->N;
  DevBuf b, grad, ft;
  b.alloc(N * sizeof(double));
  grad.alloc(3 * N * sizeof(double));
  ft.alloc(6 * c->nb * sizeof(double));
  const int blocks = (int)std::min<int64_t>((N + 255) / 256, 8192);
  lap_rhs_kernel<<<dim3(blocks), dim3(256), 0, c->stream>>>(c->otab.as<double>(), c->P, N, eta * H0[0], eta * H0[1],
                                                          eta * H0[2], b.as<double>());
  BIE_HIP(hipGetLastError());
  bie_solve_opts o = opts ? *opts : bie_solve_opts{};
  o.precision = BIE_FP64;  // the Laplace operators run in float64 only
  o.precond &= ~BIE_PC_RIGID;
  if (o.precond == BIE_PC_MLP) o.precond = BIE_PC_M0;
  *rc = solve(c, OP_LAPLACE, b.as<double>(), q_dev, N, &o, info);
  lap_grad(c, q_dev, grad.as<double>());
  lap_force_kernel<<<dim3((unsigned)c->nb), dim3(256), 0, c->stream>>>(
      grad.as<double>(), c->otab.as<double>(), c->wnode.as<double>(), c->poly ? c->radius_d.as<double>() : nullptr,
      c->P, H0[0], H0[1], H0[2], ft.as<double>());
  BIE_HIP(hipGetLastError());
  BIE_HIP(hipMemcpyAsync(ft_host, ft.ptr, 6 * c->nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  BIE_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace bie
