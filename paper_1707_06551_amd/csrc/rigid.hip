// Global rigid-mode coarse correction of the resistance form (no counterpart in the
// paper; an addition to the block preconditioner).
//
// In the completed double-layer form (Eqs. 5.18-5.19) the rigid densities of a sphere
// (W_1 and X_1, the null space of D_+ in Table 3.12) reach the other spheres only through
// the completion flow: a density a + b x x carries the force F = 4 pi a and the torque
// T = 8 pi / 3 b, and the Stokeslet + rotlet they induce decays like 1/r.  Summed over
// thousands of spheres this coupling has a wide spectrum that the sphere-by-sphere
// inverse M0 does not see, and GMRES pays for it in iterations.  The correction solves it
// on the coarse space of six rigid modes per sphere:
//
//   z <- z + P (y - R z),   M (S y) = R r,
//
// R f = (1/4pi int f, 3/8pi int x x f) per sphere (Eq. 4.4 weights), P (a, b) = a + b x x,
// S = diag(4 pi, 8 pi / 3), and M the Rotne-Prager-Yamakawa grand mobility of unit
// spheres (symmetric positive definite for non-overlapping spheres; the operator's own
// rigid-mode restriction differs only by averaging the Stokeslet over one sphere instead
// of two, and is indefinite in dense suspensions).  The coarse system is solved by
// Jacobi-preconditioned conjugate gradients with a matrix-free all-pairs product over the
// sphere centres, in float64, on the device; scalars stay on the device and the host
// reads the residual history every CHECK iterations.
//
// Spheres of radius a_k (rad != null): R f = (int f / (4 pi a^2), 3 int (x - c) x f /
// (8 pi a^4)), P (a, b) = a + b x (x - c), S = diag(4 pi a^2, 8 pi a^4 / 3), and M the
// polydisperse Rotne-Prager-Yamakawa mobility: self blocks 1/(6 pi a), 1/(8 pi a^3), the
// translation-translation pair block with (a_i^2 + a_k^2) in place of 2, the rotation
// blocks unchanged.  Without radii every a is 1 and these are the formulas above.
#include <algorithm>

#include "bie_internal.h"

namespace bie {

namespace {

constexpr int RG_SRC = 256;     // sources per work-group of the mobility product
constexpr int RG_MAXIT = 400;   // conjugate-gradient iterations per coarse solve
constexpr int RG_CHECK = 8;     // iterations between host convergence checks
constexpr double RG_TOL = 1e-7; // relative residual of the coarse solve

__device__ inline double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// 1/sqrt(x): the hardware estimate (5e-8 relative) and one Newton step, y (3 - x y^2) / 2
// (4e-15); a fraction of the instructions of a float64 division and square root.
__device__ inline double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  return fma(0.5 * y, fma(-h, y, 1.0), y);
}

// Block-wide sum of v (256 threads); every thread gets the result.
__device__ inline double block_sum256(double v, double* lds) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  return lds[0] + lds[1] + lds[2] + lds[3];
}

// xi[6k..6k+5] = R f on sphere k; one work-group per sphere.  With unit weights and
// offsets: the mean is (1/4pi) sum w f for any radius, the rotation (3/(8 pi a)) sum w o x f.
__global__ __launch_bounds__(256) void k_rigid_restrict(const double* f, const double* frame, const double* wnode,
                                                       int P, double* xi, const double* rad) {
  __shared__ double lds[4];
  const int64_t k = blockIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int g = threadIdx.x; g < P; g += 256) {
    const double* v = f + 3 * (k * P + g);
    const double* o = frame + 9 * g;   // e_r = unit offset of the node
    const double w = wnode[g];
    acc[0] += w * v[0];
    acc[1] += w * v[1];
    acc[2] += w * v[2];
    acc[3] += w * (o[1] * v[2] - o[2] * v[1]);
    acc[4] += w * (o[2] * v[0] - o[0] * v[2]);
    acc[5] += w * (o[0] * v[1] - o[1] * v[0]);
  }
  const double a = rad ? rad[k] : 1.0;
  for (int d = 0; d < 6; ++d) {
    const double s = block_sum256(acc[d], lds);
    if (threadIdx.x == 0) xi[6 * k + d] = s * (d < 3 ? 1.0 / (4.0 * M_PI) : 3.0 / (8.0 * M_PI * a));
  }
}

// z += P (y - zeta) at every node.
__global__ void k_rigid_prolong(const double* y, const double* zeta, const double* frame, int P, int64_t N,
                                double* z, const double* rad) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / P;
    const int li = (int)(g - k * P);
    const double a = rad ? rad[k] : 1.0;
    const double o[3] = {a * frame[9 * li], a * frame[9 * li + 1], a * frame[9 * li + 2]};   // x - c
    double d[6];
    for (int e = 0; e < 6; ++e) d[e] = y[6 * k + e] - zeta[6 * k + e];
    z[3 * g + 0] += d[0] + (d[4] * o[2] - d[5] * o[1]);
    z[3 * g + 1] += d[1] + (d[5] * o[0] - d[3] * o[2]);
    z[3 * g + 2] += d[2] + (d[3] * o[1] - d[4] * o[0]);
  }
}

// partial[blockIdx.y][i][0..5] = sum over the work-group's sources s of M(i, s) u_s,
// M the Rotne-Prager-Yamakawa mobility (self block included when s = i).  64 targets
// per work-group (one per lane), the four waves take every fourth source.
__global__ __launch_bounds__(256) void k_rpy_matvec(const double* centres4, const double* u, int64_t nb,
                                                   double* partial, const double* rad) {
  __shared__ double sc[RG_SRC][4];   // centre, radius^2
  __shared__ double su[RG_SRC][6];
  __shared__ double red[3][64][6];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t s0 = (int64_t)blockIdx.y * RG_SRC;
  const int ns = (int)min<int64_t>(RG_SRC, nb - s0);
  for (int e = threadIdx.x; e < ns; e += 256) {
    for (int d = 0; d < 3; ++d) sc[e][d] = centres4[4 * (s0 + e) + d];
    const double as = rad ? rad[s0 + e] : 1.0;
    sc[e][3] = as * as;
    for (int d = 0; d < 6; ++d) su[e][d] = u[6 * (s0 + e) + d];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool valid = i < nb;
  const int64_t ii = valid ? i : 0;
  const double cx = centres4[4 * ii], cy = centres4[4 * ii + 1], cz = centres4[4 * ii + 2];
  const double ai = rad ? rad[ii] : 1.0;
  const double k8 = 1.0 / (8.0 * M_PI), k16 = 1.0 / (16.0 * M_PI);
  double a[6] = {0, 0, 0, 0, 0, 0};
  for (int e = wv; e < ns; e += 4) {
    const double Fx = su[e][0], Fy = su[e][1], Fz = su[e][2];
    const double Tx = su[e][3], Ty = su[e][4], Tz = su[e][5];
    if (s0 + e == ii) {
      const double ft = 1.0 / (6.0 * M_PI * ai), fr = k8 / (ai * ai * ai);
      a[0] += Fx * ft;
      a[1] += Fy * ft;
      a[2] += Fz * ft;
      a[3] += Tx * fr;
      a[4] += Ty * fr;
      a[5] += Tz * fr;
      continue;
    }
    const double rx = cx - sc[e][0], ry = cy - sc[e][1], rz = cz - sc[e][2];
    const double d2 = rx * rx + ry * ry + rz * rz;
    const double id = rsqrt_f64(d2);
    const double id2 = id * id, id3 = id2 * id;
    const double rF = rx * Fx + ry * Fy + rz * Fz;
    const double rT = rx * Tx + ry * Ty + rz * Tz;
    // translation: (1/8pi)[(1/d + s/(3d^3)) F + (1/d - s/d^3)(e.F) e - (r x T)/d^3],
    // s = a_i^2 + a_k^2 (2 for unit spheres)
    const double s2 = ai * ai + sc[e][3];
    const double c1 = id + (s2 * (1.0 / 3.0)) * id3;
    const double c2 = (id - s2 * id3) * id2 * rF;
    a[0] += k8 * (c1 * Fx + c2 * rx - id3 * (ry * Tz - rz * Ty));
    a[1] += k8 * (c1 * Fy + c2 * ry - id3 * (rz * Tx - rx * Tz));
    a[2] += k8 * (c1 * Fz + c2 * rz - id3 * (rx * Ty - ry * Tx));
    // rotation: -(1/8pi)(r x F)/d^3 - (1/16pi)(T - 3 (e.T) e)/d^3
    const double c3 = 3.0 * rT * id2;
    a[3] += -k8 * id3 * (ry * Fz - rz * Fy) - k16 * id3 * (Tx - c3 * rx);
    a[4] += -k8 * id3 * (rz * Fx - rx * Fz) - k16 * id3 * (Ty - c3 * ry);
    a[5] += -k8 * id3 * (rx * Fy - ry * Fx) - k16 * id3 * (Tz - c3 * rz);
  }
  if (wv > 0)
    for (int d = 0; d < 6; ++d) red[wv - 1][lane][d] = a[d];
  __syncthreads();
  if (wv == 0 && valid) {
    double* out = partial + ((int64_t)blockIdx.y * nb + i) * 6;
    for (int d = 0; d < 6; ++d) out[d] = ((a[d] + red[0][lane][d]) + red[1][lane][d]) + red[2][lane][d];
  }
}

// Jacobi scaling: diagonal of M^-1 (6 pi a on forces, 8 pi a^3 on torques).
__device__ inline double jacobi(int64_t e, const double* rad) {
  const double a = rad ? rad[e / 6] : 1.0;
  return (e % 6) < 3 ? 6.0 * M_PI * a : 8.0 * M_PI * a * a * a;
}

// CG start: x = 0, r = b, z = D r, p = z; block partial sums of r.z and r.r.
__global__ __launch_bounds__(256) void k_cg_start(const double* b, int64_t n, double* x, double* r, double* z,
                                                 double* p, double* dots, const double* rad) {
  __shared__ double lds[4];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rz = 0, rr = 0;
  if (e < n) {
    const double rv = b[e], zv = jacobi(e, rad) * rv;
    x[e] = 0.0;
    r[e] = rv;
    z[e] = zv;
    p[e] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  const double s1 = block_sum256(rz, lds);
  const double s2 = block_sum256(rr, lds);
  if (threadIdx.x == 0) {
    dots[2 * blockIdx.x] = s1;
    dots[2 * blockIdx.x + 1] = s2;
  }
}

// Sum of nblk block partials (pairs), computed identically by every work-group.
__device__ inline void sum_pairs(const double* dots, int nblk, double* lds, double& s1, double& s2) {
  double a = 0, b = 0;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    a += dots[2 * k];
    b += dots[2 * k + 1];
  }
  s1 = block_sum256(a, lds);
  s2 = block_sum256(b, lds);
}

// Records the start residual: hist[0] = r.z, hist[1] = r.r.
__global__ __launch_bounds__(256) void k_cg_record(const double* dots, int nblk, double* hist) {
  __shared__ double lds[4];
  double s1, s2;
  sum_pairs(dots, nblk, lds, s1, s2);
  if (threadIdx.x == 0) {
    hist[0] = s1;
    hist[1] = s2;
  }
}

// q = sum of the split partials; block partial sums of p.q.
__global__ __launch_bounds__(256) void k_cg_q(const double* partial, int nsplit, int64_t n, const double* p, double* q,
                                             double* dots) {
  __shared__ double lds[4];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double pq = 0;
  if (e < n) {
    double s = 0;
    for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)k * n + e];
    q[e] = s;
    pq = p[e] * s;
  }
  const double t = block_sum256(pq, lds);
  if (threadIdx.x == 0) {
    dots[2 * blockIdx.x] = t;
    dots[2 * blockIdx.x + 1] = 0.0;
  }
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = D r; block partials of r.z, r.r.
__global__ __launch_bounds__(256) void k_cg_xr(const double* dots_pq, int nblk, const double* hist, int it, int64_t n,
                                              const double* p, const double* q, double* x, double* r, double* z,
                                              double* dots, const double* rad) {
  __shared__ double lds[4];
  double pq, unused;
  sum_pairs(dots_pq, nblk, lds, pq, unused);
  const double alpha = pq != 0.0 ? hist[2 * it] / pq : 0.0;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double rz = 0, rr = 0;
  if (e < n) {
    x[e] += alpha * p[e];
    const double rv = r[e] - alpha * q[e];
    const double zv = jacobi(e, rad) * rv;
    r[e] = rv;
    z[e] = zv;
    rz = rv * zv;
    rr = rv * rv;
  }
  const double s1 = block_sum256(rz, lds);
  const double s2 = block_sum256(rr, lds);
  if (threadIdx.x == 0) {
    dots[2 * blockIdx.x] = s1;
    dots[2 * blockIdx.x + 1] = s2;
  }
}

// beta = rz_new / rz_old; p = z + beta p; hist[2(it+1)] = rz_new, hist[2(it+1)+1] = r.r.
__global__ __launch_bounds__(256) void k_cg_p(const double* dots, int nblk, double* hist, int it, int64_t n,
                                             const double* z, double* p) {
  __shared__ double lds[4];
  double rz, rr;
  sum_pairs(dots, nblk, lds, rz, rr);
  const double old = hist[2 * it];
  const double beta = old != 0.0 ? rz / old : 0.0;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = z[e] + beta * p[e];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hist[2 * (it + 1)] = rz;
    hist[2 * (it + 1) + 1] = rr;
  }
}

// y = S^-1 x: forces -> a = F / (4 pi a^2), torques -> b = 3 T / (8 pi a^4).
__global__ void k_unscale(const double* x, int64_t n, double* y, const double* rad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    const double a = rad ? rad[e / 6] : 1.0;
    const double a2 = a * a;
    y[e] = x[e] * ((e % 6) < 3 ? 1.0 / (4.0 * M_PI * a2) : 3.0 / (8.0 * M_PI * a2 * a2));
  }
}

}  // namespace

void rigid_restrict(bie_ctx* c, const double* f, double* xi) {
  k_rigid_restrict<<<dim3((unsigned)c->nb), dim3(256), 0, c->stream>>>(
      f, c->frame.as<double>(), c->wnode.as<double>(), c->P, xi, c->poly ? c->radius_d.as<double>() : nullptr);
  BIE_HIP(hipGetLastError());
}

void rigid_correct(bie_ctx* c, const double* r, double* z) {
  const int64_t nb = c->nb, n = 6 * nb;
  if (nb > RIGID_MAX_SPHERES) throw Error{BIE_EINVAL, "BIE_PC_RIGID: too many spheres for the coarse solve"};
  const int nsplit = (int)((nb + RG_SRC - 1) / RG_SRC);
  const int nblk = (int)((n + 255) / 256);
  if (!c->rg_vec.ptr) {
    c->rg_vec.alloc(sizeof(double) * 8 * n);
    c->rg_partial.alloc(sizeof(double) * (size_t)nsplit * n);
    c->rg_dots.alloc(sizeof(double) * 4 * (size_t)nblk);
    c->rg_hist.alloc(sizeof(double) * 2 * (RG_MAXIT + 2));
  }
  double* xi = c->rg_vec.as<double>();
  double* zeta = xi + n;
  double* x = xi + 2 * n;
  double* rr = xi + 3 * n;
  double* zz = xi + 4 * n;
  double* pp = xi + 5 * n;
  double* qq = xi + 6 * n;
  double* y = xi + 7 * n;
  double* dots = c->rg_dots.as<double>();
  double* dots2 = dots + 2 * nblk;
  double* hist = c->rg_hist.as<double>();
  const double* frame = c->frame.as<double>();
  const double* wnode = c->wnode.as<double>();
  hipStream_t st = c->stream;

  const double* rad = c->poly ? c->radius_d.as<double>() : nullptr;
  k_rigid_restrict<<<dim3((unsigned)nb), dim3(256), 0, st>>>(r, frame, wnode, c->P, xi, rad);
  k_rigid_restrict<<<dim3((unsigned)nb), dim3(256), 0, st>>>(z, frame, wnode, c->P, zeta, rad);
  k_cg_start<<<dim3(nblk), dim3(256), 0, st>>>(xi, n, x, rr, zz, pp, dots, rad);
  k_cg_record<<<dim3(1), dim3(256), 0, st>>>(dots, nblk, hist);
  BIE_HIP(hipGetLastError());
  double h0[2];
  BIE_HIP(hipMemcpyAsync(h0, hist, sizeof(h0), hipMemcpyDeviceToHost, st));
  BIE_HIP(hipStreamSynchronize(st));
  const double stop = RG_TOL * RG_TOL * h0[1];
  int it = 0;
  if (h0[1] > 0.0) {
    while (it < RG_MAXIT) {
      const int upto = std::min(RG_MAXIT, it + RG_CHECK);
      for (; it < upto; ++it) {
        k_rpy_matvec<<<dim3((unsigned)((nb + 63) / 64), (unsigned)nsplit), dim3(256), 0, st>>>(
            c->centres4.as<double>(), pp, nb, c->rg_partial.as<double>(), rad);
        k_cg_q<<<dim3(nblk), dim3(256), 0, st>>>(c->rg_partial.as<double>(), nsplit, n, pp, qq, dots);
        k_cg_xr<<<dim3(nblk), dim3(256), 0, st>>>(dots, nblk, hist, it, n, pp, qq, x, rr, zz, dots2, rad);
        k_cg_p<<<dim3(nblk), dim3(256), 0, st>>>(dots2, nblk, hist, it, n, zz, pp);
      }
      BIE_HIP(hipGetLastError());
      double hr;
      BIE_HIP(hipMemcpyAsync(&hr, hist + 2 * it + 1, sizeof(double), hipMemcpyDeviceToHost, st));
      BIE_HIP(hipStreamSynchronize(st));
      if (!(hr == hr)) throw Error{BIE_EDEVICE, "BIE_PC_RIGID: non-finite coarse residual"};
      if (hr <= stop) break;
    }
  }
  c->rg_last_iters = it;
  k_unscale<<<dim3(nblk), dim3(256), 0, st>>>(x, n, y, rad);
  const int64_t N = c->N;
  const int pblocks = (int)std::min<int64_t>((N + 255) / 256, 8192);
  k_rigid_prolong<<<dim3(pblocks), dim3(256), 0, st>>>(y, zeta, frame, c->P, N, z, rad);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
