// Learned close-pair coarse correction: low-mode restriction / prolongation, pair
// geometry (features and pair frames), and the block apply used inside the solver.
//
// Coarse space per sphere: vector harmonics of degree <= 2 (Definition 2.2) in the
// Cartesian parametrisation (s; a; b; c; tV; tW; tX) = 25 coefficients:
//   s x,  a - 3 (a.x) x,  b,  c x x,  2 T x - 5 (x.T x) x,  2 T x,  2 x x (T x),
// T = sum_k t_k E_k over Frobenius-orthonormal symmetric traceless E (xy, yz, xz,
// xx - yy, 2zz - xx - yy).  R = weighted projection (Eq. 4.4 weights), P = synthesis.
// A directed near pair (i, j) has the frame Q (rows e1, e2, d; d = (c_j - c_i)/|.|);
// coefficients rotate as (s, Q a, Q b, Q c, D2 tV, D2 tW, D2 tX), D2_kl = tr(E_k Q E_l Q^T).
// The correction zeta_i = sum_j rot^T [K_off(theta_ij) rot rho_j + K_self(theta_ij) rot rho_i]
// with K(theta) commuting with rotations about the pair axis (139 parameters).
#include <algorithm>
#include <cmath>
#include <vector>

#include "bie_internal.h"
#include "coarse.h"

namespace bie {

static const double kS2 = 0.70710678118654752440, kS6 = 0.40824829046386301637;
static const double kE[5][3][3] = {
    {{0, kS2, 0}, {kS2, 0, 0}, {0, 0, 0}},
    {{0, 0, 0}, {0, 0, kS2}, {0, kS2, 0}},
    {{0, 0, kS2}, {0, 0, 0}, {kS2, 0, 0}},
    {{kS2, 0, 0}, {0, -kS2, 0}, {0, 0, 0}},
    {{-kS6, 0, 0}, {0, -kS6, 0}, {0, 0, 2 * kS6}},
};

// The 25 basis fields at unit normal x -> F[25][3].
void lowmode_fields_at(const double x[3], double F[25][3]) {
  for (int k = 0; k < 25; ++k) F[k][0] = F[k][1] = F[k][2] = 0.0;
  for (int d = 0; d < 3; ++d) F[kIS][d] = x[d];
  for (int k = 0; k < 3; ++k) {
    for (int d = 0; d < 3; ++d) {
      const double e = (d == k) ? 1.0 : 0.0;
      F[kIA + k][d] = e - 3.0 * x[k] * x[d];
      F[kIB + k][d] = e;
    }
    // e_k x x
    const double e[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
    F[kIC + k][0] = e[1] * x[2] - e[2] * x[1];
    F[kIC + k][1] = e[2] * x[0] - e[0] * x[2];
    F[kIC + k][2] = e[0] * x[1] - e[1] * x[0];
  }
  for (int k = 0; k < 5; ++k) {
    double Tx[3];
    for (int r = 0; r < 3; ++r) Tx[r] = kE[k][r][0] * x[0] + kE[k][r][1] * x[1] + kE[k][r][2] * x[2];
    const double xTx = x[0] * Tx[0] + x[1] * Tx[1] + x[2] * Tx[2];
    for (int d = 0; d < 3; ++d) {
      F[kITW + k][d] = 2.0 * Tx[d];
      F[kITV + k][d] = 2.0 * Tx[d] - 5.0 * xTx * x[d];
    }
    F[kITX + k][0] = 2.0 * (x[1] * Tx[2] - x[2] * Tx[1]);
    F[kITX + k][1] = 2.0 * (x[2] * Tx[0] - x[0] * Tx[2]);
    F[kITX + k][2] = 2.0 * (x[0] * Tx[1] - x[1] * Tx[0]);
  }
}

void pair_frame(const double d_in[3], double Q[9]) {
  const double n = std::sqrt(d_in[0] * d_in[0] + d_in[1] * d_in[1] + d_in[2] * d_in[2]);
  const double d[3] = {d_in[0] / n, d_in[1] / n, d_in[2] / n};
  int k = 0;
  for (int i = 1; i < 3; ++i)
    if (std::fabs(d[i]) < std::fabs(d[k])) k = i;
  double a[3] = {0, 0, 0};
  a[k] = 1.0;
  double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
  const double m = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (double& v : e1) v /= m;
  const double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
  for (int c = 0; c < 3; ++c) {
    Q[c] = e1[c];
    Q[3 + c] = e2[c];
    Q[6 + c] = d[c];
  }
}

// frame = Q (9, row-major) then D2 (25, row-major)
void frame_of(const double Q[9], double frame[kFrame]) {
  for (int i = 0; i < 9; ++i) frame[i] = Q[i];
  for (int k = 0; k < 5; ++k)
    for (int l = 0; l < 5; ++l) {
      // tr(E_k Q E_l Q^T) = sum E_k[a][b] (Q E_l Q^T)[b][a]
      double s = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double qeq = 0.0;
          for (int c = 0; c < 3; ++c)
            for (int e = 0; e < 3; ++e) qeq += Q[3 * b + c] * kE[l][c][e] * Q[3 * a + e];
          s += kE[k][a][b] * qeq;
        }
      frame[9 + 5 * k + l] = s;
    }
}

void build_coarse(bie_ctx* c) {
  const int P = c->P;
  std::vector<double> F((size_t)P * 75), nrm(25, 0.0);
  for (int j = 0; j < c->nlat; ++j) {
    const double tj = c->t[j], sj = std::sqrt(std::max(0.0, 1.0 - tj * tj));
    for (int l = 0; l < c->n_phi; ++l) {
      const int g = j * c->n_phi + l;
      const double x[3] = {sj * std::cos(c->phi[l]), sj * std::sin(c->phi[l]), tj};
      double Fg[25][3];
      lowmode_fields_at(x, Fg);
      for (int k = 0; k < 25; ++k)
        for (int d = 0; d < 3; ++d) {
          F[(size_t)g * 75 + 3 * k + d] = Fg[k][d];
          nrm[k] += c->wlat[j] * Fg[k][d] * Fg[k][d];
        }
    }
  }
  c->lowF.alloc(F.size() * sizeof(double));
  BIE_HIP(hipMemcpy(c->lowF.ptr, F.data(), F.size() * sizeof(double), hipMemcpyHostToDevice));
  c->lownorm.alloc(25 * sizeof(double));
  BIE_HIP(hipMemcpy(c->lownorm.ptr, nrm.data(), 25 * sizeof(double), hipMemcpyHostToDevice));
  // directed close pairs grouped by target sphere: features and frames
  const int64_t np = (int64_t)c->close_idx.size();
  c->pair_feat.assign((size_t)np * kNFeat, 0.0f);
  c->pair_frame.assign((size_t)np * kFrame, 0.0);
  const double* ce = c->centres.data();
  auto gap = [&](int a, int b) {
    const double dx = ce[3 * a] - ce[3 * b], dy = ce[3 * a + 1] - ce[3 * b + 1], dz = ce[3 * a + 2] - ce[3 * b + 2];
    return std::sqrt(dx * dx + dy * dy + dz * dz) - 2.0;
  };
  for (int64_t i = 0; i < c->nb; ++i) {
    const int ni = c->close_ptr[i + 1] - c->close_ptr[i];
    double crowd = 0.0;
    for (int e = c->close_ptr[i]; e < c->close_ptr[i + 1]; ++e) crowd += 0.1 / (gap((int)i, c->close_idx[e]) + 0.1);
    for (int e = c->close_ptr[i]; e < c->close_ptr[i + 1]; ++e) {
      const int j = c->close_idx[e];
      const int nj = c->close_ptr[j + 1] - c->close_ptr[j];
      const double g = gap((int)i, j);
      double mi = c->close_gap, mj = c->close_gap;
      bool hi = false, hj = false;
      for (int q = c->close_ptr[i]; q < c->close_ptr[i + 1]; ++q)
        if (c->close_idx[q] != j) {
          const double gg = gap((int)i, c->close_idx[q]);
          mi = hi ? std::min(mi, gg) : gg;
          hi = true;
        }
      for (int q = c->close_ptr[j]; q < c->close_ptr[j + 1]; ++q)
        if (c->close_idx[q] != (int)i) {
          const double gg = gap(j, c->close_idx[q]);
          mj = hj ? std::min(mj, gg) : gg;
          hj = true;
        }
      float* f = &c->pair_feat[(size_t)e * kNFeat];
      f[0] = (float)g;
      f[1] = (float)std::log(g + 0.01);
      f[2] = (float)(0.1 / (g + 0.1));
      f[3] = (float)(ni / 8.0);
      f[4] = (float)(nj / 8.0);
      f[5] = (float)mi;
      f[6] = (float)mj;
      f[7] = (float)crowd;
      const double d[3] = {ce[3 * j] - ce[3 * i], ce[3 * j + 1] - ce[3 * i + 1], ce[3 * j + 2] - ce[3 * i + 2]};
      double Q[9];
      pair_frame(d, Q);
      frame_of(Q, &c->pair_frame[(size_t)e * kFrame]);
    }
  }
  std::vector<double> fr = c->pair_frame.empty() ? std::vector<double>(kFrame, 0.0) : c->pair_frame;
  c->dframe.alloc(fr.size() * sizeof(double));
  BIE_HIP(hipMemcpy(c->dframe.ptr, fr.data(), fr.size() * sizeof(double), hipMemcpyHostToDevice));
  c->rho.alloc((size_t)c->nb * 25 * sizeof(double));
  c->zeta.alloc((size_t)c->nb * 25 * sizeof(double));
}

// rho_k = sum_nodes w F_k . f / ||F_k||^2, one work-group per sphere
__global__ void k_restrict(const double* f, const double* F, const double* wnode, const double* nrm, int P,
                           double* rho) {
  const int k = blockIdx.x;
  __shared__ double red[25][4];
  double acc[25];
  for (int m = 0; m < 25; ++m) acc[m] = 0.0;
  for (int g = threadIdx.x; g < P; g += blockDim.x) {
    const double* fv = f + 3 * ((int64_t)k * P + g);
    const double w = wnode[g];
    const double* Fg = F + (size_t)g * 75;
    for (int m = 0; m < 25; ++m) acc[m] += w * (Fg[3 * m] * fv[0] + Fg[3 * m + 1] * fv[1] + Fg[3 * m + 2] * fv[2]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int m = 0; m < 25; ++m) {
    double s = acc[m];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[m][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 25) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[threadIdx.x][w];
    rho[(int64_t)k * 25 + threadIdx.x] = s / nrm[threadIdx.x];
  }
}

// f (+)= sum_k rho_k F_k at every node
__global__ void k_prolong(const double* rho, const double* F, int P, int64_t N, int accumulate, double* f) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / P;
    const int li = (int)(g - k * P);
    const double* r = rho + k * 25;
    const double* Fg = F + (size_t)li * 75;
    double o[3] = {0, 0, 0};
    for (int m = 0; m < 25; ++m)
      for (int d = 0; d < 3; ++d) o[d] += r[m] * Fg[3 * m + d];
    for (int d = 0; d < 3; ++d) f[3 * g + d] = (accumulate ? f[3 * g + d] : 0.0) + o[d];
  }
}

// zeta_i = sum_{e in close(i)} rot_e^T [K_off(theta_e) rot_e rho_j + K_self(theta_e) rot_e rho_i]
// skip_rigid: the rigid modes (b, c: translations and rotations) are left to the global
// rigid-mode correction: they are dropped from rho and from zeta (the rotation into the
// pair frame maps each of the two vector blocks onto itself, so dropping them in the
// global frame is dropping them in every pair frame).
__global__ void k_coarse_apply(const double* rho, const int* close_ptr, const int* close_idx, const double* frames,
                               const float* theta, int64_t nb, int skip_rigid, double* zeta) {
  const int64_t sph = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sph >= nb) return;
  double z[25], ri[25];
  for (int m = 0; m < 25; ++m) {
    z[m] = 0.0;
    ri[m] = (skip_rigid && m >= kIB && m < kITV) ? 0.0 : rho[(int64_t)sph * 25 + m];
  }
  for (int e = close_ptr[sph]; e < close_ptr[sph + 1]; ++e) {
    const int j = close_idx[e];
    const double* fr = frames + (size_t)e * kFrame;
    double rj[25], y[25], x[25], c[25], back[25];
    for (int m = 0; m < 25; ++m) rj[m] = (skip_rigid && m >= kIB && m < kITV) ? 0.0 : rho[(int64_t)j * 25 + m];
    rot25_apply<double>(fr, rj, y, false);
    rot25_apply<double>(fr, ri, x, false);
    for (int m = 0; m < 25; ++m) c[m] = 0.0;
    apply_K<double, float>(theta + (size_t)e * kNTheta2, y, c);
    apply_K<double, float>(theta + (size_t)e * kNTheta2 + kNTheta, x, c);
    rot25_apply<double>(fr, c, back, true);
    for (int m = 0; m < 25; ++m) z[m] += back[m];
  }
  for (int m = 0; m < 25; ++m) zeta[(int64_t)sph * 25 + m] = (skip_rigid && m >= kIB && m < kITV) ? 0.0 : z[m];
}

__global__ void k_zero_rigid(double* rho, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb * 6) rho[(i / 6) * 25 + kIB + i % 6] = 0.0;
}

void zero_rigid_modes(bie_ctx* c, double* rho) {
  k_zero_rigid<<<dim3((unsigned)((c->nb * 6 + 255) / 256)), dim3(256), 0, c->stream>>>(rho, c->nb);
  BIE_HIP(hipGetLastError());
}

void lowmode_restrict(bie_ctx* c, const double* f, double* rho) {
  k_restrict<<<dim3((unsigned)c->nb), dim3(256), 0, c->stream>>>(f, c->lowF.as<double>(), c->wnode.as<double>(),
                                                                     c->lownorm.as<double>(), c->P, rho);
  BIE_HIP(hipGetLastError());
}

void lowmode_prolong(bie_ctx* c, const double* rho, double* f, bool accumulate) {
  const int blocks = (int)std::min<int64_t>((c->N + 255) / 256, 8192);
  k_prolong<<<dim3(blocks), dim3(256), 0, c->stream>>>(rho, c->lowF.as<double>(), c->P, c->N, accumulate ? 1 : 0, f);
  BIE_HIP(hipGetLastError());
}

// z += P zeta(R r): the learned part of the MLP preconditioner (z already holds M0 r)
void coarse_correct(bie_ctx* c, const double* r, double* z, bool skip_rigid) {
  if (!c->theta_ready || c->close_idx.empty()) return;
  lowmode_restrict(c, r, c->rho.as<double>());
  k_coarse_apply<<<dim3((unsigned)((c->nb + 63) / 64)), dim3(64), 0, c->stream>>>(
      c->rho.as<double>(), c->dclose_ptr.as<int>(), c->dclose_idx.as<int>(), c->dframe.as<double>(),
      c->mlp_theta.as<float>(), c->nb, skip_rigid ? 1 : 0, c->zeta.as<double>());
  BIE_HIP(hipGetLastError());
  lowmode_prolong(c, c->zeta.as<double>(), z, true);
}

}  // namespace bie
