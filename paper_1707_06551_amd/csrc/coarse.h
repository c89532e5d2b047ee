// Shared definitions of the learned coarse correction (coarse.hip, mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace bie {

// layout of the 25 low-mode coefficients
constexpr int kIS = 0, kIA = 1, kIB = 4, kIC = 7, kITV = 10, kITW = 15, kITX = 20;
constexpr int kNFeat = 8;       // pair features
constexpr int kFrame = 34;      // Q (3 x 3) then D2 (5 x 5), row-major
constexpr int kNTheta = 139;    // parameters of one axisymmetric 25 x 25 block
constexpr int kNTheta2 = 278;   // off-diagonal block + self block
constexpr int kHidden = 64;

// m = 0 components; |m| = 1 doublets (x-like, y-like); |m| = 2 doublets (cos, sin)
__host__ __device__ constexpr int m0_idx(int p) {
  return p == 0 ? 0 : p == 1 ? 3 : p == 2 ? 6 : p == 3 ? 9 : p == 4 ? 14 : p == 5 ? 19 : 24;
}
__host__ __device__ constexpr int dbl(int g, int which) {
  // doublets 0..5: |m| = 1 (a, b, c, tV, tW, tX); 6..8: |m| = 2 (tV, tW, tX)
  return g == 0 ? (which ? 2 : 1)
       : g == 1 ? (which ? 5 : 4)
       : g == 2 ? (which ? 8 : 7)
       : g == 3 ? (which ? 11 : 12)
       : g == 4 ? (which ? 16 : 17)
       : g == 5 ? (which ? 21 : 22)
       : g == 6 ? (which ? 10 : 13)
       : g == 7 ? (which ? 15 : 18)
                : (which ? 20 : 23);
}

// out = rot in (transpose = false) or rot^T in; rot = diag(1, Q, Q, Q, D2, D2, D2)
template <typename T>
__host__ __device__ inline void rot25_apply(const T* fr, const T* in, T* out, bool transpose) {
  out[0] = in[0];
  for (int b = 1; b < 10; b += 3)
    for (int r = 0; r < 3; ++r) {
      T s = 0;
      for (int c = 0; c < 3; ++c) s += (transpose ? fr[3 * c + r] : fr[3 * r + c]) * in[b + c];
      out[b + r] = s;
    }
  for (int b = 10; b < 25; b += 5)
    for (int k = 0; k < 5; ++k) {
      T s = 0;
      for (int l = 0; l < 5; ++l) s += (transpose ? fr[9 + 5 * l + k] : fr[9 + 5 * k + l]) * in[b + l];
      out[b + k] = s;
    }
}

// out += K(theta) in, K commuting with rotations about the pair axis:
// theta[0..49) the 7 x 7 m = 0 block (out row-major), then (alpha, beta) per
// (out doublet, in doublet) for the 6 |m| = 1 doublets and the 3 |m| = 2 doublets.
template <typename T, typename P>
__host__ __device__ inline void apply_K(const P* th, const T* in, T* out) {
  int t = 0;
  for (int p = 0; p < 7; ++p)
    for (int q = 0; q < 7; ++q) out[m0_idx(p)] += (T)th[t++] * in[m0_idx(q)];
  for (int grp = 0; grp < 2; ++grp) {
    const int g0 = grp == 0 ? 0 : 6, g1 = grp == 0 ? 6 : 9;
    for (int op = g0; op < g1; ++op)
      for (int iq = g0; iq < g1; ++iq) {
        const T al = (T)th[t], be = (T)th[t + 1];
        t += 2;
        const int xp = dbl(op, 0), yp = dbl(op, 1), xq = dbl(iq, 0), yq = dbl(iq, 1);
        out[xp] += al * in[xq] - be * in[yq];
        out[yp] += be * in[xq] + al * in[yq];
      }
  }
}

// g += d(u . K(theta) v)/d(theta)
template <typename T>
__host__ __device__ inline void K_grad_outer(const T* u, const T* v, T* g) {
  int t = 0;
  for (int p = 0; p < 7; ++p)
    for (int q = 0; q < 7; ++q) g[t++] += u[m0_idx(p)] * v[m0_idx(q)];
  for (int grp = 0; grp < 2; ++grp) {
    const int g0 = grp == 0 ? 0 : 6, g1 = grp == 0 ? 6 : 9;
    for (int op = g0; op < g1; ++op)
      for (int iq = g0; iq < g1; ++iq) {
        const int xp = dbl(op, 0), yp = dbl(op, 1), xq = dbl(iq, 0), yq = dbl(iq, 1);
        g[t] += u[xp] * v[xq] + u[yp] * v[yq];
        g[t + 1] += -u[xp] * v[yq] + u[yp] * v[xq];
        t += 2;
      }
  }
}

void lowmode_fields_at(const double x[3], double F[25][3]);
void pair_frame(const double d[3], double Q[9]);
void frame_of(const double Q[9], double frame[kFrame]);

}  // namespace bie
