// Batched vector spherical harmonic transforms and the spectral self term.
//
// One work-group per sphere.  Forward transform (Section 2.1): node values are turned
// into spherical components (f_r, f_theta, f_phi), Fourier-analysed along each latitude
// (the FFT stage of the fast transform, here a direct real DFT since n_phi <= 42), and
// projected on V, W, X with the Gauss-Legendre weights of Eq. 4.4.  The projection uses
// the Legendre tables Pbar, dPbar/dtheta and m Pbar / sin(theta), so the tangential part
// needs no division by sin(theta) (equivalent to Eqs. 2.7-2.14 on band-limited fields).
// Self term (Section 4.1, Eqs. 4.6-4.7): coefficients times the eigenvalues of Theorem 2
// (double layer as principal value), then the inverse transform (Eqs. 2.15-2.17):
// V, W, X -> (Y, G, X) coefficients -> Legendre synthesis per latitude -> inverse DFT.
//
// The Legendre stages are, per azimuthal order m, small dense contractions: projection
// (rows n = m..p) x (latitudes j) x (Fourier columns), synthesis (latitudes) x (n) x
// (coefficient columns).  They run either as per-mode FMA loops from LDS, or (MF, the
// context's legendre_mfma option) on the matrix cores: one 16 x 16 tile per (m, row
// block), K = 4 per instruction, the three tables (Pbar, dPbar, m Pbar / sin)
// accumulated into one tile with their right-hand columns arranged so that the tile's
// columns are the combinations the next step needs (see the comments at each stage).
// Lane layout of v_mfma_{f32,f64}_16x16x4 (read off the hardware with known operands):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its four results are
// D[4 (l / 16) + v][l % 16] for f32 and D[l / 16 + 4 v][l % 16] for f64, v = 0..3.
#include "bie_internal.h"

namespace bie {

struct VshParams {
  const double* mu;
  const double* coef_in;
  double* u;
  double* coef_out;
  void* q;
  double* moments;
  const void* leg;
  const void* dft;
  const void* wlat;
  const double* frame;
  const double* wnode;
  const int* modes;
  int p, nphi, mmax, P, ncoef, nlat;
  int64_t N, nb;
  double c_identity, scale_out;
  int do_self, bordered, coef_is_input, want_moments, write_q, q_float;
  int pc_border;   // isolated-sphere inverse of the bordered mobility block (preconditioner)
  int accumulate;  // u += synthesis (else u = synthesis)
  double wv1;      // n = 1 coupling: V'_1 += wv1 * W_1 (preconditioner of the completed form)
  double lam[3][33];
  const double* radius;  // per-sphere radii for lam_mode 1, 2, 3 (see VshCall)
  int lam_mode;
  int lam_pow[3];
  double lamS[3][33];
};

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd4 __attribute__((ext_vector_type(4)));
template <typename R>
struct Tile;
template <>
struct Tile<float> {
  typedef vf4 T;
  static __device__ __forceinline__ vf4 step(float a, float b, vf4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};
template <>
struct Tile<double> {
  typedef vd4 T;
  static __device__ __forceinline__ vd4 step(double a, double b, vd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename R, bool MF>
__global__ __launch_bounds__(256) void vsh_kernel(VshParams a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int P = a.P, nphi = a.nphi, nl = a.nlat, M1 = a.mmax + 1, nc = a.ncoef;
  R* fs = reinterpret_cast<R*>(smem_raw);   // 3 x P spherical components
  R* F = fs + 3 * P;                         // 3 x nl x M1 x 2 Fourier coefficients
  R* C = F + 3 * nl * M1 * 2;                // 3 x nc x 2 (Y, G, X) coefficients
  R* PJ = C + 3 * nc * 2;                    // nc x 6 projections (matrix-core path)
  double* red = reinterpret_cast<double*>(smem_raw + ((sizeof(R) * (3 * P + 3 * nl * M1 * 2 + 12 * nc) + 15) & ~size_t(15)));
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  const R* leg = reinterpret_cast<const R*>(a.leg);
  const R* dft = reinterpret_cast<const R*>(a.dft);
  const R* wl = reinterpret_cast<const R*>(a.wlat);
  const int64_t base = (int64_t)k * P;

  if (!a.coef_is_input) {
    // ---- node values -> spherical components; source strengths; moments ------------
    double mom[6] = {0, 0, 0, 0, 0, 0};
    for (int g = tid; g < P; g += nt) {
      const double* m3 = a.mu + 3 * (base + g);
      const double mx = m3[0], my = m3[1], mz = m3[2];
      const double* fr = a.frame + 9 * g;
      fs[g] = (R)(mx * fr[0] + my * fr[1] + mz * fr[2]);
      fs[P + g] = (R)(mx * fr[3] + my * fr[4] + mz * fr[5]);
      fs[2 * P + g] = (R)(mx * fr[6] + my * fr[7] + mz * fr[8]);
      const double w = a.wnode[g];
      if (a.write_q) {
        // far-field source: q = w mu and o . q (o = unit offset = e_r of the node)
        const double oq = w * (mx * fr[0] + my * fr[1] + mz * fr[2]);
        if (a.q_float) {
          float4 v = make_float4((float)(w * mx), (float)(w * my), (float)(w * mz), (float)oq);
          reinterpret_cast<float4*>(a.q)[base + g] = v;
        } else {
          double* qd = reinterpret_cast<double*>(a.q) + 4 * (base + g);
          qd[0] = w * mx;
          qd[1] = w * my;
          qd[2] = w * mz;
          qd[3] = oq;
        }
      }
      if (a.want_moments) {
        mom[0] += w * mx;
        mom[1] += w * my;
        mom[2] += w * mz;
        mom[3] += w * (fr[1] * mz - fr[2] * my);
        mom[4] += w * (fr[2] * mx - fr[0] * mz);
        mom[5] += w * (fr[0] * my - fr[1] * mx);
      }
    }
    if (a.want_moments) {
      for (int d = 0; d < 6; ++d) {
        double s = wave_sum(mom[d]);
        if (lane == 0) red[d * 4 + wv] = s;
      }
      __syncthreads();
      if (tid < 6) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[tid * 4 + w];
        if (a.radius) {
          // sphere of radius a: area element a^2, lever arm a
          const double rad = a.radius[k];
          s *= (tid < 3) ? rad * rad : rad * rad * rad;
        }
        a.moments[6 * k + tid] = s;
        red[32 + tid] = s;
      }
    }
    __syncthreads();

    // ---- real DFT along each latitude: F_c(j, m) = sum_l f_c(j, l) e^{-i m phi_l} ------
    for (int e = tid; e < 3 * nl * M1; e += nt) {
      const int c = e / (nl * M1), rem = e - c * nl * M1, j = rem / M1, m = rem - j * M1;
      const R* f = fs + c * P + j * nphi;
      const R* tw = dft + (size_t)m * nphi * 2;
      R re = 0, im = 0;
      for (int l = 0; l < nphi; ++l) {
        re += f[l] * tw[2 * l];
        im -= f[l] * tw[2 * l + 1];
      }
      F[2 * e] = re;
      F[2 * e + 1] = im;
    }
    __syncthreads();

    // ---- Legendre projection onto V, W, X ------------------------------------------
    // with b = int dPbar F_t-like sums and c = int m Pbar / sin sums (weights w_j):
    //   g = b_t - i c_p,  x = b_p + i c_t,  a = int Pbar F_r
    // V = (g - (n+1) a) / ((n+1)(2n+1)); W = (g + n a) / (n(2n+1)); X = x / (n(n+1))
    if (MF) {
      // tile rows n = m + 16 rt + (0..15), K = latitudes j, columns
      //   0: Re g  1: Im g  2: Re x  3: Im x  4: Re a  5: Im a
      // from dPbar x [Re F_t, Im F_t, Re F_p, Im F_p] + mQ x [Im F_p, -Re F_p, -Im F_t,
      // Re F_t] + Pbar x [0, 0, 0, 0, Re F_r, Im F_r]
      const int col = lane & 15, kq = lane >> 4;
      for (int task = wv; task < 2 * M1; task += nw) {
        const int m = task >> 1, rt = task & 1;
        if (16 * rt >= a.p + 1 - m) continue;   // wave-uniform
        const int off = m * (a.p + 1) - (m * (m - 1)) / 2;
        const int nA = m + 16 * rt + col;
        const bool rowok = nA <= a.p;
        const int iA = off + (rowok ? nA - m : 0);
        typename Tile<R>::T acc = {0, 0, 0, 0};
        for (int ks = 0; ks < (nl + 3) / 4; ++ks) {
          const int j = 4 * ks + kq;
          const bool jok = j < nl;
          const int jc = jok ? j : 0;
          const R wj = (rowok && jok) ? wl[jc] : (R)0;
          const R ap = wj * leg[((size_t)0 * nc + iA) * nl + jc];
          const R ad = wj * leg[((size_t)1 * nc + iA) * nl + jc];
          const R aq = wj * leg[((size_t)2 * nc + iA) * nl + jc];
          const R jm = jok ? (R)1 : (R)0;
          const R* Fr = F + ((0 * nl + jc) * M1 + m) * 2;
          const R* Ft = F + ((1 * nl + jc) * M1 + m) * 2;
          const R* Fp = F + ((2 * nl + jc) * M1 + m) * 2;
          const R trr = jm * Ft[0], tri = jm * Ft[1], prr = jm * Fp[0], pri = jm * Fp[1];
          const R bd = col == 0 ? trr : col == 1 ? tri : col == 2 ? prr : col == 3 ? pri : (R)0;
          const R bq = col == 0 ? pri : col == 1 ? -prr : col == 2 ? -tri : col == 3 ? trr : (R)0;
          const R bp = col == 4 ? jm * Fr[0] : col == 5 ? jm * Fr[1] : (R)0;
          acc = Tile<R>::step(ad, bd, acc);
          acc = Tile<R>::step(aq, bq, acc);
          acc = Tile<R>::step(ap, bp, acc);
        }
        if (col < 6)
          for (int v = 0; v < 4; ++v) {
            const int nD = m + 16 * rt + Tile<R>::row(kq, v);
            if (nD <= a.p) PJ[(off + nD - m) * 6 + col] = acc[v];
          }
      }
      __syncthreads();
    }
    for (int i = tid; i < nc; i += nt) {
      const int m = a.modes[2 * i], n = a.modes[2 * i + 1];
      R gr, gi, xnr, xni, ar, ai;
      if (MF) {
        gr = PJ[6 * i];
        gi = PJ[6 * i + 1];
        xnr = PJ[6 * i + 2];
        xni = PJ[6 * i + 3];
        ar = PJ[6 * i + 4];
        ai = PJ[6 * i + 5];
      } else {
        const R* Lp = leg + ((size_t)0 * nc + i) * nl;
        const R* Ld = leg + ((size_t)1 * nc + i) * nl;
        const R* Lq = leg + ((size_t)2 * nc + i) * nl;
        R sar = 0, sai = 0, btr = 0, bti = 0, bpr = 0, bpi = 0, ctr = 0, cti = 0, cpr = 0, cpi = 0;
        for (int j = 0; j < nl; ++j) {
          const R w = wl[j];
          const R pw = w * Lp[j], dw = w * Ld[j], qw = w * Lq[j];
          const R* Fr = F + ((0 * nl + j) * M1 + m) * 2;
          const R* Ft = F + ((1 * nl + j) * M1 + m) * 2;
          const R* Fp = F + ((2 * nl + j) * M1 + m) * 2;
          sar += pw * Fr[0];
          sai += pw * Fr[1];
          btr += dw * Ft[0];
          bti += dw * Ft[1];
          bpr += dw * Fp[0];
          bpi += dw * Fp[1];
          ctr += qw * Ft[0];
          cti += qw * Ft[1];
          cpr += qw * Fp[0];
          cpi += qw * Fp[1];
        }
        gr = btr + cpi;
        gi = bti - cpr;
        xnr = bpr - cti;
        xni = bpi + ctr;
        ar = sar;
        ai = sai;
      }
      const R nn = (R)n;
      R vr = (gr - (nn + 1) * ar) / ((nn + 1) * (2 * nn + 1));
      R vi = (gi - (nn + 1) * ai) / ((nn + 1) * (2 * nn + 1));
      R wr = 0, wi = 0, xr = 0, xi = 0;
      if (n >= 1) {
        wr = (gr + nn * ar) / (nn * (2 * nn + 1));
        wi = (gi + nn * ai) / (nn * (2 * nn + 1));
        xr = xnr / (nn * (nn + 1));
        xi = xni / (nn * (nn + 1));
      }
      if (a.coef_out) {
        double* co = a.coef_out + (size_t)k * 3 * nc * 2;
        co[(0 * nc + i) * 2] = vr;
        co[(0 * nc + i) * 2 + 1] = vi;
        co[(1 * nc + i) * 2] = wr;
        co[(1 * nc + i) * 2 + 1] = wi;
        co[(2 * nc + i) * 2] = xr;
        co[(2 * nc + i) * 2 + 1] = xi;
      }
      if (a.do_self) {
        R lv = (R)a.lam[0][n], lw = (R)a.lam[1][n], lx = (R)a.lam[2][n];
        if (a.lam_mode != 0) {
          // sphere of radius a_k: the single layer's eigenvalues scale with a_k
          const double rad = a.radius[k];
          double l3[3];
          for (int f = 0; f < 3; ++f) {
            if (a.lam_mode == 3) {
              double sc = 1.0;
              for (int e = 0; e < -a.lam_pow[f]; ++e) sc /= rad;
              l3[f] = a.lamS[f][n] * sc + a.lam[f][n];
            } else {
              const double s = rad * a.lamS[f][n] + a.lam[f][n];
              l3[f] = (a.lam_mode == 1) ? s : (s != 0.0 ? 1.0 / s - 2.0 : 0.0);
            }
          }
          lv = (R)l3[0];
          lw = (R)l3[1];
          lx = (R)l3[2];
        }
        const R w0r = wr, w0i = wi;
        vr *= lv;
        vi *= lv;
        wr *= lw;
        wi *= lw;
        xr *= lx;
        xi *= lx;
        if (n == 1) {
          vr += (R)a.wv1 * w0r;
          vi += (R)a.wv1 * w0i;
        }
        // Eqs. 2.16-2.17: G = V + W, Y = -(n+1) V + n W
        C[(0 * nc + i) * 2] = -(nn + 1) * vr + nn * wr;
        C[(0 * nc + i) * 2 + 1] = -(nn + 1) * vi + nn * wi;
        C[(1 * nc + i) * 2] = vr + wr;
        C[(1 * nc + i) * 2 + 1] = vi + wi;
        C[(2 * nc + i) * 2] = xr;
        C[(2 * nc + i) * 2 + 1] = xi;
      }
    }
  } else {
    for (int i = tid; i < nc; i += nt) {
      const int n = a.modes[2 * i + 1];
      const double* ci = a.coef_in + (size_t)k * 3 * nc * 2;
      const R nn = (R)n;
      const R vr = (R)ci[(0 * nc + i) * 2], vi = (R)ci[(0 * nc + i) * 2 + 1];
      const R wr = (R)ci[(1 * nc + i) * 2], wi = (R)ci[(1 * nc + i) * 2 + 1];
      C[(0 * nc + i) * 2] = -(nn + 1) * vr + nn * wr;
      C[(0 * nc + i) * 2 + 1] = -(nn + 1) * vi + nn * wi;
      C[(1 * nc + i) * 2] = vr + wr;
      C[(1 * nc + i) * 2 + 1] = vi + wi;
      C[(2 * nc + i) * 2] = (R)ci[(2 * nc + i) * 2];
      C[(2 * nc + i) * 2 + 1] = (R)ci[(2 * nc + i) * 2 + 1];
    }
  }
  __syncthreads();

  if (!a.do_self && !a.coef_is_input) {
    // no synthesis: the output starts at zero (later stages accumulate into it)
    if (a.u) {
      for (int g = tid; g < P; g += nt)
        for (int d = 0; d < 3; ++d) a.u[3 * (base + g) + d] = 0.0;
      if (a.bordered && tid < 6) {
        if (tid < 3)
          a.u[3 * a.N + 3 * (int64_t)k + tid] = 0.0;
        else
          a.u[3 * a.N + 3 * a.nb + 3 * (int64_t)k + (tid - 3)] = 0.0;
      }
    }
    return;
  }

  // ---- Legendre synthesis per latitude (Eqs. 2.9-2.10 written with dPbar, m Pbar/s) --
  //   F_r = sum_n Pbar Y;  F_t = sum_n (dPbar G - i mQ X);  F_p = sum_n (i mQ G + dPbar X)
  if (MF) {
    // tile rows j = 16 jt + (0..15), K = degrees n, columns
    //   0: Re F_t  1: Im F_t  2: Re F_p  3: Im F_p  4: Re F_r  5: Im F_r
    // from dPbar x [Re G, Im G, Re X, Im X] + mQ x [Im X, -Re X, -Im G, Re G] +
    // Pbar x [0, 0, 0, 0, Re Y, Im Y]
    const int col = lane & 15, kq = lane >> 4;
    for (int task = wv; task < 2 * M1; task += nw) {
      const int m = task >> 1, jt = task & 1;
      if (16 * jt >= nl) continue;   // wave-uniform
      const int off = m * (a.p + 1) - (m * (m - 1)) / 2;
      const int L = a.p + 1 - m;
      const int jA = 16 * jt + col;
      const bool jok = jA < nl;
      const int jc = jok ? jA : 0;
      typename Tile<R>::T acc = {0, 0, 0, 0};
      for (int ks = 0; ks < (L + 3) / 4; ++ks) {
        const int dn = 4 * ks + kq;
        const bool nok = dn < L;
        const int i = off + (nok ? dn : 0);
        const R am = (jok && nok) ? (R)1 : (R)0;
        const R ap = am * leg[((size_t)0 * nc + i) * nl + jc];
        const R ad = am * leg[((size_t)1 * nc + i) * nl + jc];
        const R aq = am * leg[((size_t)2 * nc + i) * nl + jc];
        const R bm = nok ? (R)1 : (R)0;
        const R yr = bm * C[(0 * nc + i) * 2], yi = bm * C[(0 * nc + i) * 2 + 1];
        const R gr = bm * C[(1 * nc + i) * 2], gi = bm * C[(1 * nc + i) * 2 + 1];
        const R xr = bm * C[(2 * nc + i) * 2], xi = bm * C[(2 * nc + i) * 2 + 1];
        const R bd = col == 0 ? gr : col == 1 ? gi : col == 2 ? xr : col == 3 ? xi : (R)0;
        const R bq = col == 0 ? xi : col == 1 ? -xr : col == 2 ? -gi : col == 3 ? gr : (R)0;
        const R bp = col == 4 ? yr : col == 5 ? yi : (R)0;
        acc = Tile<R>::step(ad, bd, acc);
        acc = Tile<R>::step(aq, bq, acc);
        acc = Tile<R>::step(ap, bp, acc);
      }
      if (col < 6) {
        const int c = col < 2 ? 1 : col < 4 ? 2 : 0;
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * jt + Tile<R>::row(kq, v);
          if (j < nl) F[((c * nl + j) * M1 + m) * 2 + (col & 1)] = acc[v];
        }
      }
    }
  }
  for (int e = MF ? nl * M1 : tid; e < nl * M1; e += nt) {
    const int j = e / M1, m = e - j * M1;
    const int off = m * (a.p + 1) - (m * (m - 1)) / 2;
    R rr = 0, ri = 0, tr = 0, ti = 0, pr = 0, pi = 0;
    for (int n = m; n <= a.p; ++n) {
      const int i = off + (n - m);
      const R lp = leg[((size_t)0 * nc + i) * nl + j];
      const R ld = leg[((size_t)1 * nc + i) * nl + j];
      const R lq = leg[((size_t)2 * nc + i) * nl + j];
      const R yr = C[(0 * nc + i) * 2], yi = C[(0 * nc + i) * 2 + 1];
      const R gr = C[(1 * nc + i) * 2], gi = C[(1 * nc + i) * 2 + 1];
      const R xr = C[(2 * nc + i) * 2], xi = C[(2 * nc + i) * 2 + 1];
      rr += lp * yr;
      ri += lp * yi;
      tr += ld * gr + lq * xi;
      ti += ld * gi - lq * xr;
      pr += -lq * gi + ld * xr;
      pi += lq * gr + ld * xi;
    }
    F[((0 * nl + j) * M1 + m) * 2] = rr;
    F[((0 * nl + j) * M1 + m) * 2 + 1] = ri;
    F[((1 * nl + j) * M1 + m) * 2] = tr;
    F[((1 * nl + j) * M1 + m) * 2 + 1] = ti;
    F[((2 * nl + j) * M1 + m) * 2] = pr;
    F[((2 * nl + j) * M1 + m) * 2 + 1] = pi;
  }
  __syncthreads();

  // ---- inverse DFT, spherical -> Cartesian, identity and bordered terms ------------
  const double* vk = nullptr;
  const double* ok = nullptr;
  if (a.bordered && a.do_self) {
    vk = a.mu + 3 * a.N + 3 * (int64_t)k;
    ok = a.mu + 3 * a.N + 3 * a.nb + 3 * (int64_t)k;
  }
  // Preconditioner of the bordered block: with A^-1 the isolated self inverse applied to
  // the node part r_u, int A^-1 r_u = 3/2 int r_u and int o x A^-1 r_u = 3 int o x r_u
  // (W_1 and X_1 eigenvalues 2/3 and 1/3 of 1/2 + S + D_pv), so the rigid motion that
  // meets the force / torque rows r_F, r_T is
  //   v = (4 pi r_F - 3/2 int r_u) / (6 pi),  w = (8pi/3 r_T - 3 int o x r_u) / (8 pi),
  // and the density is A^-1 r_u + 3/2 v + 3 w x o.
  // On a sphere of radius a (moments then carry a^2, a^3): A^-1 is 3/(2a) on W_1 and 3/a
  // on X_1, so v = (4 pi r_F - 3/(2a) int r_u) / (6 pi a), w = (8pi/3 r_T - 3/a int (y - c)
  // x r_u) / (8 pi a^3), and the density gains 3/(2a) v + 3 w x o.
  const double rad = a.radius ? a.radius[k] : 1.0;
  double pv[3] = {0, 0, 0}, pw[3] = {0, 0, 0};
  if (a.pc_border) {
    const double* rF = a.mu + 3 * a.N + 3 * (int64_t)k;
    const double* rT = a.mu + 3 * a.N + 3 * a.nb + 3 * (int64_t)k;
    for (int d = 0; d < 3; ++d) {
      pv[d] = (4.0 * M_PI * rF[d] - (1.5 / rad) * red[32 + d]) / (6.0 * M_PI * rad);
      pw[d] = ((8.0 * M_PI / 3.0) * rT[d] - (3.0 / rad) * red[35 + d]) / (8.0 * M_PI * rad * rad * rad);
    }
  }
  const double pv_scale = 1.5 / rad;
  for (int g = tid; g < P; g += nt) {
    const int j = g / nphi, l = g - j * nphi;
    R f[3];
    for (int c = 0; c < 3; ++c) {
      const R* Fc = F + ((c * nl + j) * M1) * 2;
      R s = Fc[0];
      R s2 = 0;
      const R* tw1 = dft + 2 * nphi;  // row m = 1: cos, sin of 2 pi idx / n_phi
      for (int m = 1; m < M1; ++m) {
        const int idx = (m * l) % nphi;
        s2 += Fc[2 * m] * tw1[2 * idx] - Fc[2 * m + 1] * tw1[2 * idx + 1];
      }
      f[c] = s + 2 * s2;
    }
    const double* fr = a.frame + 9 * g;
    double out[3];
    for (int d = 0; d < 3; ++d)
      out[d] = a.scale_out * ((double)f[0] * fr[d] + (double)f[1] * fr[3 + d] + (double)f[2] * fr[6 + d]);
    if (!a.coef_is_input) {
      const double* m3 = a.mu + 3 * (base + g);
      for (int d = 0; d < 3; ++d) out[d] += a.c_identity * m3[d];
    }
    if (vk) {
      // - v_k - omega_k x (x - c_k), x - c_k = a e_r
      const double w0 = rad * ok[0], w1 = rad * ok[1], w2 = rad * ok[2];
      out[0] -= vk[0] + (w1 * fr[2] - w2 * fr[1]);
      out[1] -= vk[1] + (w2 * fr[0] - w0 * fr[2]);
      out[2] -= vk[2] + (w0 * fr[1] - w1 * fr[0]);
    }
    if (a.pc_border) {
      out[0] += pv_scale * pv[0] + 3.0 * (pw[1] * fr[2] - pw[2] * fr[1]);
      out[1] += pv_scale * pv[1] + 3.0 * (pw[2] * fr[0] - pw[0] * fr[2]);
      out[2] += pv_scale * pv[2] + 3.0 * (pw[0] * fr[1] - pw[1] * fr[0]);
    }
    for (int d = 0; d < 3; ++d) a.u[3 * (base + g) + d] = a.accumulate ? a.u[3 * (base + g) + d] + out[d] : out[d];
  }
  if (a.pc_border && tid < 6) {
    if (tid < 3)
      a.u[3 * a.N + 3 * (int64_t)k + tid] = pv[tid];
    else
      a.u[3 * a.N + 3 * a.nb + 3 * (int64_t)k + (tid - 3)] = pw[tid - 3];
  }
  if (vk && tid < 6) {
    // constraint rows: (1/4pi) int mu, (3/8pi) int (y - c) x mu
    const double s = red[32 + tid];
    if (tid < 3)
      a.u[3 * a.N + 3 * (int64_t)k + tid] = s / (4.0 * M_PI);
    else
      a.u[3 * a.N + 3 * a.nb + 3 * (int64_t)k + (tid - 3)] = 3.0 * s / (8.0 * M_PI);
  }
}

static size_t vsh_smem(const bie_ctx* c, size_t rs) {
  size_t b = rs * (3 * (size_t)c->P + 3 * (size_t)c->nlat * (c->mmax + 1) * 2 + 12 * (size_t)c->ncoef);
  b = (b + 15) & ~size_t(15);
  return b + 64 * sizeof(double);
}

void launch_vsh(bie_ctx* c, int precision, const VshCall& v) {
  VshParams a{};
  a.mu = v.mu;
  a.coef_in = v.coef_in;
  a.u = v.u;
  a.coef_out = v.write_coef ? c->coef.as<double>() : nullptr;
  a.q = c->q.ptr;
  a.moments = c->moments.as<double>();
  const bool f32 = precision == BIE_MIXED;
  a.leg = f32 ? c->leg_f.ptr : c->leg.ptr;
  a.dft = f32 ? c->dft_f.ptr : c->dft.ptr;
  a.wlat = f32 ? c->wlat_f.ptr : c->wlat_d.ptr;
  a.frame = c->frame.as<double>();
  a.wnode = c->wnode.as<double>();
  a.modes = c->modes.as<int>();
  a.p = c->p;
  a.nphi = c->n_phi;
  a.mmax = c->mmax;
  a.P = c->P;
  a.ncoef = c->ncoef;
  a.nlat = c->nlat;
  a.N = c->N;
  a.nb = c->nb;
  a.c_identity = v.c_identity;
  a.scale_out = v.scale_out;
  a.do_self = v.do_self ? 1 : 0;
  a.bordered = v.bordered ? 1 : 0;
  a.coef_is_input = v.coef_is_input ? 1 : 0;
  a.want_moments = (v.want_moments || v.bordered || v.pc_border) ? 1 : 0;
  a.write_q = v.write_q ? 1 : 0;
  a.q_float = f32 ? 1 : 0;
  a.pc_border = v.pc_border ? 1 : 0;
  a.accumulate = v.accumulate ? 1 : 0;
  a.wv1 = v.wv1;
  for (int f = 0; f < 3; ++f)
    for (int n = 0; n < 33; ++n) a.lam[f][n] = v.lam[f][n];
  a.radius = v.radius;
  a.lam_mode = v.radius ? v.lam_mode : 0;
  for (int f = 0; f < 3; ++f) a.lam_pow[f] = v.lam_pow[f];
  for (int f = 0; f < 3; ++f)
    for (int n = 0; n < 33; ++n) a.lamS[f][n] = v.lamS[f][n];
  const size_t sm = vsh_smem(c, f32 ? sizeof(float) : sizeof(double));
  const dim3 grid((unsigned)c->nb), block(256);
  if (f32 && c->legendre_mfma)
    vsh_kernel<float, true><<<grid, block, sm, c->stream>>>(a);
  else if (f32)
    vsh_kernel<float, false><<<grid, block, sm, c->stream>>>(a);
  else if (c->legendre_mfma)
    vsh_kernel<double, true><<<grid, block, sm, c->stream>>>(a);
  else
    vsh_kernel<double, false><<<grid, block, sm, c->stream>>>(a);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
