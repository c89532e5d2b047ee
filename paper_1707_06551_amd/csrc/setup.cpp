// Host-side set-up of the discretisation (Section 4: grid of Eq. 4.2, weights of Eq. 4.4,
// near-pair classification of Eq. 4.5) and the tables the kernels read.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>

#include "bie_internal.h"

namespace bie {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) n = 16;
  hipError_t e = hipMalloc(&ptr, n);
  if (e != hipSuccess) {
    ptr = nullptr;
    throw Error{BIE_ENOMEM, std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e)};
  }
  bytes = n;
}
void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

OpSpec op_spec(int op_base) {
  switch (op_base) {
    case BIE_OP_S: return {1.0, 0.0, 0.0, false, false};
    case BIE_OP_D: return {0.0, 1.0, 0.0, false, false};
    case BIE_OP_SD_BIE: return {1.0, 1.0, 0.5, false, false};
    case BIE_OP_DN_BIE: return {0.0, 1.0, 0.5, true, false};
    case BIE_OP_MOBILITY: return {1.0, 1.0, 0.5, false, true};
    // K: self K_pv = D_pv on every mode (Table 3.12), so the self multipliers are a_D's
    case BIE_OP_K: return {0.0, 1.0, 0.0, false, false, true, false};
    case BIE_OP_KL_BIE: return {0.0, 1.0, 0.5, false, false, true, true};
    default: throw Error{BIE_EINVAL, "unknown operator " + std::to_string(op_base)};
  }
}

// Gauss-Legendre nodes (descending) and weights on [-1, 1] by Newton's method on
// P_n, with the three-term recurrence for P_n and its derivative.
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? x : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (x * pn - pm) / (x * x - 1.0);
      double dx = pn / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16 && it > 2) break;
    }
    t[i] = x;
    w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// Normalised associated Legendre functions without the Condon-Shortley phase
// (Eq. 2.1) at t = cos(theta), s = sin(theta) > 0, for 0 <= m <= mmax, m <= n <= nmax:
//   Pbar_0^0 = 1/sqrt(4 pi), Pbar_m^m = sqrt((2m+1)/(2m)) s Pbar_{m-1}^{m-1},
//   Pbar_{m+1}^m = sqrt(2m+3) t Pbar_m^m,
//   Pbar_n^m = a_nm (t Pbar_{n-1}^m - b_nm Pbar_{n-2}^m).
// Q_n^m = Pbar_n^m / s obeys the same recurrence in n.  out[m][n].
static void legendre_column(int m, int nmax, double t, double s, std::vector<double>& pm, std::vector<double>& qm) {
  pm.assign(nmax + 2, 0.0);
  qm.assign(nmax + 2, 0.0);
  double pmm = 1.0 / std::sqrt(4.0 * M_PI), qmm = 0.0;
  for (int k = 1; k <= m; ++k) {
    double f = std::sqrt((2.0 * k + 1.0) / (2.0 * k));
    qmm = f * pmm;  // Pbar_k^k / s
    pmm = f * s * pmm;
  }
  if (m > nmax + 1) return;
  pm[m] = pmm;
  qm[m] = qmm;
  if (m + 1 <= nmax + 1) {
    pm[m + 1] = std::sqrt(2.0 * m + 3.0) * t * pmm;
    qm[m + 1] = std::sqrt(2.0 * m + 3.0) * t * qmm;
  }
  for (int n = m + 2; n <= nmax + 1; ++n) {
    double a = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
    double b = std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
    pm[n] = a * (t * pm[n - 1] - b * pm[n - 2]);
    qm[n] = a * (t * qm[n - 1] - b * qm[n - 2]);
  }
}

static double alpha_nm(int n, int m) {
  return std::sqrt((double)n * n * ((n + 1.0) * (n + 1.0) - (double)m * m) / ((2.0 * n + 1.0) * (2.0 * n + 3.0)));
}
static double beta_nm(int n, int m) {
  return std::sqrt((n + 1.0) * (n + 1.0) * ((double)n * n - (double)m * m) / ((2.0 * n + 1.0) * (2.0 * n - 1.0)));
}

// Recurrence constants per coefficient slot (m, n), slots ordered by m (0..mmax) then n
// (m..p), for the series evaluations at arbitrary points (series.h):
//   A_{n,m} = sqrt((4n^2-1)/(n^2-m^2)), B_{n,m} = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)).
//   m = 0:  [A_{n+1,0}, B_{n+1,0}, -sqrt(n(n+1)), 0, A_{n+2,1}, B_{n+2,1}]
//   m >= 1: [A_{n+2,m}, B_{n+2,m}, alpha_n^m, beta_n^m, sqrt(2m+3), sqrt((2m+1)/(2m))]
std::vector<double> recurrence_table(int p, int mmax) {
  auto Anm = [](int n, int m) { return std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m)); };
  auto Bnm = [](int n, int m) {
    return std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
  };
  std::vector<double> rec;
  for (int m = 0; m <= mmax; ++m)
    for (int n = m; n <= p; ++n) {
      double r[6];
      if (m == 0) {
        r[0] = Anm(n + 1, 0);
        r[1] = Bnm(n + 1, 0);
        r[2] = -std::sqrt((double)n * (n + 1.0));
        r[3] = 0.0;
        r[4] = Anm(n + 2, 1);
        r[5] = Bnm(n + 2, 1);
      } else {
        r[0] = Anm(n + 2, m);
        r[1] = Bnm(n + 2, m);
        r[2] = alpha_nm(n, m);
        r[3] = beta_nm(n, m);
        r[4] = std::sqrt(2.0 * m + 3.0);
        r[5] = std::sqrt((2.0 * m + 1.0) / (2.0 * m));
      }
      rec.insert(rec.end(), r, r + 6);
    }
  return rec;
}

// Table at one latitude: Pbar_n^m, dPbar_n^m/dtheta, m Pbar_n^m / sin(theta).
// dPbar/dtheta uses sin(theta) dY_n/dtheta = alpha_n^m Y_{n+1} - beta_n^m Y_{n-1}
// (the Legendre recurrence behind Eq. 2.9) for m >= 1 and dPbar_n^0/dtheta =
// -sqrt(n(n+1)) Pbar_n^1 for m = 0.
void legendre_tables(int p, int mmax, double t, double s, const std::vector<int>& cm, const std::vector<int>& cn,
                     double* outP, double* outD, double* outQ) {
  std::vector<double> pm, qm, p1, q1;
  legendre_column(1, p, t, s, p1, q1);
  for (int m = 0; m <= mmax; ++m) {
    legendre_column(m, p, t, s, pm, qm);
    for (size_t i = 0; i < cm.size(); ++i) {
      if (cm[i] != m) continue;
      int n = cn[i];
      outP[i] = pm[n];
      if (m == 0) {
        outD[i] = -std::sqrt((double)n * (n + 1.0)) * p1[n];
        outQ[i] = 0.0;
      } else {
        outD[i] = alpha_nm(n, m) * qm[n + 1] - (n >= 1 ? beta_nm(n, m) * qm[n - 1] : 0.0);
        outQ[i] = m * qm[n];
      }
    }
  }
}

// Matrices E_n = D^n(R_x(-pi/2)), n = 0..p, of the rotation of spherical harmonic
// expansions (Y_n^m(T^T x) = sum_m' E_n[m', m] Y_n^m'(x), T = R_x(-pi/2), so
// T^T x = (x, -z, y)), computed by their definition: the projection
// E_n[m', m] = sum_g w_g conj(Y_n^m'(x_g)) Y_n^m(T^T x_g) on a Gauss-Legendre x uniform
// grid of n + 1 latitudes and 2n + 2 longitudes, exact for products of degree-n
// harmonics.  Layout: for each n, (2n+1) x (2n+1) complex, row m' + n, column m + n.
static std::vector<double> wigner_x90(int p) {
  std::vector<double> out;
  std::vector<double> pm, qm, gt, gw;
  for (int n = 0; n <= p; ++n) {
    const int w = 2 * n + 1, nphi = 2 * n + 2;
    gauss_legendre(n + 1, gt, gw);
    std::vector<double> E(2 * (size_t)w * w, 0.0);
    std::vector<double> ya(2 * w), yb(2 * w);
    // Y_n^m at (t, phi), m = -n..n, no Condon-Shortley phase: Pbar_n^|m|(t) e^{i m phi}
    auto ylm = [&](double t, double s, double phi, std::vector<double>& y) {
      for (int m = 0; m <= n; ++m) {
        legendre_column(m, n, t, s, pm, qm);
        const double v = pm[n];
        y[2 * (n + m)] = v * std::cos(m * phi);
        y[2 * (n + m) + 1] = v * std::sin(m * phi);
        y[2 * (n - m)] = v * std::cos(m * phi);
        y[2 * (n - m) + 1] = -v * std::sin(m * phi);
      }
    };
    for (int j = 0; j <= n; ++j) {
      const double t = gt[j], s = std::sqrt(std::max(0.0, 1.0 - t * t));
      for (int l = 0; l < nphi; ++l) {
        const double phi = 2.0 * M_PI * l / nphi;
        const double wt = 2.0 * M_PI * gw[j] / nphi;
        const double x = s * std::cos(phi), y = s * std::sin(phi), z = t;
        const double rx = x, ry = -z, rz = y;   // T^T x
        const double rs = std::sqrt(std::max(0.0, rx * rx + ry * ry));
        ylm(t, s, phi, ya);
        ylm(rz, rs, std::atan2(ry, rx), yb);
        for (int a = 0; a < w; ++a)
          for (int b = 0; b < w; ++b) {
            // conj(ya[a]) * yb[b]
            const double ar = ya[2 * a], ai = -ya[2 * a + 1], br = yb[2 * b], bi = yb[2 * b + 1];
            E[2 * (a * w + b)] += wt * (ar * br - ai * bi);
            E[2 * (a * w + b) + 1] += wt * (ar * bi + ai * br);
          }
      }
    }
    out.insert(out.end(), E.begin(), E.end());
  }
  return out;
}

static void upload(DevBuf& b, const void* src, size_t bytes) {
  b.alloc(bytes);
  BIE_HIP(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
}

template <typename T>
static void upload_vec(DevBuf& b, const std::vector<T>& v) {
  upload(b, v.data(), v.size() * sizeof(T));
}

void require_unit(const bie_ctx* c, const char* what) {
  if (c->poly) throw Error{BIE_EINVAL, std::string(what) + " is built for unit spheres only"};
}

void build(bie_ctx* c, const double* centres, const double* radii, int64_t nb, const bie_opts* o) {
  if (!centres || nb <= 0 || !o) throw Error{BIE_EINVAL, "null centres/opts or no spheres"};
  if (o->p < 1 || o->p > 20) throw Error{BIE_EINVAL, "p must be in [1, 20]"};
  int nphi = o->n_phi > 0 ? o->n_phi : 2 * o->p;
  if (nphi < 2 * o->p || (nphi & 1)) throw Error{BIE_EINVAL, "n_phi must be even and >= 2p"};
  if (nb > 65536) throw Error{BIE_EINVAL, "at most 65536 spheres per context"};
  c->p = o->p;
  c->n_phi = nphi;
  c->mmax = std::min(o->p, nphi / 2 - 1);
  c->nlat = o->p + 1;
  c->P = c->nlat * nphi;
  c->nb = nb;
  c->N = nb * c->P;
  // d* of Eq. 4.5: given, or measured for this grid at the requested precision
  if (!(o->near_gap <= 0.0 || std::isfinite(o->near_gap))) throw Error{BIE_EINVAL, "near_gap must be finite"};
  if (std::isnan(o->near_tol)) throw Error{BIE_EINVAL, "near_tol is NaN"};
  if (o->near_gap > 0) {
    c->near_gap = o->near_gap;
    c->near_tol = 0.0;
  } else {
    c->near_tol = o->near_tol > 0 ? o->near_tol : kDefaultNearTol;
    c->near_gap = near_gap_for(o->p, nphi, c->near_tol);
  }
  if (o->near_method != 0 && o->near_method != 1) throw Error{BIE_EINVAL, "near_method must be 0 or 1"};
  c->near_method = o->near_method;
  if (o->legendre_mfma != 0 && o->legendre_mfma != 1) throw Error{BIE_EINVAL, "legendre_mfma must be 0 or 1"};
  c->legendre_mfma = o->legendre_mfma;
  c->device = o->device;
  c->stream = (hipStream_t)o->hip_stream;
  c->centres.assign(centres, centres + 3 * nb);
  for (double x : c->centres)
    if (!std::isfinite(x)) throw Error{BIE_EINVAL, "non-finite centre coordinate"};
  c->radius.assign(nb, 1.0);
  if (radii) {
    for (int64_t k = 0; k < nb; ++k) {
      const double a = radii[k];
      if (!(a >= 1.0 / 16.0 && a <= 16.0)) throw Error{BIE_EINVAL, "radii must lie in [1/16, 16]"};
      c->radius[k] = a;
    }
  }
  double amax = 0.0;
  c->poly = false;
  for (double a : c->radius) {
    amax = std::max(amax, a);
    if (a != 1.0) c->poly = true;
  }
  const double* rad = c->radius.data();

  // ---- near pairs (Eq. 4.5 as a surface-gap test) with a uniform cell list --------
  // unit spheres: near when |c_t - c_s| - 2 < d*; radii a: when the gap
  // |c_t - c_s| - a_t - a_s is below d* a_s (the source's own length scale).  Close pairs
  // of the learned correction: |c_t - c_s| - 2 < close_gap (unit spheres).  An infinite
  // d* makes every pair near: one cell holds every sphere.
  const bool all_near = !std::isfinite(c->near_gap);
  const double reach = all_near ? 0.0 : std::max(c->near_gap, c->close_gap);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t k = 0; k < nb; ++k)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], centres[3 * k + d]);
      hi[d] = std::max(hi[d], centres[3 * k + d]);
    }
  double cut = (2.0 + reach) * amax;
  // a cell at least 2 a_max wide (overlap test) and at most 2^20 cells per axis
  for (int d = 0; d < 3; ++d) cut = std::max(cut, (hi[d] - lo[d]) / 1048576.0);
  if (all_near) cut = 1e300;
  std::unordered_map<int64_t, std::vector<int>> cells;
  auto key = [](int64_t a, int64_t b, int64_t d) { return (a * 2097152 + b) * 2097152 + d; };
  std::vector<int64_t> cidx(3 * nb);
  for (int64_t k = 0; k < nb; ++k) {
    for (int d = 0; d < 3; ++d)
      cidx[3 * k + d] = all_near ? 0 : (int64_t)std::floor((centres[3 * k + d] - lo[d]) / cut);
    cells[key(cidx[3 * k], cidx[3 * k + 1], cidx[3 * k + 2])].push_back((int)k);
  }
  const double ccut = (2.0 + c->close_gap) * (2.0 + c->close_gap);
  std::vector<std::vector<int>> nbr(nb), cls(nb);
  int64_t total = 0;
  for (int64_t k = 0; k < nb; ++k) {
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          if (all_near && (dx || dy || dz)) continue;
          auto it = cells.find(key(cidx[3 * k] + dx, cidx[3 * k + 1] + dy, cidx[3 * k + 2] + dz));
          if (it == cells.end()) continue;
          for (int s : it->second) {
            if (s == k) continue;
            double ddx = centres[3 * k] - centres[3 * s];
            double ddy = centres[3 * k + 1] - centres[3 * s + 1];
            double ddz = centres[3 * k + 2] - centres[3 * s + 2];
            double d2 = ((ddx * ddx) + (ddy * ddy)) + (ddz * ddz);
            const double rs = rad[k] + rad[s];
            if (d2 < rs * rs)
              throw Error{BIE_EOVERLAP, "spheres " + std::to_string(k) + " and " + std::to_string(s) + " overlap"};
            if (!c->poly && d2 < ccut) cls[k].push_back(s);
            if (all_near || std::sqrt(d2) - rs < c->near_gap * rad[s]) nbr[k].push_back(s);
          }
        }
    std::sort(nbr[k].begin(), nbr[k].end());
    std::sort(cls[k].begin(), cls[k].end());
    total += (int64_t)nbr[k].size();
    if (total > 2000000000)
      throw Error{BIE_EINVAL, "more than 2e9 near pairs at d* = " + std::to_string(c->near_gap) +
                                  ": ask for a larger near_tol or give near_gap"};
  }
  c->near_ptr.assign(nb + 1, 0);
  c->near_idx.clear();
  c->near_idx.reserve((size_t)total);
  c->close_ptr.assign(nb + 1, 0);
  c->close_idx.clear();
  for (int64_t k = 0; k < nb; ++k) {
    c->near_idx.insert(c->near_idx.end(), nbr[k].begin(), nbr[k].end());
    c->near_ptr[k + 1] = (int)c->near_idx.size();
    c->close_idx.insert(c->close_idx.end(), cls[k].begin(), cls[k].end());
    c->close_ptr[k + 1] = (int)c->close_idx.size();
  }
  c->far_node_pairs = (nb * (nb - 1) - total) * (int64_t)c->P * c->P;
  c->nwords = (int)((nb + 31) / 32);
  std::vector<uint32_t> ex((size_t)nb * c->nwords, 0u);
  for (int64_t k = 0; k < nb; ++k) {
    ex[(size_t)k * c->nwords + (k >> 5)] |= 1u << (k & 31);
    for (int s : nbr[k]) ex[(size_t)k * c->nwords + (s >> 5)] |= 1u << (s & 31);
  }

  // ---- grid (Eq. 4.2) and weights (Eq. 4.4) ----------------------------------------
  std::vector<double> tt, ww;
  gauss_legendre(c->nlat, tt, ww);
  c->t = tt;
  c->lam = ww;
  c->theta.resize(c->nlat);
  c->wlat.resize(c->nlat);
  for (int j = 0; j < c->nlat; ++j) {
    c->theta[j] = std::acos(tt[j]);
    c->wlat[j] = 2.0 * M_PI * ww[j] / nphi;
  }
  c->phi.resize(nphi);
  for (int l = 0; l < nphi; ++l) c->phi[l] = 2.0 * M_PI * l / nphi;
  const int P = c->P;
  std::vector<double> otab(4 * P), frame(9 * P), wnode(P);
  std::vector<float> otab_f(4 * P);
  std::vector<double> osrc(4 * P, 0.0);
  std::vector<float> osrc_f(4 * P, 0.0f);
  for (int j = 0; j < c->nlat; ++j) {
    double tj = tt[j], sj = std::sqrt(std::max(0.0, 1.0 - tj * tj));
    for (int l = 0; l < nphi; ++l) {
      int g = j * nphi + l;
      double cp = std::cos(c->phi[l]), sp = std::sin(c->phi[l]);
      double x[3] = {sj * cp, sj * sp, tj};
      for (int d = 0; d < 3; ++d) {
        otab[4 * g + d] = x[d];
        otab_f[4 * g + d] = (float)x[d];
        osrc[4 * g + d] = -2.0 * x[d];   // exact: a power-of-two scaling
        osrc_f[4 * g + d] = -2.0f * (float)x[d];
      }
      otab[4 * g + 3] = 0.0;
      otab_f[4 * g + 3] = 0.0f;
      double fr[9] = {x[0], x[1], x[2], tj * cp, tj * sp, -sj, -sp, cp, 0.0};
      for (int d = 0; d < 9; ++d) frame[9 * g + d] = fr[d];
      wnode[g] = c->wlat[j];
    }
  }

  // ---- transform tables -----------------------------------------------------------
  c->coef_m.clear();
  c->coef_n.clear();
  c->coef_off.assign(c->mmax + 2, 0);
  for (int m = 0; m <= c->mmax; ++m) {
    c->coef_off[m] = (int)c->coef_m.size();
    for (int n = m; n <= c->p; ++n) {
      c->coef_m.push_back(m);
      c->coef_n.push_back(n);
    }
  }
  c->coef_off[c->mmax + 1] = (int)c->coef_m.size();
  c->ncoef = (int)c->coef_m.size();
  const int nc = c->ncoef, nl = c->nlat;
  std::vector<double> leg(3 * (size_t)nc * nl);
  std::vector<double> cp(nc), cd(nc), cq(nc);
  for (int j = 0; j < nl; ++j) {
    double sj = std::sqrt(std::max(0.0, 1.0 - tt[j] * tt[j]));
    legendre_tables(c->p, c->mmax, tt[j], sj, c->coef_m, c->coef_n, cp.data(), cd.data(), cq.data());
    for (int i = 0; i < nc; ++i) {
      leg[(0 * (size_t)nc + i) * nl + j] = cp[i];
      leg[(1 * (size_t)nc + i) * nl + j] = cd[i];
      leg[(2 * (size_t)nc + i) * nl + j] = cq[i];
    }
  }
  std::vector<double> dft((size_t)(c->mmax + 1) * nphi * 2);
  for (int m = 0; m <= c->mmax; ++m)
    for (int l = 0; l < nphi; ++l) {
      double a = 2.0 * M_PI * (double)((m * l) % nphi) / nphi;
      dft[((size_t)m * nphi + l) * 2 + 0] = std::cos(a);
      dft[((size_t)m * nphi + l) * 2 + 1] = std::sin(a);
    }
  std::vector<int> modes(2 * nc);
  for (int i = 0; i < nc; ++i) {
    modes[2 * i] = c->coef_m[i];
    modes[2 * i + 1] = c->coef_n[i];
  }
  std::vector<double> rec = recurrence_table(c->p, c->mmax);
  auto tof = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };

  // ---- device upload (every input has been checked and every host table built) -------
  BIE_HIP(hipSetDevice(c->device));
  std::vector<double> c4(4 * nb);
  for (int64_t k = 0; k < nb; ++k) {
    for (int d = 0; d < 3; ++d) c4[4 * k + d] = centres[3 * k + d];
    c4[4 * k + 3] = 0.0;
  }
  upload_vec(c->centres4, c4);
  if (c->poly) upload_vec(c->radius_d, c->radius);
  upload_vec(c->excl, ex);
  upload_vec(c->dnear_ptr, c->near_ptr);
  upload_vec(c->dnear_idx, c->near_idx.empty() ? std::vector<int>{0} : c->near_idx);
  upload_vec(c->dclose_ptr, c->close_ptr);
  upload_vec(c->dclose_idx, c->close_idx.empty() ? std::vector<int>{0} : c->close_idx);
  upload_vec(c->otab, otab);
  upload_vec(c->otab_f, otab_f);
  upload_vec(c->osrc, osrc);
  upload_vec(c->osrc_f, osrc_f);
  upload_vec(c->frame, frame);
  upload_vec(c->wnode, wnode);
  upload_vec(c->leg, leg);
  upload_vec(c->leg_f, tof(leg));
  upload_vec(c->dft, dft);
  upload_vec(c->dft_f, tof(dft));
  upload_vec(c->wlat_d, c->wlat);
  upload_vec(c->wlat_f, tof(c->wlat));
  upload_vec(c->modes, modes);
  upload_vec(c->rec, rec);
  c->coef.alloc((size_t)nb * 3 * nc * 2 * sizeof(double));
  c->q.alloc((size_t)c->N * 4 * sizeof(double));
  c->moments.alloc((size_t)nb * 6 * sizeof(double));
  c->scal.alloc(262144 * sizeof(double));  // [0,1024) scalars, [1024,...) dot partials, [200000,...) Krylov host-exchange
  // far-field source splits: each launch picks its count (launch_far), up to this capacity
  BIE_HIP(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device));
  c->num_cus = std::max(1, c->num_cus);
  c->nsplit = far_split_capacity(c->N, nb);
  c->partial.alloc((size_t)c->nsplit * c->N * 3 * sizeof(double));
  upload_vec(c->tlat_d, tt);
  if (!c->near_idx.empty()) {
    const std::vector<int> order = near_launch_order(c->near_ptr, nb);
    c->n_near_targets = (int64_t)order.size();
    upload_vec(c->dnear_order, order);
    if (c->near_method == 0) {
      c->near_slots = near_table_slots(c->p, c->mmax);
      c->neartab.alloc((size_t)nb * c->near_slots * 16 * sizeof(double));
    }
  }
  if (c->near_method == 1) {
    upload_vec(c->wig, wigner_x90(c->p));
    c->nearcoef.alloc((size_t)nb * 3 * nc * 2 * sizeof(double));
  }
  build_coarse(c);
  BIE_HIP(hipDeviceSynchronize());
}

}  // namespace bie
