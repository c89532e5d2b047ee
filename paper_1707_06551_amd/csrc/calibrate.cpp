// Separation threshold of Eq. 4.5 from a requested precision.
//
// Eq. 4.5 calls two spheres well separated (smooth quadrature of Eq. 4.4 between them)
// when their distance is at least eta times the larger diameter, and leaves eta to be set
// from the precision the user asks for; for unit spheres that is a surface-gap test
// g >= d* = 2 eta.  The library measures d* for its own grid with the test of Section 6
// (Fig. 5): random densities on one unit sphere, targets on spherical shells at a given
// distance from the surface, the smooth quadrature against the exact exterior potentials
// of Section 3.2, and takes the smallest gap at which the quadrature error stays within
// a tenth of the tolerance.
//
// The measurement (host, float64):
//  - densities: every V, W, X coefficient of degree n <= p and order 0 <= m <= mmax has
//    real and imaginary parts uniform on [-1, 1) (m = 0 real, W_0 = X_0 = 0), the band
//    limit of the grid with a flat spectrum; draw ((d*3 + f)*ncoef + slot)*2 + {0, 1} of
//    a counter-based SplitMix64 stream (Steele, Lea and Flood 2014: output i is the
//    generator's mix of (i + 1) times the golden-ratio increment), top 53 bits;
//  - targets: K = 256 directions of the golden-angle spiral (z_i = 1 - (2i + 1)/K,
//    phi_i = i pi (3 - sqrt 5)) at radius 1 + g;
//  - exact: the exterior series of S and of D (Eqs. 3.6-3.11, series.h);
//  - quadrature: the Stokeslet and the double-layer kernel summed over the grid's nodes
//    with the weights of Eq. 4.4;
//  - error: the largest |quadrature - exact| over both operators, both densities, the
//    targets and the components, divided by the largest |sigma| over the nodes - an error
//    against the density's size, which is how a far pair's error enters a second-kind
//    matvec beside 1/2 mu;
//  - gaps g_k = 2^(k/8) / 64, k = 0..104: from k = 104 down in steps of 8 while the error
//    is <= tol/10, then in steps of 1 below the last passing gap; d* is the last gap that
//    passed, +infinity if the largest one already fails (every pair near).
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "bie_internal.h"
#include "series.h"

namespace bie {

namespace {

constexpr int kDirs = 256;
constexpr int kDens = 2;
constexpr int kGapSteps = 104;

uint64_t splitmix64(uint64_t i) {
  uint64_t z = (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform_pm1(uint64_t i) { return (double)(splitmix64(i) >> 11) * 0x1p-53 * 2.0 - 1.0; }

struct SeriesK {
  int p, mmax, ncoef;
  double kvv[33], kww[33], kwv[33], kxx[33];
};

struct Shell {
  int p, mmax, nphi, nlat, P, nc;
  std::vector<double> node;   // P x 3 unit positions (= normals)
  std::vector<double> wq;     // kDens x P x 3: w * sigma
  std::vector<double> coef;   // kDens x (3 x nc x 2) coefficients in the series layout
  std::vector<double> rec;    // recurrence table of series.h
  std::vector<double> dirs;   // kDirs x 3
  double sigma_max = 0.0;
  SeriesK ks{}, kd{};

  Shell(int p_, int nphi_) : p(p_), nphi(nphi_) {
    mmax = std::min(p, nphi / 2 - 1);
    nlat = p + 1;
    P = nlat * nphi;
    std::vector<int> cm, cn;
    for (int m = 0; m <= mmax; ++m)
      for (int n = m; n <= p; ++n) {
        cm.push_back(m);
        cn.push_back(n);
      }
    nc = (int)cm.size();
    rec = recurrence_table(p, mmax);
    ks.p = kd.p = p;
    ks.mmax = kd.mmax = mmax;
    ks.ncoef = kd.ncoef = nc;
    series_radial(1.0, 0.0, p, ks.kvv, ks.kww, ks.kwv, ks.kxx);
    series_radial(0.0, 1.0, p, kd.kvv, kd.kww, kd.kwv, kd.kxx);

    // coefficients of the test densities
    coef.assign((size_t)kDens * 6 * nc, 0.0);
    for (int d = 0; d < kDens; ++d)
      for (int f = 0; f < 3; ++f)
        for (int i = 0; i < nc; ++i) {
          const uint64_t base = ((uint64_t)(d * 3 + f) * nc + i) * 2;
          double re = uniform_pm1(base), im = uniform_pm1(base + 1);
          if (cm[i] == 0) im = 0.0;
          if (cn[i] == 0 && f > 0) re = im = 0.0;
          coef[(size_t)d * 6 * nc + 2 * (f * nc + i)] = re;
          coef[(size_t)d * 6 * nc + 2 * (f * nc + i) + 1] = im;
        }

    // grid (Eq. 4.2), weights (Eq. 4.4), densities at the nodes by synthesis
    std::vector<double> t, lam;
    gauss_legendre(nlat, t, lam);
    node.assign((size_t)P * 3, 0.0);
    wq.assign((size_t)kDens * P * 3, 0.0);
    std::vector<double> Pb(nc), Db(nc), Qb(nc);
    std::vector<double> sig((size_t)kDens * P * 3, 0.0);
    for (int j = 0; j < nlat; ++j) {
      const double tj = t[j], sj = std::sqrt(std::max(0.0, 1.0 - tj * tj));
      const double wj = 2.0 * M_PI * lam[j] / nphi;
      legendre_tables(p, mmax, tj, sj, cm, cn, Pb.data(), Db.data(), Qb.data());
      for (int l = 0; l < nphi; ++l) {
        const int g = j * nphi + l;
        const double ph = 2.0 * M_PI * l / nphi, cp = std::cos(ph), sp = std::sin(ph);
        const double er[3] = {sj * cp, sj * sp, tj}, et[3] = {tj * cp, tj * sp, -sj}, ep[3] = {-sp, cp, 0.0};
        for (int x = 0; x < 3; ++x) node[3 * g + x] = er[x];
        for (int d = 0; d < kDens; ++d) {
          // spherical components (r, theta, phi) of sum_f sum_slots fac Re(c Z)
          double ur = 0, ut = 0, up = 0;
          const double* cd = &coef[(size_t)d * 6 * nc];
          for (int i = 0; i < nc; ++i) {
            const int m = cm[i], n = cn[i];
            const double a = 2.0 * M_PI * (double)((m * l) % nphi) / nphi;
            const double em_r = std::cos(a), em_i = std::sin(a), fac = m == 0 ? 1.0 : 2.0;
            // Y = Pb e, grad Y = Db e e_theta + i Qb e e_phi (Qb = m Pbar / sin theta)
            const double Yr = Pb[i] * em_r, Yi = Pb[i] * em_i;
            const double Gtr = Db[i] * em_r, Gti = Db[i] * em_i;
            const double Gpr = -Qb[i] * em_i, Gpi = Qb[i] * em_r;
            const double vr = cd[2 * i], vi = cd[2 * i + 1];
            const double wr = cd[2 * (nc + i)], wi = cd[2 * (nc + i) + 1];
            const double xr = cd[2 * (2 * nc + i)], xi = cd[2 * (2 * nc + i) + 1];
            auto re = [](double ar, double ai, double br, double bi) { return ar * br - ai * bi; };
            // V = grad Y - (n+1) Y e_r, W = grad Y + n Y e_r, X = e_r x grad Y
            ur += fac * (-(n + 1.0) * re(vr, vi, Yr, Yi) + n * re(wr, wi, Yr, Yi));
            ut += fac * (re(vr, vi, Gtr, Gti) + re(wr, wi, Gtr, Gti) - re(xr, xi, Gpr, Gpi));
            up += fac * (re(vr, vi, Gpr, Gpi) + re(wr, wi, Gpr, Gpi) + re(xr, xi, Gtr, Gti));
          }
          for (int x = 0; x < 3; ++x) {
            const double s = ur * er[x] + ut * et[x] + up * ep[x];
            sig[((size_t)d * P + g) * 3 + x] = s;
            wq[((size_t)d * P + g) * 3 + x] = wj * s;
            sigma_max = std::max(sigma_max, std::fabs(s));
          }
        }
      }
    }
    dirs.assign(3 * kDirs, 0.0);
    for (int i = 0; i < kDirs; ++i) {
      const double z = 1.0 - (2.0 * i + 1.0) / kDirs, s = std::sqrt(std::max(0.0, 1.0 - z * z));
      const double ph = (i * M_PI) * (3.0 - std::sqrt(5.0));
      dirs[3 * i] = s * std::cos(ph);
      dirs[3 * i + 1] = s * std::sin(ph);
      dirs[3 * i + 2] = z;
    }
  }

  double error(double gap) const {
    const double R = 1.0 + gap, cS = 1.0 / (8.0 * M_PI), cD = 3.0 / (4.0 * M_PI);
    double e = 0.0;
    for (int i = 0; i < kDirs; ++i) {
      const double x[3] = {R * dirs[3 * i], R * dirs[3 * i + 1], R * dirs[3 * i + 2]};
      for (int d = 0; d < kDens; ++d) {
        double qs[3] = {0, 0, 0}, qd[3] = {0, 0, 0};
        const double* w = &wq[(size_t)d * P * 3];
        for (int g = 0; g < P; ++g) {
          const double r[3] = {x[0] - node[3 * g], x[1] - node[3 * g + 1], x[2] - node[3 * g + 2]};
          const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
          const double ir = 1.0 / std::sqrt(r2), ir2 = ir * ir;
          const double rq = r[0] * w[3 * g] + r[1] * w[3 * g + 1] + r[2] * w[3 * g + 2];
          const double rn = r[0] * node[3 * g] + r[1] * node[3 * g + 1] + r[2] * node[3 * g + 2];
          for (int k = 0; k < 3; ++k) {
            qs[k] += cS * (w[3 * g + k] * ir + r[k] * rq * ir * ir2);
            qd[k] += cD * r[k] * rq * rn * ir2 * ir2 * ir;
          }
        }
        double es[3] = {0, 0, 0}, ed[3] = {0, 0, 0};
        const double* cd = &coef[(size_t)d * 6 * nc];
        exterior_series(ks, cd, rec.data(), x[0], x[1], x[2], es[0], es[1], es[2]);
        exterior_series(kd, cd, rec.data(), x[0], x[1], x[2], ed[0], ed[1], ed[2]);
        for (int k = 0; k < 3; ++k) e = std::max(e, std::max(std::fabs(qs[k] - es[k]), std::fabs(qd[k] - ed[k])));
      }
    }
    return e / sigma_max;
  }
};

double gap_grid(int k) { return std::pow(2.0, k / 8.0) / 64.0; }

}  // namespace

double near_gap_for(int p, int n_phi, double tol) {
  if (p < 1 || p > 20) throw Error{BIE_EINVAL, "p must be in [1, 20]"};
  const int nphi = n_phi > 0 ? n_phi : 2 * p;
  if (nphi < 2 * p || (nphi & 1)) throw Error{BIE_EINVAL, "n_phi must be even and >= 2p"};
  if (!(tol > 0.0 && tol < 1.0)) throw Error{BIE_EINVAL, "near_tol must lie in (0, 1)"};
  static std::mutex mu;
  static std::map<std::tuple<int, int, double>, double> cache;
  const auto key = std::make_tuple(p, nphi, tol);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const Shell sh(p, nphi);
  const double target = tol / 10.0;
  double d = INFINITY;
  int k = kGapSteps;
  if (sh.error(gap_grid(k)) <= target) {
    while (k - 8 >= 0 && sh.error(gap_grid(k - 8)) <= target) k -= 8;
    while (k - 1 >= 0 && sh.error(gap_grid(k - 1)) <= target) k -= 1;
    d = gap_grid(k);
  }
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = d;
  return d;
}

}  // namespace bie
