// Host-side checks of the set-up and validation code of the library, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host pass
// (tests/test_host_sanitize.py compiles every library source and this driver).  Needs no
// GPU: bie::build does all of its host work (input checks, near and close pair lists of
// Eq. 4.5, grid and transform tables, the separation threshold) before its first device
// call, so without a device it ends in BIE_EDEVICE with the host state in place.
//
// Checks: near / close lists and the far node-pair count against brute force on random
// suspensions (unit spheres and spheres of several radii, several d*), a 65536-sphere
// lattice against its closed-form neighbour count, overlap and non-finite-centre
// rejection, every option bound, the separation threshold over all orders, and the
// solver's option checks.  Prints one line per failure; exit status = failures.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "bie_internal.h"

namespace bie {
void build(bie_ctx* c, const double* centres, const double* radii, int64_t nb, const bie_opts* o);
}

static int g_fail = 0;
#define CHECK(cond, ...)                                               \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "FAIL line %d: ", __LINE__);                \
      std::fprintf(stderr, __VA_ARGS__);                               \
      std::fprintf(stderr, "\n");                                      \
      ++g_fail;                                                        \
    }                                                                  \
  } while (0)

static bie_opts opts(int p, double near_gap, double near_tol = 0.0) {
  bie_opts o{};
  o.p = p;
  o.n_phi = 0;
  o.near_gap = near_gap;
  o.device = 0;
  o.hip_stream = nullptr;
  o.near_method = 0;
  o.legendre_mfma = 0;
  o.near_tol = near_tol;
  return o;
}

// the host part of bie::build: 0 (device present) or BIE_EDEVICE (none) mean it passed
static int build_host(bie_ctx& c, const std::vector<double>& cen, const std::vector<double>* rad, const bie_opts& o,
                      int64_t nb = -1) {
  try {
    bie::build(&c, cen.data(), rad ? rad->data() : nullptr, nb >= 0 ? nb : (int64_t)cen.size() / 3, &o);
    return 0;
  } catch (const bie::Error& e) {
    return e.code;
  }
}

static bool host_ok(int rc) { return rc == 0 || rc == BIE_EDEVICE; }

// random sequential addition in a cube of side L, surface gap >= gmin
static void place(int n, double L, double gmin, const std::vector<double>& rad, std::mt19937_64& rng,
                  std::vector<double>& cen) {
  std::uniform_real_distribution<double> U(0.0, 1.0);
  cen.clear();
  for (int k = 0; k < n; ++k) {
    for (int tries = 0;; ++tries) {
      if (tries > 1000000) {
        std::fprintf(stderr, "placement stalled\n");
        std::exit(99);
      }
      double x[3];
      for (int d = 0; d < 3; ++d) x[d] = rad[k] + (L - 2 * rad[k]) * U(rng);
      bool ok = true;
      for (int j = 0; j < k && ok; ++j) {
        const double dx = x[0] - cen[3 * j], dy = x[1] - cen[3 * j + 1], dz = x[2] - cen[3 * j + 2];
        ok = std::sqrt(dx * dx + dy * dy + dz * dz) - rad[j] - rad[k] >= gmin;
      }
      if (ok) {
        cen.insert(cen.end(), x, x + 3);
        break;
      }
    }
  }
}

static void check_lists(const bie_ctx& c, const std::vector<double>& cen, const std::vector<double>& rad,
                        const char* what) {
  const int64_t nb = (int64_t)rad.size();
  int64_t total = 0;
  bool unit = true;
  for (double a : rad) unit = unit && a == 1.0;
  for (int64_t t = 0; t < nb; ++t) {
    std::vector<int> near, close;
    for (int64_t s = 0; s < nb; ++s) {
      if (s == t) continue;
      const double dx = cen[3 * t] - cen[3 * s], dy = cen[3 * t + 1] - cen[3 * s + 1], dz = cen[3 * t + 2] - cen[3 * s + 2];
      const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
      if (!std::isfinite(c.near_gap) || d - rad[t] - rad[s] < c.near_gap * rad[s]) near.push_back((int)s);
      if (unit && d - 2.0 < c.close_gap) close.push_back((int)s);
    }
    const std::vector<int> got(c.near_idx.begin() + c.near_ptr[t], c.near_idx.begin() + c.near_ptr[t + 1]);
    CHECK(got == near, "%s: near list of sphere %lld (%zu vs %zu entries)", what, (long long)t, got.size(), near.size());
    if (unit) {
      const std::vector<int> gc(c.close_idx.begin() + c.close_ptr[t], c.close_idx.begin() + c.close_ptr[t + 1]);
      CHECK(gc == close, "%s: close list of sphere %lld", what, (long long)t);
    }
    total += (int64_t)near.size();
  }
  CHECK(c.far_node_pairs == (nb * (nb - 1) - total) * (int64_t)c.P * c.P, "%s: far node pairs", what);
}

int main() {
  std::mt19937_64 rng(12345);
  // ---- near lists against brute force ------------------------------------------
  const int sizes[] = {1, 2, 17, 300, 1500};
  const double gaps[] = {0.05, 1.0, 4.0, 58.7};
  for (int n : sizes)
    for (double dstar : gaps) {
      std::vector<double> rad(n, 1.0), cen;
      const double L = std::cbrt(n * 4.18879 / 0.2) + 2.0;
      place(n, L, 0.02, rad, rng, cen);
      bie_ctx c;
      const int rc = build_host(c, cen, nullptr, opts(6, dstar));
      CHECK(host_ok(rc), "unit n=%d d*=%g: rc %d", n, dstar, rc);
      if (host_ok(rc)) check_lists(c, cen, rad, "unit spheres");
    }
  for (int n : {5, 60, 400}) {
    std::uniform_real_distribution<double> U(0.3, 2.0);
    std::vector<double> rad(n), cen;
    for (double& a : rad) a = U(rng);
    place(n, std::cbrt(n * 30.0) + 6.0, 0.05, rad, rng, cen);
    for (double dstar : {0.5, 2.0}) {
      bie_ctx c;
      const int rc = build_host(c, cen, &rad, opts(5, dstar));
      CHECK(host_ok(rc), "radii n=%d: rc %d", n, rc);
      if (host_ok(rc)) check_lists(c, cen, rad, "radii");
    }
  }
  // calibrated d* (near_gap <= 0): the list follows the measured threshold
  {
    std::vector<double> rad(200, 1.0), cen;
    place(200, 22.0, 0.02, rad, rng, cen);
    bie_ctx c;
    const int rc = build_host(c, cen, nullptr, opts(12, 0.0, 1e-8));
    CHECK(host_ok(rc) && c.near_gap == bie::near_gap_for(12, 24, 1e-8) && c.near_tol == 1e-8, "calibrated d*");
    if (host_ok(rc)) check_lists(c, cen, rad, "calibrated");
  }
  // ---- 65536 spheres on a 32 x 32 x 64 lattice of spacing 2.5: face neighbours only --
  {
    std::vector<double> cen;
    for (int i = 0; i < 32; ++i)
      for (int j = 0; j < 32; ++j)
        for (int k = 0; k < 64; ++k) {
          cen.push_back(2.5 * i);
          cen.push_back(2.5 * j);
          cen.push_back(2.5 * k);
        }
    bie_ctx c;
    const int rc = build_host(c, cen, nullptr, opts(2, 1.0));
    CHECK(host_ok(rc), "lattice rc %d", rc);
    const int64_t faces = 2 * (31LL * 32 * 64 + 32LL * 31 * 64 + 32LL * 32 * 63);
    CHECK((int64_t)c.near_idx.size() == faces, "lattice near pairs %zu vs %lld", c.near_idx.size(), (long long)faces);
    std::vector<double> one(3 * 65537, 0.0);
    bie_ctx c2;
    CHECK(build_host(c2, one, nullptr, opts(2, 1.0), 65537) == BIE_EINVAL, "65537 spheres accepted");
  }
  // ---- overlaps and non-finite centres --------------------------------------------
  for (double base : {0.0, 1e6, -3e7}) {
    std::vector<double> cen = {base, base, base, base + 1.999, base, base, base + 9.0, base, base};
    bie_ctx c;
    CHECK(build_host(c, cen, nullptr, opts(4, 1.0)) == BIE_EOVERLAP, "overlap at %g", base);
    std::vector<double> touching = {base, base, base, base + 2.0, base, base};
    bie_ctx c2;
    CHECK(host_ok(build_host(c2, touching, nullptr, opts(4, 1.0))), "touching spheres at %g rejected", base);
  }
  {
    // an overlapping pair deep inside a larger suspension (found through the cell list)
    std::vector<double> rad(300, 1.0), cen;
    place(300, 30.0, 0.1, rad, rng, cen);
    cen[3 * 150] = cen[3 * 77] + 1.5;
    cen[3 * 150 + 1] = cen[3 * 77 + 1];
    cen[3 * 150 + 2] = cen[3 * 77 + 2];
    bie_ctx c;
    CHECK(build_host(c, cen, nullptr, opts(4, 1.0)) == BIE_EOVERLAP, "hidden overlap");
    std::vector<double> radii = {1.0, 0.5, 1.0};
    std::vector<double> cp = {0, 0, 0, 1.4, 0, 0, 10, 0, 0};
    bie_ctx c3;
    CHECK(build_host(c3, cp, &radii, opts(4, 1.0)) == BIE_EOVERLAP, "overlap with radii");
  }
  for (double bad : {(double)NAN, (double)INFINITY, -(double)INFINITY}) {
    std::vector<double> cen = {0, 0, 0, 5, bad, 0};
    bie_ctx c;
    CHECK(build_host(c, cen, nullptr, opts(4, 1.0)) == BIE_EINVAL, "non-finite centre %g accepted", bad);
  }
  {
    std::vector<double> cen = {0, 0, 0, 5, 0, 0};
    for (double a : {0.0, -1.0, 0.01, 17.0, (double)NAN}) {
      std::vector<double> rad = {1.0, a};
      bie_ctx c;
      CHECK(build_host(c, cen, &rad, opts(4, 1.0)) == BIE_EINVAL, "radius %g accepted", a);
    }
  }
  // ---- option bounds -----------------------------------------------------------------
  {
    std::vector<double> cen = {0, 0, 0, 4, 0, 0};
    struct Case {
      int p, nphi, method, mfma;
      double gap, tol;
      int want;  // 1 = accepted
    };
    const Case cases[] = {{0, 0, 0, 0, 1, 0, 0},     {21, 0, 0, 0, 1, 0, 0},   {1, 0, 0, 0, 1, 0, 1},
                          {20, 0, 0, 0, 1, 0, 1},    {4, 7, 0, 0, 1, 0, 0},    {4, 6, 0, 0, 1, 0, 0},
                          {4, 8, 0, 0, 1, 0, 1},     {4, 10, 0, 0, 1, 0, 1},   {8, 120, 0, 0, 1, 0, 1},
                          {16, 64, 0, 0, 1, 0, 1},   {4, 0, 2, 0, 1, 0, 0},    {4, 0, -1, 0, 1, 0, 0},
                          {4, 0, 1, 0, 1, 0, 1},     {4, 0, 0, 2, 1, 0, 0},    {4, 0, 0, 1, 1, 0, 1},
                          {4, 0, 0, 0, INFINITY, 0, 0}, {4, 0, 0, 0, NAN, 0, 0}, {4, 0, 0, 0, 0, NAN, 0},
                          {4, 0, 0, 0, 0, 2.0, 0},   {4, 0, 0, 0, -1, 1e-6, 1}, {4, 0, 0, 0, 0, 1e-300, 1}};
    for (const Case& k : cases) {
      bie_opts o = opts(k.p, k.gap, k.tol);
      o.n_phi = k.nphi;
      o.near_method = k.method;
      o.legendre_mfma = k.mfma;
      bie_ctx c;
      const int rc = build_host(c, cen, nullptr, o);
      CHECK(k.want ? host_ok(rc) : rc == BIE_EINVAL, "p %d n_phi %d method %d mfma %d gap %g tol %g: rc %d", k.p,
            k.nphi, k.method, k.mfma, k.gap, k.tol, rc);
    }
    bie_ctx c;
    CHECK(build_host(c, cen, nullptr, opts(4, 1.0), 0) == BIE_EINVAL, "no spheres accepted");
  }
  // ---- separation threshold ---------------------------------------------------------------
  for (int p = 1; p <= 20; ++p) {
    double prev = 0.0;
    for (double tol : {1e-3, 1e-6, 1e-9, 1e-12}) {
      double d = -1.0;
      try {
        d = bie::near_gap_for(p, 0, tol);
      } catch (const bie::Error& e) {
        CHECK(false, "near_gap_for(%d, %g) threw %s", p, tol, e.msg.c_str());
      }
      CHECK(d > 0.0 && d >= prev, "d*(%d, %g) = %g not increasing", p, tol, d);
      prev = d;
    }
  }
  for (double tol : {0.0, 1.0, -1e-8, (double)NAN}) {
    bool threw = false;
    try {
      bie::near_gap_for(4, 0, tol);
    } catch (const bie::Error& e) {
      threw = e.code == BIE_EINVAL;
    }
    CHECK(threw, "near_gap_for accepted tol %g", tol);
  }
  // ---- solver option checks (before any device use) -----------------------------------
  {
    std::vector<double> cen = {0, 0, 0, 4, 0, 0};
    bie_ctx c;
    build_host(c, cen, nullptr, opts(4, 1.0));
    struct SCase {
      int restart, precond, cap;
      bool hist;
    };
    for (SCase k : {SCase{501, BIE_PC_M0, 0, false}, SCase{100, 7, 0, false}, SCase{100, BIE_PC_RIGID, 0, false},
                    SCase{100, BIE_PC_MLP, 0, false}, SCase{100, BIE_PC_M0, -1, true}}) {
      bie_solve_opts so{};
      so.tol = 1e-8;
      so.restart = k.restart;
      so.precond = k.precond;
      double h[4];
      so.res_hist = k.hist ? h : nullptr;
      so.res_hist_cap = k.cap;
      int code = 0;
      try {
        bie::solve(&c, BIE_OP_DN_BIE, nullptr, nullptr, 3 * c.N, &so, nullptr);
      } catch (const bie::Error& e) {
        code = e.code;
      }
      CHECK(code == BIE_EINVAL, "solve accepted restart %d precond %d cap %d (rc %d)", k.restart, k.precond, k.cap,
            code);
    }
  }
  std::printf("host checks: %d failure(s)\n", g_fail);
  return g_fail;
}
