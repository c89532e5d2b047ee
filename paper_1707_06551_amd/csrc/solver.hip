// Krylov solver for the second-kind equations of Section 5 (the paper names no solver):
// restarted, right-preconditioned flexible GMRES with classical Gram-Schmidt applied
// twice (CGS2) on the device in float64, Givens rotations on the host.  One device ->
// host transfer (k+1 Hessenberg entries and a norm) per Arnoldi step.  Mixed precision
// is iterative refinement: float64 residual b - A x, inner GMRES on the correction with
// float32 transforms and far-field sums, x += d.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "bie_internal.h"

namespace bie {

static constexpr int DOT_BLOCKS = 240;

__global__ void k_dot_many(const double* V, int64_t ld, const double* w, int64_t n, double* partial) {
  const int i = blockIdx.y;
  const double* v = V + (int64_t)i * ld;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    s += v[e] * w[e];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)i * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_finish(const double* partial, int nblk, double* out) {
  const int i = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[(int64_t)i * nblk + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// w -= sum_i h[i] V_i  (sign = -1) or w += sum_i h[i] V_i (sign = +1)
__global__ void k_gemv(const double* V, int64_t ld, int k, const double* h, double sign, double* w, int64_t n) {
  __shared__ double hs[512];
  for (int i = threadIdx.x; i < k; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += hs[i] * V[(int64_t)i * ld + e];
    w[e] += sign * s;
  }
}

__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + (b == 0.0 ? 0.0 : b * y[e]);
}

__global__ void k_scale_inv_sqrt(const double* x, const double* nrm2, double* y, int64_t n) {
  const double s = 1.0 / sqrt(*nrm2);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = x[e] * s;
}

__global__ void k_fill(double* y, double v, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) y[e] = v;
}

// b = v_k + omega_k x (x - c_k) at every node (x - c_k = unit offset of the node)
__global__ void k_rigid(const double* v, const double* om, const double* otab, int P, int64_t N, double* b) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / P;
    const int li = (int)(g - k * P);
    const double ox = otab[4 * li], oy = otab[4 * li + 1], oz = otab[4 * li + 2];
    const double* vk = v + 3 * k;
    const double* wk = om + 3 * k;
    b[3 * g] = vk[0] + (wk[1] * oz - wk[2] * oy);
    b[3 * g + 1] = vk[1] + (wk[2] * ox - wk[0] * oz);
    b[3 * g + 2] = vk[2] + (wk[0] * oy - wk[1] * ox);
  }
}

static int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

void dev_axpby(bie_ctx* c, double a, const double* x, double b, double* y, int64_t n) {
  k_axpby<<<grid_for(n), 256, 0, c->stream>>>(a, x, b, y, n);
  BIE_HIP(hipGetLastError());
}
void dev_copy(bie_ctx* c, const double* x, double* y, int64_t n) {
  BIE_HIP(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
}
void dev_fill(bie_ctx* c, double* y, double v, int64_t n) {
  k_fill<<<grid_for(n), 256, 0, c->stream>>>(y, v, n);
  BIE_HIP(hipGetLastError());
}
void dev_rigid_rhs(bie_ctx* c, const double* v, const double* om, double* b) {
  k_rigid<<<grid_for(c->N), 256, 0, c->stream>>>(v, om, c->otab.as<double>(), c->P, c->N, b);
  BIE_HIP(hipGetLastError());
}

// dots of w with k vectors V_i -> dev_out[0..k) (device), stream ordered
static void dots_dev(bie_ctx* c, const double* V, int64_t ld, int k, const double* w, int64_t n, double* dev_out) {
  double* partial = c->scal.as<double>() + 1024;
  k_dot_many<<<dim3(DOT_BLOCKS, k), 256, 0, c->stream>>>(V, ld, w, n, partial);
  BIE_HIP(hipGetLastError());
  k_finish<<<k, 256, 0, c->stream>>>(partial, DOT_BLOCKS, dev_out);
  BIE_HIP(hipGetLastError());
}

double dev_norm(bie_ctx* c, const double* x, int64_t n) {
  double* d = c->scal.as<double>();
  dots_dev(c, x, 0, 1, x, n, d);
  double h = 0.0;
  BIE_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  BIE_HIP(hipStreamSynchronize(c->stream));
  return std::sqrt(h);
}

StageScope::StageScope(bie_ctx* c, int stage) : c_(c) {
  StageTimer& t = c->timer;
  if (!t.on || t.depth++ > 0) return;
  if (2 * (t.used + 1) > t.ev.size()) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return;
    }
    t.ev.push_back(e0);
    t.ev.push_back(e1);
  }
  if (t.tag.size() <= t.used) t.tag.resize(t.used + 1);
  t.tag[t.used] = stage;
  rec_ = hipEventRecord(t.ev[2 * t.used], c->stream) == hipSuccess;
}

StageScope::~StageScope() {
  StageTimer& t = c_->timer;
  if (t.depth > 0) --t.depth;
  if (!rec_) return;
  if (hipEventRecord(t.ev[2 * t.used + 1], c_->stream) == hipSuccess) ++t.used;
}

void timer_start(bie_ctx* c) {
  c->timer.on = true;
  c->timer.depth = 0;
  c->timer.used = 0;
  c->timer.far_pairs = 0;
  c->timer.near_evals = 0;
}

void timer_collect(bie_ctx* c, double t[8]) {
  StageTimer& tm = c->timer;
  for (int i = 0; i < 8; ++i) t[i] = 0.0;
  tm.on = false;
  if (tm.used == 0) return;
  BIE_HIP(hipEventSynchronize(tm.ev[2 * tm.used - 1]));
  for (size_t i = 0; i < tm.used; ++i) {
    float ms = 0.0f;
    BIE_HIP(hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]));
    t[tm.tag[i] & 7] += 1e-3 * ms;
  }
  tm.used = 0;
}

void timer_release(bie_ctx* c) {
  for (hipEvent_t e : c->timer.ev) (void)hipEventDestroy(e);
  c->timer.ev.clear();
  c->timer.tag.clear();
  c->timer.used = 0;
  c->timer.on = false;
}

namespace {

struct Krylov {
  bie_ctx* c;
  int64_t n;
  int m;  // restart length
  bool flexible;
  double* V;
  double* Z;
  double* w;
  double* hdev;  // device: [h1 (m+1) | h2 (m+1) | nrm2]
};

// Operator application used by the solver: y = A M x (M = preconditioner or identity)
struct OpCtx {
  bie_ctx* c;
  int op;           // BIE_OP_DN_BIE, BIE_OP_MOBILITY, BIE_OP_SD_BIE or BIE_OP_KL_BIE
  int precision;    // matvec precision inside this Krylov solve
  int precond;      // BIE_PC_*
  int* matvecs64;
  int* matvecs32;
};

void apply_A(const OpCtx& o, const double* x, double* y) {
  apply(o.c, o.op, o.precision, x, y);
  if (o.precision == BIE_MIXED)
    ++*o.matvecs32;
  else
    ++*o.matvecs64;
}

void apply_M(const OpCtx& o, const double* x, double* z, int64_t n) {
  (void)n;
  StageScope ts(o.c, BIE_T_PRECOND);
  apply_precond(o.c, o.op, o.precision, o.precond, x, z);
}

// One flexible GMRES solve of A d = r from d = 0 to relative tolerance tol (estimate);
// returns iterations used, writes d.  best-effort on stagnation (max_it reached).
int fgmres(const OpCtx& o, Krylov& K, const double* r, double rnorm, double tol, int max_it, double* d,
           std::vector<double>* hist, double hist_den, bool* bad) {
  bie_ctx* c = o.c;
  const int64_t n = K.n;
  const int m = K.m;
  *bad = false;
  {
    StageScope ts(c, BIE_T_KRYLOV);
    dev_fill(c, d, 0.0, n);
  }
  if (rnorm == 0.0) return 0;
  int it = 0;
  double cur = rnorm;
  const double* rr = r;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hh(2 * (m + 1) + 1), ests;
  while (it < max_it) {
    // V_0 = current residual / its norm.  First cycle: r; later cycles: r - A d.
    if (rr == r) {
      StageScope ts(c, BIE_T_KRYLOV);
      dev_axpby(c, 1.0 / cur, r, 0.0, K.V, n);
    } else {
      apply_A(o, d, K.w);  // d is already in solution space (d = Z y), so plain A
      StageScope ts(c, BIE_T_KRYLOV);
      dev_axpby(c, 1.0, r, -1.0, K.w, n);
      cur = dev_norm(c, K.w, n);
      if (cur <= tol * rnorm) break;
      dev_axpby(c, 1.0 / cur, K.w, 0.0, K.V, n);
    }
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = cur;
    int j = 0;
    bool done = false;
    for (; j < m && it < max_it; ++j) {
      double* vj = K.V + (int64_t)j * n;
      double* zj = K.flexible ? K.Z + (int64_t)j * n : vj;
      if (K.flexible) apply_M(o, vj, zj, n);
      apply_A(o, zj, K.w);
      StageScope ts(c, BIE_T_KRYLOV);
      // CGS2
      dots_dev(c, K.V, n, j + 1, K.w, n, K.hdev);
      k_gemv<<<grid_for(n), 256, 0, c->stream>>>(K.V, n, j + 1, K.hdev, -1.0, K.w, n);
      dots_dev(c, K.V, n, j + 1, K.w, n, K.hdev + (m + 1));
      k_gemv<<<grid_for(n), 256, 0, c->stream>>>(K.V, n, j + 1, K.hdev + (m + 1), -1.0, K.w, n);
      dots_dev(c, K.w, n, 1, K.w, n, K.hdev + 2 * (m + 1));
      k_scale_inv_sqrt<<<grid_for(n), 256, 0, c->stream>>>(K.w, K.hdev + 2 * (m + 1), K.V + (int64_t)(j + 1) * n, n);
      BIE_HIP(hipGetLastError());
      BIE_HIP(hipMemcpyAsync(hh.data(), K.hdev, (2 * (m + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      BIE_HIP(hipStreamSynchronize(c->stream));
      double* Hj = &H[(size_t)j * (m + 1)];
      for (int i = 0; i <= j; ++i) Hj[i] = hh[i] + hh[(m + 1) + i];
      Hj[j + 1] = std::sqrt(std::max(0.0, hh[2 * (m + 1)]));
      for (int i = 0; i < j; ++i) {
        const double a0 = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
        const double a1 = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
        Hj[i] = a0;
        Hj[i + 1] = a1;
      }
      const double den = std::hypot(Hj[j], Hj[j + 1]);
      cs[j] = den > 0 ? Hj[j] / den : 1.0;
      sn[j] = den > 0 ? Hj[j + 1] / den : 0.0;
      Hj[j] = den;
      Hj[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      const double est = std::fabs(g[j + 1]);
      if (!std::isfinite(est) || !std::isfinite(den)) {
        *bad = true;
        return it;
      }
      // stagnation of a preconditioned solve: less than 10% reduction in 20 steps
      if (K.flexible) {
        ests.push_back(est);
        const size_t q = ests.size();
        if (q > 20 && ests[q - 1] > 0.9 * ests[q - 21]) {
          *bad = true;
          return it;
        }
      }
      if (hist) hist->push_back(est / hist_den);
      if (est <= tol * rnorm || den == 0.0) {
        ++j;
        done = true;
        break;
      }
    }
    // back substitution and update d += Z y
    const int kk = j;
    std::vector<double> y(kk);
    for (int i = kk - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < kk; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    StageScope ts(c, BIE_T_KRYLOV);
    double* ydev = K.hdev + 2 * (m + 1) + 8;
    BIE_HIP(hipMemcpyAsync(ydev, y.data(), kk * sizeof(double), hipMemcpyHostToDevice, c->stream));
    k_gemv<<<grid_for(n), 256, 0, c->stream>>>(K.flexible ? K.Z : K.V, n, kk, ydev, +1.0, d, n);
    BIE_HIP(hipGetLastError());
    BIE_HIP(hipStreamSynchronize(c->stream));
    if (done) break;
    rr = nullptr;  // restart from the true residual of the current d
  }
  return it;
}

}  // namespace

// Solves A x = b (b, x device, length n).  Returns BIE_OK or BIE_ENOCONV.
int solve(bie_ctx* c, int op, const double* b, double* x, int64_t n, const bie_solve_opts* so, bie_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  bie_solve_opts o{};
  if (so) o = *so;
  if (!(o.tol > 0)) o.tol = 1e-8;
  if (o.restart <= 0) o.restart = 100;
  if (o.max_iter <= 0) o.max_iter = 1000;
  if (!(o.inner_tol > 0)) o.inner_tol = 1e-4;
  if (o.restart > 500) throw Error{BIE_EINVAL, "restart must be <= 500"};
  if (o.res_hist && o.res_hist_cap < 0) throw Error{BIE_EINVAL, "res_hist_cap must be >= 0"};
  const int pc_base = o.precond & ~(BIE_PC_RIGID | BIE_PC_LOCAL);
  if ((o.precond & BIE_PC_LOCAL) && pc_base != BIE_PC_MLP) throw Error{BIE_EINVAL, "BIE_PC_LOCAL modifies BIE_PC_MLP only"};
  if (pc_base == BIE_PC_MLP && !c->theta_ready) throw Error{BIE_EINVAL, "BIE_PC_MLP needs bie_precond_load first"};
  if (pc_base < BIE_PC_NONE || pc_base > BIE_PC_MLP) throw Error{BIE_EINVAL, "unknown preconditioner"};
  if ((o.precond & BIE_PC_RIGID) && pc_base == BIE_PC_NONE)
    throw Error{BIE_EINVAL, "BIE_PC_RIGID needs BIE_PC_M0 or BIE_PC_MLP"};
  const int m = o.restart;
  const bool flexible = o.precond != BIE_PC_NONE;
  // work space
  if (c->krylov_cols < m + 1 || c->krylov_n != n) {
    c->krylov.alloc((size_t)(m + 1) * n * sizeof(double));
    c->zbasis.alloc(flexible ? (size_t)m * n * sizeof(double) : 16);
    c->krylov_cols = m + 1;
    c->krylov_n = n;
    for (int i = 0; i < 4; ++i) c->vec[i].alloc(n * sizeof(double));
  } else if (flexible && c->zbasis.bytes < (size_t)m * n * sizeof(double)) {
    c->zbasis.alloc((size_t)m * n * sizeof(double));
  }
  Krylov K{c, n, m, flexible, c->krylov.as<double>(), c->zbasis.as<double>(), c->vec[0].as<double>(),
           c->scal.as<double>() + 200000};
  double* r = c->vec[1].as<double>();
  double* d = c->vec[2].as<double>();
  int mv64 = 0, mv32 = 0;
  if (info) timer_start(c);
  std::vector<double> hist;
  std::vector<double>* hp = (o.res_hist && o.res_hist_cap > 0) ? &hist : nullptr;
  double bnorm;
  {
    StageScope ts(c, BIE_T_KRYLOV);
    bnorm = dev_norm(c, b, n);
    if (o.x0) {
      if (o.x0 != x) dev_copy(c, o.x0, x, n);
    } else {
      dev_fill(c, x, 0.0, n);
    }
  }
  int iters = 0, outer = 0, fallback = 0;
  bool fallback_failed = false;
  double rel = 0.0;
  int status = BIE_ENOCONV;
  if (bnorm == 0.0) {
    // b = 0: the solution is 0 whatever the initial guess
    if (o.x0) {
      StageScope ts(c, BIE_T_KRYLOV);
      dev_fill(c, x, 0.0, n);
    }
    status = BIE_OK;
  } else {
    OpCtx op64{c, op, BIE_FP64, o.precond, &mv64, &mv32};
    OpCtx opin{c, op, o.precision, o.precond, &mv64, &mv32};
    bool first = o.x0 == nullptr;
    while (iters < o.max_iter) {
      // r = b - A x (float64)
      double rn;
      if (first) {
        StageScope ts(c, BIE_T_KRYLOV);
        dev_copy(c, b, r, n);
        rn = bnorm;
      } else {
        apply_A(op64, x, r);
        StageScope ts(c, BIE_T_KRYLOV);
        dev_axpby(c, 1.0, b, -1.0, r, n);
        rn = dev_norm(c, r, n);
      }
      rel = rn / bnorm;
      if (!std::isfinite(rel)) break;
      if (rel <= o.tol) {
        status = BIE_OK;
        break;
      }
      first = false;
      ++outer;
      // inner tolerance: refinement asks for inner_tol, a float64 solve for the target
      double itol = (o.precision == BIE_MIXED) ? std::max(o.inner_tol, 0.5 * o.tol / rel) : 0.7 * o.tol / rel;
      bool bad = false;
      iters += fgmres(fallback ? op64 : opin, K, r, rn, itol, o.max_iter - iters, d, hp, bnorm, &bad);
      if (bad) {
        if (fallback) {
          fallback_failed = true;
          break;
        }
        // stagnation / non-finite values: restart plain float64 GMRES from x
        fallback = 1;
        opin.precond = BIE_PC_NONE;
        opin.precision = BIE_FP64;
        K.flexible = false;
        continue;
      }
      {
        StageScope ts(c, BIE_T_KRYLOV);
        dev_axpby(c, 1.0, d, 1.0, x, n);
      }
      if (o.precision != BIE_MIXED && outer > 50) break;
    }
    if (status != BIE_OK && iters > 0 && !fallback_failed) {
      // not converged: report the true residual of the returned iterate
      apply_A(op64, x, r);
      StageScope ts(c, BIE_T_KRYLOV);
      dev_axpby(c, 1.0, b, -1.0, r, n);
      rel = dev_norm(c, r, n) / bnorm;
    }
  }
  BIE_HIP(hipStreamSynchronize(c->stream));
  if (info) {
    info->iters = iters;
    info->outer_steps = outer;
    info->matvecs_fp64 = mv64;
    info->matvecs_mixed = mv32;
    info->fallback_used = fallback;
    info->rel_residual = rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    timer_collect(c, info->t_stage_s);
    info->pairs_evaluated = c->timer.far_pairs;
    info->near_evals = c->timer.near_evals;
    info->res_hist_len = 0;
  }
  if (hp) {
    const int k = (int)std::min<size_t>(hist.size(), (size_t)o.res_hist_cap);
    std::memcpy(o.res_hist, hist.data(), k * sizeof(double));
    if (info) info->res_hist_len = k;
  }
  return status;
}

}  // namespace bie
