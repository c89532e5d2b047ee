// Internal declarations of the MI355X sphere-BIE library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bie.h"

namespace bie {

// Thread-local error text behind bie_last_error().
void set_error(const std::string& msg);
void clear_error();

struct Error {
  int code;
  std::string msg;
};

#define BIE_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::bie::Error{BIE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)};    \
  } while (0)

// Device buffer owned by a context.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t n);
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(ptr); }
};

// Per-operator constants of the layer-potential combination a_S S + a_D D.
struct OpSpec {
  double a_s, a_d, c_identity;
  bool completion, bordered;
  bool traction = false;  // the single-layer traction K (target normal) instead of a_D D
  bool rigid_local = false;  // + L: int mu + (int (y - c) x mu) x (x - c) on the own sphere
};
OpSpec op_spec(int op_base);

// Device time per step of the hot path during one solve (bie_solve_info.t_stage_s):
// pairs of HIP events recorded on the context's stream around the launches of a step,
// drawn from a pool that the context keeps; nested scopes record only the outermost.
struct StageTimer {
  bool on = false;
  int depth = 0;
  std::vector<hipEvent_t> ev;  // 2 per record
  std::vector<int> tag;        // step of each record
  size_t used = 0;
  long long far_pairs = 0;     // far-field node pairs of the solve's matvecs
  long long near_evals = 0;    // near-series evaluations of the solve's matvecs
};

}  // namespace bie

struct bie_ctx {
  // discretisation
  int p = 0, n_phi = 0, mmax = 0, P = 0, ncoef = 0, nlat = 0;
  int64_t nb = 0, N = 0;
  double near_gap = 1.0;   // d* of Eq. 4.5 (+infinity: every pair near)
  double near_tol = 0.0;   // precision d* was calibrated for (0 when near_gap was given)
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t far_node_pairs = 0;  // node pairs on distinct, well-separated spheres (one far pass)
  bie::StageTimer timer;

  // host copies
  std::vector<double> centres;  // nb x 3
  std::vector<double> radius;   // nb sphere radii (all 1 unless built with radii)
  bool poly = false;            // some radius differs from 1
  std::vector<double> t, lam, theta, wlat, phi;
  std::vector<int> near_ptr, near_idx;  // CSR, target sphere -> near source spheres
  // close pairs of the learned correction: surface gap below close_gap (the gap its
  // network was trained with), independent of d*
  double close_gap = 1.0;
  std::vector<int> close_ptr, close_idx;
  std::vector<int> coef_m, coef_n, coef_off;  // mode (m, n) of each coefficient slot; slot of (m, m)

  // device: geometry
  bie::DevBuf centres4;   // nb x 4 double (x, y, z, 0)
  bie::DevBuf radius_d;   // nb double radii (allocated when poly)
  bie::DevBuf excl;       // nb x nwords uint32: bit s of row t set if s == t or (t, s) near
  int nwords = 0;
  bie::DevBuf dnear_ptr, dnear_idx;
  bie::DevBuf dnear_order;     // target spheres with near neighbours, longest near list first
  int64_t n_near_targets = 0;
  bie::DevBuf neartab;         // nb x near_slots x 16 double: per-source series constants (near.hip)
  int near_slots = 0;
  bie::DevBuf dclose_ptr, dclose_idx;
  bie::DevBuf otab, otab_f;    // P x 4 unit offsets of the nodes of a sphere (double / float)
  bie::DevBuf osrc, osrc_f;    // P x 4 the same offsets times -2 (far-field source table)
  bie::DevBuf frame;           // P x 9 double: e_r, e_theta, e_phi at each node
  bie::DevBuf wnode;           // P double: quadrature weight of each node of a sphere
  // device: transform tables, double and float copies
  bie::DevBuf leg, leg_f;      // 3 x ncoef x nlat: Pbar, dPbar/dtheta, m Pbar / sin(theta)
  bie::DevBuf dft, dft_f;      // (mmax+1) x n_phi x 2: cos(m phi_l), sin(m phi_l)
  bie::DevBuf wlat_d, wlat_f;  // nlat latitude weights
  bie::DevBuf modes;           // ncoef x 2 int: (m, n)
  bie::DevBuf rec;             // ncoef x 6 double: Legendre recurrence constants (near series)
  // device: per-call work
  bie::DevBuf coef;            // nb x 3 x ncoef x 2 double: raw coefficients (near series input)
  bie::DevBuf q;               // N x 4 (double): far-field source strengths w * mu
  bie::DevBuf partial;         // nsplit x N x 3 double: far-field partial sums
  bie::DevBuf moments;         // nb x 6 double: int mu, int (y - c) x mu
  bie::DevBuf scal;            // small scratch for reductions
  int nsplit = 1;              // source splits the partial-sum buffer holds (upper bound per launch)
  int num_cus = 256;           // compute units of the device

  // solver work space (allocated on first solve)
  bie::DevBuf krylov, zbasis, vec[6];
  int krylov_cols = 0;
  int64_t krylov_n = 0;

  // learned coarse correction (coarse.hip, mlp.hip)
  bie::DevBuf lowF;                 // P x 25 x 3 double: low-mode basis fields at the nodes
  bie::DevBuf lownorm;              // 25 double: their squared norms
  std::vector<float> pair_feat;     // directed near pairs (CSR order) x 8 features
  std::vector<double> pair_frame;   // directed near pairs x 34: Q and D2
  bie::DevBuf dframe;               // device copy of pair_frame
  bie::DevBuf mlp_theta;            // near pairs x 278 float: MLP output
  bie::DevBuf rho, zeta;            // nb x 25 double
  bie::DevBuf pc_tmp;               // solve-length work vector of BIE_PC_LOCAL (allocated on first use)
  bool theta_ready = false;

  // global rigid-mode coarse correction (rigid.hip), allocated on first use
  bie::DevBuf rg_vec;               // 8 x 6 nb double: R r, R z, CG vectors, solution
  bie::DevBuf rg_partial;           // source splits x 6 nb double: mobility product partials
  bie::DevBuf rg_dots, rg_hist;     // block partial sums; CG scalars per iteration
  int rg_last_iters = 0;            // CG iterations of the last coarse solve

  // near evaluation by pole rotation (near_rot.hip), near_method = 1
  int near_method = 0;
  int legendre_mfma = 0;   // Legendre stages of the transforms on the matrix cores
  bie::DevBuf wig;                  // sum_n (2n+1)^2 complex: Wigner matrices of R_x(-pi/2)
  bie::DevBuf nearcoef;             // nb x 3 x ncoef x 2: summed near-field coefficients
  bie::DevBuf tlat_d;               // nlat cos(theta_j)

  // single-layer traction near series (traction.hip): recurrence table of degree p+1
  bie::DevBuf rec2;
  int mm2 = 0, ncoef2 = 0;

  // Laplace single layer and the magnetostatic problem (laplace.hip)
  bie::DevBuf lapcoef;              // nb x ncoef x 2 scalar coefficients
  double lap_eta = 0.0;             // eta of Eq. 5.13 for the current solve
};

namespace bie {
// One launch of the per-sphere transform kernel (vsh.hip).
struct VshCall {
  const double* mu = nullptr;       // node field input (3N, or 3N + 6 n_b when bordered)
  const double* coef_in = nullptr;  // coefficient input (coef_is_input)
  double* u = nullptr;              // node field output
  bool write_q = false;             // far-field source strengths w * mu -> ctx->q
  bool write_coef = false;          // raw V, W, X coefficients -> ctx->coef
  bool do_self = false;             // synthesise lam * coefficients (+ identity term)
  bool want_moments = false;        // int mu, int o x mu -> ctx->moments
  bool coef_is_input = false;
  bool bordered = false;            // mobility matvec rows
  bool pc_border = false;           // mobility block preconditioner rows
  bool accumulate = false;          // add the synthesis to u instead of overwriting it
  double c_identity = 0.0, scale_out = 1.0, wv1 = 0.0;
  double lam[3][33] = {};
  // per-sphere multipliers for spheres of radius a_k (radius != nullptr):
  //   lam_mode 1: a_k lamS + lam (operator);  2: 1 / (a_k lamS + lam) - 2 (M0), 0 where
  //   both vanish;  3: lamS a_k^lam_pow[f] + lam (M0 of the completed and traction forms).
  //   With radius set the moments carry a_k^2 (force) and a_k^3 (torque)
  const double* radius = nullptr;
  int lam_mode = 0;
  int lam_pow[3] = {-1, -1, -1};
  double lamS[3][33] = {};
};
void launch_vsh(bie_ctx* c, int precision, const VshCall& v);
// EINVAL unless every sphere has unit radius (features built for unit spheres only)
void require_unit(const bie_ctx* c, const char* what);
void launch_near(bie_ctx* c, const OpSpec& spec, double* u);
void launch_near_rot(bie_ctx* c, const OpSpec& spec, double* u);
void series_radial(double a_s, double a_d, int p, double* kvv, double* kww, double* kwv, double* kxx);
int near_table_slots(int p, int mmax);
std::vector<int> near_launch_order(const std::vector<int>& near_ptr, int64_t nb);
// Source splits the far-field partial-sum buffer is sized for (N nodes, nb spheres).
int far_split_capacity(int64_t N, int64_t nb);
void launch_far(bie_ctx* c, int precision, const OpSpec& spec, double* u);
void apply(bie_ctx* c, int op, int precision, const double* mu, double* u);

// Records the device time of the enclosed launches under step `stage` (BIE_T_*) while
// c->timer.on; no-op otherwise.
class StageScope {
 public:
  StageScope(bie_ctx* c, int stage);
  ~StageScope();
  StageScope(const StageScope&) = delete;
  StageScope& operator=(const StageScope&) = delete;

 private:
  bie_ctx* c_;
  bool rec_ = false;
};
void timer_start(bie_ctx* c);
// Waits for the recorded events and sums their durations per step into t[8]; stops the timer.
void timer_collect(bie_ctx* c, double t[8]);
void timer_release(bie_ctx* c);

// Set-up helpers (setup.cpp): Gauss-Legendre rule (nodes descending), Legendre tables
// at one latitude per coefficient slot (Pbar, dPbar/dtheta, m Pbar / sin theta), the
// recurrence table of the series evaluations (series.h).
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w);
void legendre_tables(int p, int mmax, double t, double s, const std::vector<int>& cm, const std::vector<int>& cn,
                     double* outP, double* outD, double* outQ);
std::vector<double> recurrence_table(int p, int mmax);
// d* of Eq. 4.5 for grid order p on n_phi longitudes and precision tol (calibrate.cpp);
// +infinity when no gap of the search range reaches it
double near_gap_for(int p, int n_phi, double tol);
constexpr double kDefaultNearTol = 1e-8;

// Small BLAS-1 helpers on device vectors (float64), stream-ordered on c->stream.
void dev_dot_many(bie_ctx* c, const double* V, int64_t ld, int k, const double* w, int64_t n, double* host_out);
void dev_gemv_sub(bie_ctx* c, const double* V, int64_t ld, int k, const double* h_host, double* w, int64_t n);
void dev_axpby(bie_ctx* c, double a, const double* x, double b, double* y, int64_t n);  // y = a x + b y
void dev_copy(bie_ctx* c, const double* x, double* y, int64_t n);
void dev_fill(bie_ctx* c, double* y, double v, int64_t n);
double dev_norm(bie_ctx* c, const double* x, int64_t n);
void dev_rigid_rhs(bie_ctx* c, const double* v_dev, const double* om_dev, double* b);
void dev_precond_m0(bie_ctx* c, int op_base, int precision, const double* r, double* z);
void apply_precond(bie_ctx* c, int op_base, int precision, int precond, const double* r, double* z);
void precond_sample(bie_ctx* c, int op_base, int precond, const double* b, const double* x, double* xi,
                    double* target);

// learned coarse correction
void build_coarse(bie_ctx* c);
void lowmode_restrict(bie_ctx* c, const double* f, double* rho);
void lowmode_prolong(bie_ctx* c, const double* rho, double* f, bool accumulate);
// skip_rigid: the learned part acts on the non-rigid low modes only (the rigid ones are
// the global rigid-mode correction's)
void coarse_correct(bie_ctx* c, const double* r, double* z, bool skip_rigid);
void zero_rigid_modes(bie_ctx* c, double* rho);

// global rigid-mode coarse correction: z <- z + P (A_c^-1 R r - R z)
constexpr int64_t RIGID_MAX_SPHERES = 65536;
void rigid_correct(bie_ctx* c, const double* r, double* z);
// xi[6k..6k+5] = mean velocity and rotation of f on sphere k: (int f / (4 pi a^2),
// 3 int (x - c) x f / (8 pi a^4)) (a = 1 for unit spheres)
void rigid_restrict(bie_ctx* c, const double* f, double* xi);

// single-layer traction K on the near pairs; u += a_k + b_k x (x - c_k) (ab = nb x 6)
void launch_near_traction(bie_ctx* c, double* u);
// with radius (nullable): u += a_k + r_k b_k x o, i.e. b_k x (x - c_k) on a sphere of radius r_k
void add_rigid_local(bie_ctx* c, const double* ab, double* u, const double* radius = nullptr);

// Laplace / magnetostatic operators (laplace.hip); OP_LAPLACE is the solver's internal
// operator code for (1/2 I + eta K^L) on N scalar unknowns
constexpr int OP_LAPLACE = 0x40;
void lap_apply(bie_ctx* c, const double* q, double* out);
void lap_precond(bie_ctx* c, const double* r, double* z);
void lap_grad(bie_ctx* c, const double* q, double* grad);
void solve_magnetic(bie_ctx* c, const double H0[3], double eta, const bie_solve_opts* opts, double* q_dev,
                    double* ft_host, bie_solve_info* info, int* rc);
int solve(bie_ctx* c, int op, const double* b, double* x, int64_t n, const bie_solve_opts* so, bie_solve_info* info);

// layer potentials at fluid points (field.hip)
void eval_field(bie_ctx* c, int op_base, const double* mu, int64_t M, const double* x, double* u);
int64_t mlp_n_weights();
double mlp_eval(const bie_mlp_data* d, const float* weights, float* grad);
void mlp_train(const bie_mlp_data* d, float* weights, int epochs, int cfg_per_batch, double lr, double* loss_hist);
void mlp_infer(bie_ctx* c, const float* weights);
}  // namespace bie
