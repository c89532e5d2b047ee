// C ABI entry points (include/bie.h) and the matvec orchestration.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "bie_internal.h"

namespace bie {
void build(bie_ctx* c, const double* centres, const double* radii, int64_t nb, const bie_opts* o);
const char* last_error();

// Table 3.12: S, D_+ eigenvalues per family (V, W, X) and degree n.
static void eig_S(int n, double e[3]) {
  const double d = n;
  e[0] = d / ((2 * d + 1) * (2 * d + 3));
  e[1] = n >= 1 ? (d + 1) / ((2 * d + 1) * (2 * d - 1)) : 0.0;
  e[2] = n >= 1 ? 1.0 / (2 * d + 1) : 0.0;
}
static void eig_Dplus(int n, double e[3]) {
  const double d = n;
  e[0] = (2 * d * d + 4 * d + 3) / ((2 * d + 1) * (2 * d + 3));
  e[1] = n >= 1 ? 2.0 * (d - 1) * (d + 1) / ((2 * d + 1) * (2 * d - 1)) : 0.0;
  e[2] = n >= 1 ? (d - 1) / (2 * d + 1) : 0.0;
}

// Self-term multipliers a_S lambda_S + a_D lambda_Dpv (D_pv = D_+ - 1/2, jump A.7).
static void self_lambda(const OpSpec& s, int p, double lam[3][33]) {
  for (int n = 0; n <= p; ++n) {
    double es[3], ed[3];
    eig_S(n, es);
    eig_Dplus(n, ed);
    for (int f = 0; f < 3; ++f) {
      const bool exists = (f == 0) || n >= 1;
      lam[f][n] = exists ? s.a_s * es[f] + s.a_d * (ed[f] - 0.5) : 0.0;
    }
  }
}

void apply(bie_ctx* c, int op, int precision, const double* mu, double* u) {
  if (op == OP_LAPLACE) {
    lap_apply(c, mu, u);
    return;
  }
  const int base = op & 0xff;
  int stages = op & (BIE_STAGE_SELF | BIE_STAGE_NEAR | BIE_STAGE_FAR);
  if (stages == 0) stages = BIE_STAGE_SELF | BIE_STAGE_NEAR | BIE_STAGE_FAR;
  if (precision != BIE_FP64 && precision != BIE_MIXED) throw Error{BIE_EINVAL, "bad precision"};
  const OpSpec spec = op_spec(base);
  if (spec.traction && c->near_method != 0)
    throw Error{BIE_EINVAL, "the traction operator supports near_method 0 (series at the target nodes) only"};
  VshCall v;
  v.mu = mu;
  v.u = u;
  v.write_q = (stages & BIE_STAGE_FAR) != 0;
  v.write_coef = (stages & BIE_STAGE_NEAR) != 0 && !c->near_idx.empty();
  v.do_self = (stages & BIE_STAGE_SELF) != 0;
  v.want_moments = (spec.completion && (stages & BIE_STAGE_FAR)) || (spec.rigid_local && (stages & BIE_STAGE_SELF));
  v.bordered = spec.bordered;
  v.c_identity = spec.c_identity;
  if (c->poly) {
    // per-sphere multipliers: a_k a_S lambda_S + a_D lambda_Dpv
    OpSpec ss = spec, sd = spec;
    ss.a_d = 0.0;
    sd.a_s = 0.0;
    self_lambda(ss, c->p, v.lamS);
    self_lambda(sd, c->p, v.lam);
    v.radius = c->radius_d.as<double>();
    v.lam_mode = 1;
  } else {
    self_lambda(spec, c->p, v.lam);
  }
  {
    StageScope ts(c, BIE_T_TRANSFORM);
    launch_vsh(c, precision, v);
  }
  // L of Eq. 5.8 on the own sphere: int mu + (int (y - c) x mu) x (x - c)
  if (spec.rigid_local && (stages & BIE_STAGE_SELF)) {
    StageScope ts(c, BIE_T_OTHER);
    add_rigid_local(c, c->moments.as<double>(), u, c->poly ? c->radius_d.as<double>() : nullptr);
  }
  if (stages & BIE_STAGE_NEAR) {
    StageScope ts(c, BIE_T_NEAR);
    if (spec.traction)
      launch_near_traction(c, u);
    else
      launch_near(c, spec, u);
    if (c->timer.on) c->timer.near_evals += (long long)c->near_idx.size() * c->P;
  }
  if (stages & BIE_STAGE_FAR) {
    StageScope ts(c, BIE_T_FAR);
    launch_far(c, precision, spec, u);
    if (c->timer.on) c->timer.far_pairs += c->far_node_pairs;
  }
}

// Block-diagonal preconditioner M0: the exact inverse of every sphere's isolated self
// operator.  On the band-limited part it is diagonal in V, W, X (Theorem 2); on the
// grid complement the operator is 1/2 I, so M0 = 2 I + Pi^+ (Lambda^-1 - 2) Pi.
//  - resistance form 1/2 + D_pv + N: D_+ vanishes on W_1, X_1 and the completion flow
//    maps W_1[a] -> 2/3 W_1[a] - 1/6 V_1[a], X_1 -> 1/3 X_1 (V_1 and higher modes carry
//    no force or torque), so the degree-one block inverse is
//    V_1: 5/3, W_1: 3/2 with V'_1 += 5/12 W_1, X_1: 3; elsewhere 1 / D_+.
//  - mobility form 1/2 + S + D_pv = S + D_+ ((n+1)/(2n+1) on V, W; n/(2n+1) on X),
//    plus the rigid-body rows solved in closed form (see the transform kernel).
//  - traction form of Eq. 5.8, 1/2 + K_pv + L: K_pv = D_pv on the sphere, so the
//    eigenvalues are D_+'s; L acts on the rigid modes only, W_1[a] = a -> 4 pi a and
//    X_1 (rotations) -> 8 pi / 3, which replace the zeros of D_+ there.
void dev_precond_m0(bie_ctx* c, int op_base, int precision, const double* r, double* z) {
  VshCall v;
  v.mu = r;
  v.u = z;
  v.do_self = true;
  v.c_identity = 2.0;
  if (c->poly && op_base == BIE_OP_KL_BIE) {
    // 1/2 + K_pv + L on a sphere of radius a: D_+'s eigenvalues except W_1 -> 4 pi a^2 and
    // X_1 -> 8 pi a^4 / 3 (L with moments a^2, a^3 and lever arm a)
    for (int n = 0; n <= c->p; ++n) {
      double ed[3];
      eig_Dplus(n, ed);
      for (int f = 0; f < 3; ++f) {
        const bool exists = (f == 0) || n >= 1;
        v.lamS[f][n] = 0.0;
        if (!exists) {
          v.lam[f][n] = 0.0;
        } else if (n == 1 && f > 0) {
          v.lamS[f][n] = (f == 1) ? 1.0 / (4.0 * M_PI) : 3.0 / (8.0 * M_PI);
          v.lam[f][n] = -2.0;
        } else {
          v.lam[f][n] = 1.0 / ed[f] - 2.0;
        }
      }
    }
    v.lam_pow[0] = -1;
    v.lam_pow[1] = -2;
    v.lam_pow[2] = -4;
    v.radius = c->radius_d.as<double>();
    v.lam_mode = 3;
    launch_vsh(c, precision, v);
    return;
  }
  if (c->poly && op_base == BIE_OP_DN_BIE) {
    // completed form on a sphere of radius a: the completion's moments carry a^2 and a^3
    // at distance a, so W_1 -> 3/(2a) and X_1 -> 3/a; V_1 (5/3, coupling 5/12) and the
    // other modes (1/D_+) do not depend on a
    for (int n = 0; n <= c->p; ++n) {
      double ed[3];
      eig_Dplus(n, ed);
      for (int f = 0; f < 3; ++f) {
        const bool exists = (f == 0) || n >= 1;
        v.lamS[f][n] = 0.0;
        if (!exists) {
          v.lam[f][n] = 0.0;
        } else if (n == 1 && f == 0) {
          v.lam[f][n] = 5.0 / 3.0 - 2.0;
        } else if (n == 1) {
          v.lamS[f][n] = (f == 1) ? 1.5 : 3.0;
          v.lam[f][n] = -2.0;
        } else {
          v.lam[f][n] = 1.0 / ed[f] - 2.0;
        }
      }
    }
    v.wv1 = 5.0 / 12.0;
    v.radius = c->radius_d.as<double>();
    v.lam_mode = 3;
    launch_vsh(c, precision, v);
    return;
  }
  if (c->poly) {
    // spheres of radius a_k, 1/2 + S + D_pv: 1 / (a_k lambda_S + lambda_D+) per mode (and,
    // for the bordered form, the closed-form rigid rows of the transform kernel)
    if (op_base != BIE_OP_SD_BIE && op_base != BIE_OP_MOBILITY)
      throw Error{BIE_EINVAL, "spheres of several radii: M0 exists for BIE_OP_SD_BIE, _DN_BIE and _MOBILITY"};
    if (op_base == BIE_OP_MOBILITY) v.pc_border = true;
    for (int n = 0; n <= c->p; ++n) {
      double es[3], ed[3];
      eig_S(n, es);
      eig_Dplus(n, ed);
      for (int f = 0; f < 3; ++f) {
        const bool exists = (f == 0) || n >= 1;
        v.lamS[f][n] = exists ? es[f] : 0.0;
        v.lam[f][n] = exists ? ed[f] : 0.0;
      }
    }
    v.radius = c->radius_d.as<double>();
    v.lam_mode = 2;
    launch_vsh(c, precision, v);
    return;
  }
  for (int n = 0; n <= c->p; ++n) {
    double es[3], ed[3];
    eig_S(n, es);
    eig_Dplus(n, ed);
    for (int f = 0; f < 3; ++f) {
      const bool exists = (f == 0) || n >= 1;
      double inv = 0.0;
      if (exists) {
        if (op_base == BIE_OP_DN_BIE) {
          if (n == 1 && f == 0) inv = 5.0 / 3.0;
          else if (n == 1 && f == 1) inv = 1.5;
          else if (n == 1 && f == 2) inv = 3.0;
          else inv = 1.0 / ed[f];
        } else if (op_base == BIE_OP_KL_BIE) {
          if (n == 1 && f == 1) inv = 1.0 / (4.0 * M_PI);
          else if (n == 1 && f == 2) inv = 3.0 / (8.0 * M_PI);
          else inv = 1.0 / ed[f];
        } else {
          inv = 1.0 / (es[f] + ed[f]);
        }
      }
      v.lam[f][n] = exists ? inv - 2.0 : 0.0;
    }
  }
  if (op_base == BIE_OP_DN_BIE) v.wv1 = 5.0 / 12.0;
  if (op_base == BIE_OP_MOBILITY) v.pc_border = true;
  launch_vsh(c, precision, v);
}

void apply_precond(bie_ctx* c, int op_base, int precision, int precond, const double* r, double* z) {
  if (op_base == OP_LAPLACE) {
    if (precond == BIE_PC_NONE)
      dev_copy(c, r, z, c->N);
    else
      lap_precond(c, r, z);
    return;
  }
  if (op_base != BIE_OP_DN_BIE && op_base != BIE_OP_MOBILITY && op_base != BIE_OP_SD_BIE && op_base != BIE_OP_KL_BIE)
    throw Error{BIE_EINVAL,
                "preconditioners exist for BIE_OP_DN_BIE, BIE_OP_MOBILITY, BIE_OP_SD_BIE and BIE_OP_KL_BIE"};
  if (op_base == BIE_OP_KL_BIE && (precond & ~BIE_PC_M0) != 0)
    throw Error{BIE_EINVAL, "BIE_OP_KL_BIE takes BIE_PC_NONE or BIE_PC_M0"};
  if (precision != BIE_FP64 && precision != BIE_MIXED) throw Error{BIE_EINVAL, "bad precision"};
  const int64_t n = 3 * c->N + (op_base == BIE_OP_MOBILITY ? 6 * c->nb : 0);
  const bool rigid = (precond & BIE_PC_RIGID) != 0;
  const bool local = (precond & BIE_PC_LOCAL) != 0;
  const int base = precond & ~(BIE_PC_RIGID | BIE_PC_LOCAL);
  if (local && base != BIE_PC_MLP) throw Error{BIE_EINVAL, "BIE_PC_LOCAL modifies BIE_PC_MLP only"};
  if (c->poly && base == BIE_PC_MLP)
    throw Error{BIE_EINVAL, "spheres of several radii: the learned correction is trained for unit spheres"};
  if (rigid && base == BIE_PC_NONE) throw Error{BIE_EINVAL, "BIE_PC_RIGID needs BIE_PC_M0 or BIE_PC_MLP"};
  if (rigid && c->nb > RIGID_MAX_SPHERES) throw Error{BIE_EINVAL, "BIE_PC_RIGID: too many spheres for the coarse solve"};
  switch (base) {
    case BIE_PC_NONE:
      dev_copy(c, r, z, n);
      return;
    case BIE_PC_M0:
      dev_precond_m0(c, op_base, precision, r, z);
      break;
    case BIE_PC_MLP:
      if (!c->theta_ready) throw Error{BIE_EINVAL, "BIE_PC_MLP needs bie_precond_load first"};
      dev_precond_m0(c, op_base, precision, r, z);
      break;
    default:
      throw Error{BIE_EINVAL, "unknown preconditioner"};
  }
  // The global rigid-mode correction acts on the resistance form only (the mobility form
  // carries the rigid motions as unknowns with their own rows); it resets the rigid part
  // of M0 r.  The learned close-pair correction acts on the density part of the
  // resistance and mobility forms (weights are trained per form) and is added last, so
  // that a network trained on a base keeps its rigid-mode output.
  if (op_base == BIE_OP_SD_BIE || op_base == BIE_OP_KL_BIE) return;
  const bool rigid_on = rigid && op_base == BIE_OP_DN_BIE;
  if (rigid_on) rigid_correct(c, r, z);
  if (base == BIE_PC_MLP) {
    if (local) {
      // the learned correction of the residual that z leaves under the self and
      // near-series parts of the operator: w = r - A_loc z
      if (c->pc_tmp.bytes < (size_t)n * sizeof(double)) c->pc_tmp.alloc((size_t)n * sizeof(double));
      double* w = c->pc_tmp.as<double>();
      apply(c, op_base | BIE_STAGE_SELF | BIE_STAGE_NEAR, precision, z, w);
      dev_axpby(c, 1.0, r, -1.0, w, n);
      coarse_correct(c, w, z, rigid_on);
    } else {
      coarse_correct(c, r, z, rigid_on);
    }
  }
}

// Training sample of the learned correction for one right-hand side b with solution
// x = A^-1 b: target = R x - R z0, xi = R b, or R (b - A_loc z0) for BIE_PC_LOCAL, with
// z0 = B b for the base preconditioner B (M0, optionally with the rigid correction).
void precond_sample(bie_ctx* c, int op_base, int precond, const double* b, const double* x, double* xi,
                    double* target) {
  if (op_base != BIE_OP_DN_BIE && op_base != BIE_OP_MOBILITY)
    throw Error{BIE_EINVAL, "training samples exist for BIE_OP_DN_BIE and BIE_OP_MOBILITY"};
  if (c->poly) throw Error{BIE_EINVAL, "spheres of several radii: the learned correction is for unit spheres"};
  const bool local = (precond & BIE_PC_LOCAL) != 0;
  const int base = precond & ~(BIE_PC_LOCAL | BIE_PC_MLP);
  if ((base & ~BIE_PC_RIGID) != BIE_PC_M0) throw Error{BIE_EINVAL, "the base of a training sample is BIE_PC_M0 (| BIE_PC_RIGID)"};
  const int64_t n = 3 * c->N + (op_base == BIE_OP_MOBILITY ? 6 * c->nb : 0);
  DevBuf z0, w;
  z0.alloc((size_t)n * sizeof(double));
  w.alloc((size_t)n * sizeof(double));
  apply_precond(c, op_base, BIE_FP64, base, b, z0.as<double>());
  // target = R (x - z0)
  dev_copy(c, x, w.as<double>(), n);
  dev_axpby(c, -1.0, z0.as<double>(), 1.0, w.as<double>(), n);
  lowmode_restrict(c, w.as<double>(), target);
  if (local) {
    apply(c, op_base | BIE_STAGE_SELF | BIE_STAGE_NEAR, BIE_FP64, z0.as<double>(), w.as<double>());
    dev_axpby(c, 1.0, b, -1.0, w.as<double>(), n);
    lowmode_restrict(c, w.as<double>(), xi);
  } else {
    lowmode_restrict(c, b, xi);
  }
  if ((base & BIE_PC_RIGID) && op_base == BIE_OP_DN_BIE) {
    // with the rigid-mode correction the learned part acts on the non-rigid modes
    zero_rigid_modes(c, xi);
    zero_rigid_modes(c, target);
  }
  BIE_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace bie

using bie::Error;

#define BIE_TRY(...)                               \
  try {                                            \
    bie::clear_error();                            \
    __VA_ARGS__;                                   \
  } catch (const Error& e) {                       \
    bie::set_error(e.msg);                         \
    return e.code;                                 \
  } catch (const std::bad_alloc&) {                \
    bie::set_error("host allocation failed");      \
    return BIE_ENOMEM;                             \
  } catch (const std::exception& e) {              \
    bie::set_error(e.what());                      \
    return BIE_EINVAL;                             \
  }

extern "C" {

int bie_build_spheres(const double* centres, int64_t n_spheres, const bie_opts* opts, bie_ctx** out) {
  return bie_build_spheres_radii(centres, nullptr, n_spheres, opts, out);
}

int bie_build_spheres_radii(const double* centres, const double* radii, int64_t n_spheres, const bie_opts* opts,
                            bie_ctx** out) {
  if (!out) {
    bie::set_error("out is NULL");
    return BIE_EINVAL;
  }
  *out = nullptr;
  bie_ctx* c = new (std::nothrow) bie_ctx();
  if (!c) return BIE_ENOMEM;
  try {
    bie::clear_error();
    bie::build(c, centres, radii, n_spheres, opts);
  } catch (const Error& e) {
    bie::set_error(e.msg);
    bie_free(c);
    return e.code;
  } catch (const std::exception& e) {
    bie::set_error(e.what());
    bie_free(c);
    return BIE_EINVAL;
  }
  *out = c;
  return BIE_OK;
}

void bie_free(bie_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  bie::DevBuf* bufs[] = {&c->centres4, &c->excl, &c->dnear_ptr, &c->dnear_idx, &c->otab, &c->otab_f, &c->frame,
                         &c->wnode, &c->leg, &c->leg_f, &c->dft, &c->dft_f, &c->wlat_d, &c->wlat_f, &c->modes,
                         &c->rec, &c->coef, &c->q, &c->partial, &c->moments, &c->scal, &c->krylov, &c->zbasis,
                         &c->vec[0], &c->vec[1], &c->vec[2], &c->vec[3], &c->vec[4], &c->vec[5]};
  for (auto* b : bufs) b->release();
  bie::timer_release(c);
  delete c;
}

int bie_sizes(const bie_ctx* c, int64_t* n_nodes, int64_t* n_spheres, int64_t* nodes_per_sphere, int64_t* mmax) {
  if (!c) return BIE_EINVAL;
  if (n_nodes) *n_nodes = c->N;
  if (n_spheres) *n_spheres = c->nb;
  if (nodes_per_sphere) *nodes_per_sphere = c->P;
  if (mmax) *mmax = c->mmax;
  return BIE_OK;
}

int bie_num_nodes(const bie_ctx* c, int64_t* n_nodes) {
  if (!c || !n_nodes) return BIE_EINVAL;
  *n_nodes = c->N;
  return BIE_OK;
}

int bie_near_gap(const bie_ctx* c, double* d_star, double* near_tol) {
  if (!c) return BIE_EINVAL;
  if (d_star) *d_star = c->near_gap;
  if (near_tol) *near_tol = c->near_tol;
  return BIE_OK;
}

int bie_near_gap_for(int p, int n_phi, double tol, double* d_star) {
  if (!d_star) {
    bie::set_error("d_star is NULL");
    return BIE_EINVAL;
  }
  BIE_TRY(*d_star = bie::near_gap_for(p, n_phi, tol));
  return BIE_OK;
}

int bie_get_nodes(const bie_ctx* c, double* xyz, double* w) {
  if (!c) return BIE_EINVAL;
  for (int64_t k = 0; k < c->nb; ++k)
    for (int j = 0; j < c->nlat; ++j) {
      const double tj = c->t[j], sj = std::sqrt(std::max(0.0, 1.0 - tj * tj));
      for (int l = 0; l < c->n_phi; ++l) {
        const int64_t g = k * c->P + j * c->n_phi + l;
        const double a = c->radius[k];
        if (xyz) {
          xyz[3 * g] = c->centres[3 * k] + a * (sj * std::cos(c->phi[l]));
          xyz[3 * g + 1] = c->centres[3 * k + 1] + a * (sj * std::sin(c->phi[l]));
          xyz[3 * g + 2] = c->centres[3 * k + 2] + a * tj;
        }
        if (w) w[g] = a * a * c->wlat[j];
      }
    }
  return BIE_OK;
}

int bie_near_pairs(const bie_ctx* c, int64_t* count, int64_t* pairs) {
  if (!c || !count) return BIE_EINVAL;
  *count = (int64_t)c->near_idx.size();
  if (pairs) {
    int64_t e = 0;
    for (int64_t t = 0; t < c->nb; ++t)
      for (int i = c->near_ptr[t]; i < c->near_ptr[t + 1]; ++i, ++e) {
        pairs[e] = t;
        pairs[*count + e] = c->near_idx[i];
      }
  }
  return BIE_OK;
}

int bie_apply_bio(bie_ctx* c, int op, int precision, const double* mu, double* u) {
  if (!c || !mu || !u) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  if (mu == u) {
    bie::set_error("mu and u alias");
    return BIE_EINVAL;
  }
  BIE_TRY(bie::apply(c, op, precision, mu, u));
  return BIE_OK;
}

int bie_vsh_forward(bie_ctx* c, int precision, const double* mu, double* coef) {
  if (!c || !mu || !coef) return BIE_EINVAL;
  BIE_TRY({
    bie::VshCall v;
    v.mu = mu;
    v.write_coef = true;
    bie::launch_vsh(c, precision, v);
    BIE_HIP(hipMemcpyAsync(coef, c->coef.ptr, (size_t)c->nb * 3 * c->ncoef * 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
  });
  return BIE_OK;
}

int bie_vsh_inverse(bie_ctx* c, int precision, const double* coef, double* u) {
  if (!c || !coef || !u) return BIE_EINVAL;
  BIE_TRY({
    bie::VshCall v;
    v.coef_in = coef;
    v.coef_is_input = true;
    v.u = u;
    bie::launch_vsh(c, precision, v);
  });
  return BIE_OK;
}

int bie_solve_resistance(bie_ctx* c, const double* v, const double* omega, const bie_solve_opts* opts, double* F,
                         double* T, double* psi, bie_solve_info* info) {
  if (!c || !v || !omega || !F || !T) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  int rc = BIE_OK;
  BIE_TRY({
    const int64_t n = 3 * c->N;
    bie::DevBuf rhs, x, vw;
    rhs.alloc(n * sizeof(double));
    x.alloc(n * sizeof(double));
    vw.alloc(6 * c->nb * sizeof(double));
    // omega_i x (x - c_i) with x - c_i = a_i o: the unit-offset kernel takes a_i omega_i
    std::vector<double> om(omega, omega + 3 * c->nb);
    for (int64_t k = 0; k < c->nb; ++k)
      for (int d = 0; d < 3; ++d) om[3 * k + d] *= c->radius[k];
    BIE_HIP(hipMemcpyAsync(vw.ptr, v, 3 * c->nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
    BIE_HIP(hipMemcpyAsync(vw.as<double>() + 3 * c->nb, om.data(), 3 * c->nb * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    bie::dev_rigid_rhs(c, vw.as<double>(), vw.as<double>() + 3 * c->nb, rhs.as<double>());
    rc = bie::solve(c, BIE_OP_DN_BIE, rhs.as<double>(), x.as<double>(), n, opts, info);
    // F_k = int psi, T_k = int (y - c_k) x psi
    bie::VshCall m;
    m.mu = x.as<double>();
    m.want_moments = true;
    if (c->poly) {
      m.radius = c->radius_d.as<double>();
      m.lam_mode = 1;
    }
    bie::launch_vsh(c, BIE_FP64, m);
    std::vector<double> mom(6 * c->nb);
    BIE_HIP(hipMemcpyAsync(mom.data(), c->moments.ptr, mom.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (psi) BIE_HIP(hipMemcpyAsync(psi, x.ptr, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    BIE_HIP(hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < c->nb; ++k)
      for (int d = 0; d < 3; ++d) {
        F[3 * k + d] = mom[6 * k + d];
        T[3 * k + d] = mom[6 * k + 3 + d];
      }
    rhs.release();
    x.release();
    vw.release();
  });
  return rc;
}

int bie_solve_mobility(bie_ctx* c, const double* F, const double* T, const double* slip, const bie_solve_opts* opts,
                       double* v, double* omega, double* mu, bie_solve_info* info) {
  if (!c || !F || !T || !v || !omega) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  int rc = BIE_OK;
  BIE_TRY({
    const int64_t n3 = 3 * c->N, n = n3 + 6 * c->nb;
    bie::DevBuf rhs, x;
    rhs.alloc(n * sizeof(double));
    x.alloc(n * sizeof(double));
    if (slip)
      BIE_HIP(hipMemcpyAsync(rhs.ptr, slip, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else
      bie::dev_fill(c, rhs.as<double>(), 0.0, n3);
    std::vector<double> tail(6 * c->nb);
    for (int64_t k = 0; k < 3 * c->nb; ++k) {
      tail[k] = F[k] / (4.0 * M_PI);
      tail[3 * c->nb + k] = 3.0 * T[k] / (8.0 * M_PI);
    }
    BIE_HIP(hipMemcpyAsync(rhs.as<double>() + n3, tail.data(), tail.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    rc = bie::solve(c, BIE_OP_MOBILITY, rhs.as<double>(), x.as<double>(), n, opts, info);
    std::vector<double> out(6 * c->nb);
    BIE_HIP(hipMemcpyAsync(out.data(), x.as<double>() + n3, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    if (mu) BIE_HIP(hipMemcpyAsync(mu, x.ptr, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    BIE_HIP(hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < 3 * c->nb; ++k) {
      v[k] = out[k];
      omega[k] = out[3 * c->nb + k];
    }
    rhs.release();
    x.release();
  });
  return rc;
}

int bie_solve_mobility_traction(bie_ctx* c, const double* F, const double* T, const bie_solve_opts* opts, double* v,
                                double* omega, double* mu, bie_solve_info* info) {
  if (!c || !F || !T || !v || !omega) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  if (opts && (opts->precond & ~BIE_PC_M0) != 0) {
    bie::set_error("bie_solve_mobility_traction takes BIE_PC_NONE or BIE_PC_M0");
    return BIE_EINVAL;
  }
  int rc = BIE_OK;
  BIE_TRY({
    const int64_t n3 = 3 * c->N, nb = c->nb;
    bie::DevBuf rho, rhs, x, ab;
    rho.alloc(n3 * sizeof(double));
    rhs.alloc(n3 * sizeof(double));
    x.alloc(n3 * sizeof(double));
    ab.alloc(6 * nb * sizeof(double));
    // rho of Eq. 5.7: F_k / (4 pi a^2) + 3/(8 pi a^4) T_k x (x - c_k) on a sphere of
    // radius a (int rho = F_k, int (x - c_k) x rho = T_k); x - c_k = a o
    std::vector<double> h(6 * nb);
    for (int64_t k = 0; k < nb; ++k) {
      const double a = c->radius[k];
      for (int d = 0; d < 3; ++d) {
        h[6 * k + d] = F[3 * k + d] / (4.0 * M_PI * a * a);
        h[6 * k + 3 + d] = 3.0 * T[3 * k + d] / (8.0 * M_PI * a * a * a * a);
      }
    }
    BIE_HIP(hipMemcpyAsync(ab.ptr, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    bie::dev_fill(c, rho.as<double>(), 0.0, n3);
    bie::add_rigid_local(c, ab.as<double>(), rho.as<double>(), c->poly ? c->radius_d.as<double>() : nullptr);
    // right-hand side of Eq. 5.8: -(1/2 rho + sum_k K_k[rho]), float64
    bie::apply(c, BIE_OP_K, BIE_FP64, rho.as<double>(), rhs.as<double>());
    bie::dev_axpby(c, -0.5, rho.as<double>(), -1.0, rhs.as<double>(), n3);
    rc = bie::solve(c, BIE_OP_KL_BIE, rhs.as<double>(), x.as<double>(), n3, opts, info);
    if (mu) BIE_HIP(hipMemcpyAsync(mu, x.ptr, n3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    // u = sum_k S_k[mu + rho] on the surfaces (Eq. 5.7), its rigid motion per sphere
    bie::dev_axpby(c, 1.0, rho.as<double>(), 1.0, x.as<double>(), n3);
    bie::apply(c, BIE_OP_S, BIE_FP64, x.as<double>(), rhs.as<double>());
    bie::rigid_restrict(c, rhs.as<double>(), ab.as<double>());
    BIE_HIP(hipMemcpyAsync(h.data(), ab.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    BIE_HIP(hipStreamSynchronize(c->stream));
    // rigid_restrict returns the mean velocity and rotation of u on each sphere
    for (int64_t k = 0; k < nb; ++k)
      for (int d = 0; d < 3; ++d) {
        v[3 * k + d] = h[6 * k + d];
        omega[3 * k + d] = h[6 * k + 3 + d];
      }
    rho.release();
    rhs.release();
    x.release();
    ab.release();
  });
  return rc;
}

int bie_solve(bie_ctx* c, int op, const double* b, double* x, const bie_solve_opts* opts, bie_solve_info* info) {
  if (!c || !b || !x) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  if (op != BIE_OP_DN_BIE && op != BIE_OP_MOBILITY && op != BIE_OP_SD_BIE && op != BIE_OP_KL_BIE) {
    bie::set_error("bie_solve supports BIE_OP_DN_BIE, BIE_OP_MOBILITY, BIE_OP_SD_BIE and BIE_OP_KL_BIE");
    return BIE_EINVAL;
  }
  int rc = BIE_OK;
  const int64_t n = 3 * c->N + (op == BIE_OP_MOBILITY ? 6 * c->nb : 0);
  BIE_TRY(rc = bie::solve(c, op, b, x, n, opts, info));
  return rc;
}

int bie_apply_precond(bie_ctx* c, int op, int precision, int precond, const double* r, double* z) {
  if (!c || !r || !z || r == z) {
    bie::set_error("null or aliased argument");
    return BIE_EINVAL;
  }
  BIE_TRY(bie::apply_precond(c, op, precision, precond, r, z));
  return BIE_OK;
}

int bie_apply_laplace(bie_ctx* c, int kind, double eta, const double* q, double* out) {
  if (!c || !q || !out || q == out || (kind != 0 && kind != 1)) {
    bie::set_error("bie_apply_laplace: bad arguments");
    return BIE_EINVAL;
  }
  BIE_TRY(if (kind == 0) {
    c->lap_eta = eta;
    bie::lap_apply(c, q, out);
  } else {
    bie::lap_grad(c, q, out);
  });
  return BIE_OK;
}

int bie_solve_magnetic(bie_ctx* c, const double* H0, double eta, const bie_solve_opts* opts, double* q, double* F,
                       double* T, bie_solve_info* info) {
  if (!c || !H0 || !F || !T) {
    bie::set_error("bie_solve_magnetic: null argument");
    return BIE_EINVAL;
  }
  int rc = BIE_OK;
  BIE_TRY({
    bie::DevBuf qtmp;
    double* qd = q;
    if (!qd) {
      qtmp.alloc(c->N * sizeof(double));
      qd = qtmp.as<double>();
    }
    std::vector<double> ft(6 * c->nb);
    bie::solve_magnetic(c, H0, eta, opts, qd, ft.data(), info, &rc);
    for (int64_t k = 0; k < c->nb; ++k)
      for (int d = 0; d < 3; ++d) {
        F[3 * k + d] = ft[6 * k + d];
        T[3 * k + d] = ft[6 * k + 3 + d];
      }
  });
  return rc;
}

int bie_eval_field(bie_ctx* c, int op, const double* mu, int64_t n_targets, const double* targets, double* u) {
  if (!c) {
    bie::set_error("null context");
    return BIE_EINVAL;
  }
  BIE_TRY(bie::eval_field(c, op, mu, n_targets, targets, u));
  return BIE_OK;
}

int bie_lowmodes(bie_ctx* c, const double* f, double* rho) {
  if (!c || !f || !rho) return BIE_EINVAL;
  BIE_TRY(bie::require_unit(c, "bie_lowmodes"); bie::lowmode_restrict(c, f, rho));
  return BIE_OK;
}

int bie_lowmodes_synth(bie_ctx* c, const double* rho, double* f) {
  if (!c || !f || !rho) return BIE_EINVAL;
  BIE_TRY(bie::require_unit(c, "bie_lowmodes_synth"); bie::lowmode_prolong(c, rho, f, false));
  return BIE_OK;
}

int bie_pair_geometry(const bie_ctx* c, int64_t* count, int32_t* pair_i, int32_t* pair_j, float* feats,
                      double* frames) {
  if (!c || !count) return BIE_EINVAL;
  const int64_t np = (int64_t)c->close_idx.size();
  *count = np;
  for (int64_t i = 0; i < c->nb; ++i)
    for (int e = c->close_ptr[i]; e < c->close_ptr[i + 1]; ++e) {
      if (pair_i) pair_i[e] = (int32_t)i;
      if (pair_j) pair_j[e] = c->close_idx[e];
    }
  if (feats && np) std::memcpy(feats, c->pair_feat.data(), c->pair_feat.size() * sizeof(float));
  if (frames && np) std::memcpy(frames, c->pair_frame.data(), c->pair_frame.size() * sizeof(double));
  return BIE_OK;
}

int bie_precond_sample(bie_ctx* c, int op, int precond, const double* b, const double* x, double* xi,
                       double* target) {
  if (!c || !b || !x || !xi || !target) {
    bie::set_error("null argument");
    return BIE_EINVAL;
  }
  BIE_TRY(bie::precond_sample(c, op, precond, b, x, xi, target));
  return BIE_OK;
}

int64_t bie_mlp_n_weights(void) { return bie::mlp_n_weights(); }

int bie_precond_load(bie_ctx* c, const float* weights, int64_t n_weights) {
  if (!c || !weights || n_weights != bie::mlp_n_weights()) {
    bie::set_error("null context / weights or wrong weight count");
    return BIE_EINVAL;
  }
  BIE_TRY(bie::require_unit(c, "bie_precond_load"); bie::mlp_infer(c, weights));
  return BIE_OK;
}

int bie_mlp_eval(const bie_mlp_data* data, const float* weights, double* loss, float* grad) {
  if (!data || !weights || !loss || !grad) return BIE_EINVAL;
  BIE_TRY(*loss = bie::mlp_eval(data, weights, grad));
  return BIE_OK;
}

int bie_mlp_train(const bie_mlp_data* data, float* weights, int epochs, int cfg_per_batch, double lr,
                  double* loss_hist) {
  if (!data || !weights) return BIE_EINVAL;
  BIE_TRY(bie::mlp_train(data, weights, epochs, cfg_per_batch, lr, loss_hist));
  return BIE_OK;
}

const char* bie_last_error(void) { return bie::last_error(); }

}  // extern "C"
