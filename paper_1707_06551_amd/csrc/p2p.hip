// Far-field smooth quadrature (Eq. 4.4): all-pairs Stokeslet / double-layer sums over the
// nodes of every well-separated sphere pair (Eq. 4.5), the stage the paper hands to an
// FMM (Section 4.3).  Here it is a tiled direct sum on the GPU.
//
// Work decomposition: a work-group owns 256 x TPL target nodes and one contiguous range
// of source spheres (grid.y splits the spheres so that the launch has thousands of
// work-groups).  Sources are staged in LDS one sphere at a time: the unit offsets o of a
// sphere's nodes (the same table for every sphere, loaded once) and the strengths
// q = w mu of the current sphere with g = o . q packed in the fourth lane.  All lanes
// read the same LDS words per source (broadcast).
//
// Pair arithmetic.  For a target x and a source sphere with centre c, let p = x - c
// (formed from the float64 centre difference plus the target's own offset, so float32
// keeps full relative accuracy at any box size).  A source node y = c + o has
// r = x - y = p - o, and because |o| = 1:
//   r.r = (|p|^2 + 1) - 2 p.o,  r.n_y = r.o = p.o - 1,  r.q = p.q - o.q.
// The source table holds o~ = -2 o (an exact scaling), so that r.r = K + p.o~ with
// K = |p|^2 + 1 is one chain of three fused multiply-adds started from K.
// The sums over a source sphere are kept as  C = sum c_y,  Co~ = sum c_y o~_y,  Q = sum q_y / r
// so that  sum c_y r_y = p C + Co~ / 2.  For the allowed (far) pairs r >= d* so the
// cancellation in r.r costs a few ulp at most.  For S+D the double-layer factor
// 1 + 6 (r.n)/r^2 is rewritten with r.n = (|p|^2 - 1 - r.r)/2 as
// 3 (|p|^2 - 1)/r^2 - 2, one fused multiply-add per pair with 3 (|p|^2 - 1) formed once
// per (target, source sphere); the factor stays near 1 (|p| <= r + 1), so this costs no
// cancellation.  Per pair: S+D 18 VALU + 1 rsqrt, D 17, S 16, K 18.  All inner-loop operands
// are VGPRs, literals or inline constants: on gfx950 a float32 VALU instruction with an
// SGPR operand issues at half the rate of one without (measured), which is why float32
// sources are staged in LDS rather than read through the scalar cache.  Self and near source spheres are skipped through a per-target bit mask (a whole
// wave skips when all its lanes are excluded); per-sphere partial sums are added to the
// running total with Kahan compensation.  The completion flow of the resistance problem
// (Stokeslet + rotlet at every centre, Eqs. 5.18-5.19) is added once per (target, sphere)
// in float64.
#include "bie_internal.h"

namespace bie {

struct FarParams {
  const void* q;          // N x 4 (R): w * mu, w * (o . mu)
  const void* otab;       // P x 4 (R): unit offsets of the nodes of a sphere (targets)
  const void* osrc;       // P x 4 (R): the same offsets times -2 (sources)
  const double* centres4; // nb x 4
  const uint32_t* excl;   // nb x nwords
  const double* moments;  // nb x 6 (completion only)
  const double* radius;   // nb radii (RADII kernels only)
  double* partial;        // nsplit x N x 3
  int64_t N, nb;
  int P, nwords, sph_per_split, completion;
  double cscale;          // kernel constant applied to the pair sums
};

template <typename R>
__device__ __forceinline__ R rsqrt_r(R x);
template <>
__device__ __forceinline__ float rsqrt_r<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ __forceinline__ double rsqrt_r<double>(double x) {
  // hardware estimate (measured max relative error 5.2e-8 on gfx950) refined by one
  // Newton step y <- y (3 - x y^2) / 2 (measured 4.1e-15)
  double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  const double e = fma(-h, y, 1.0);
  return fma(0.5 * y, e, y);
}

template <typename R>
struct R4 {
  R x, y, z, w;
};

// KIND: 1 = Stokeslet, 2 = double layer, 3 = Stokeslet + double layer, 4 = single-layer
// traction K (Eq. 2.22, normal of the TARGET node).  Constants:
//   S:   (1/8pi) [q/r + r (r.q)/r^3]            -> c = (r.q) / r^3
//   D:   (3/4pi) r (r.q)(r.n)/r^5               -> c = (r.q)(2 + p.o~) / r^5 = -2 (r.q)(r.n) / r^5,
//        the factor -1/2 applied once to the sum (an exact power-of-two scaling)
//   S+D: (1/8pi) [q/r + r (r.q)/r^3 (1 + 6 (r.n)/r^2)]  -> c = (r.q)/r^3 (3 (|p|^2 - 1)/r^2 - 2)
//   K:   -(3/4pi) r (r.q)(r.n_x)/r^5            -> c = (r.q)(r.n_x) / r^5, with
//        r.n_x = p.n_x - o.n_x = K3 + o~.(n_x / 2), K3 = p.n_x formed once per (target,
//        source sphere) and tn = n_x / 2 per target
// o holds o~ = -2 o.  tc is -2 for unit spheres (a literal after inlining); a_s - 3 in
// units of a source radius a_s (the single layer's share of t scales with a_s, the double
// layer's not).
template <typename R, int KIND>
__device__ __forceinline__ void pair(R px, R py, R pz, R K, R K3, R tnx, R tny, R tnz, R tc, const R4<R>& o,
                                     const R4<R>& q, R& C, R& Cx, R& Cy, R& Cz, R& Qx, R& Qy, R& Qz) {
  R r2, d2 = 0;
  if (KIND == 2) {
    d2 = fma(pz, o.z, fma(py, o.y, fma(px, o.x, (R)2)));   // 2 - 2 p.o = -2 r.n
    r2 = K + d2;                                           // K = |p|^2 - 1
  } else {
    r2 = fma(pz, o.z, fma(py, o.y, fma(px, o.x, K)));
  }
  const R ir = rsqrt_r<R>(r2);
  const R ir2 = ir * ir;
  const R rq = fma(pz, q.z, fma(py, q.y, fma(px, q.x, -q.w)));
  R c;
  if (KIND == 1) {
    c = rq * ir * ir2;
  } else if (KIND == 2) {
    c = (rq * d2) * (ir2 * ir2 * ir);
  } else if (KIND == 4) {
    const R rn = fma(o.z, tnz, fma(o.y, tny, fma(o.x, tnx, K3)));
    c = (rq * rn) * (ir2 * ir2 * ir);
  } else {
    const R t = fma(K3, ir2, tc);   // 1 + 6 (r.n)/r^2 with K3 = 3 (|p|^2 - 1), tc = -2
    c = ((rq * ir) * ir2) * t;
  }
  C += c;
  Cx = fma(c, o.x, Cx);
  Cy = fma(c, o.y, Cy);
  Cz = fma(c, o.z, Cz);
  if (KIND == 1 || KIND == 3) {
    Qx = fma(ir, q.x, Qx);
    Qy = fma(ir, q.y, Qy);
    Qz = fma(ir, q.z, Qz);
  }
}

// SRC = 0: sources staged in LDS (broadcast reads); SRC = 1: sources read through the
// scalar data cache (constant address space, wave-uniform addresses -> s_load into
// SGPRs that the VALU reads directly).
// RADII: spheres of radius a_k.  Each source sphere's sum is formed in units of its
// radius, p~ = (x - c_s) / a_s with x = c_t + a_t o_t, where the node offsets are unit
// vectors again; with q = w mu (unit weights) the sphere's Stokeslet sum scales by a_s
// and its double-layer and traction sums not at all (homogeneity 1 and 0 in length).
// The float32 double layer (112 VGPRs unconstrained, four waves per SIMD) is held to
// five waves: 94 VGPRs, no spills, the same inner loop; measured 1-2% faster (4096
// spheres, p = 8: 123.5 -> 122.1 ms; 1024 spheres, p = 16: 106.9 -> 104.7 ms).
template <typename R, int KIND, int TPL, int SRC, bool RADII>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && KIND == 2 && !RADII ? 5 : 1, 8)))
void far_kernel(FarParams a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // source table interleaved in LDS: sm[2 i] = o~_i (the same for every sphere, loaded
  // once), sm[2 i + 1] = q_i of the current sphere; one address serves both reads
  R4<R>* sm = reinterpret_cast<R4<R>*>(smem_raw);
  const int tid = threadIdx.x;
  const int P = a.P;
  const R4<R>* qg = reinterpret_cast<const R4<R>*>(a.q);
  const R4<R>* og = reinterpret_cast<const R4<R>*>(a.otab);
  const R4<R>* osg = reinterpret_cast<const R4<R>*>(a.osrc);
  typedef __attribute__((address_space(4))) const R4<R> CR4;
  const CR4* qc = (const CR4*)qg;
  const CR4* oc = (const CR4*)osg;
  if (SRC == 0)
    for (int i = tid; i < P; i += 256) sm[2 * i] = osg[i];

  const int s_begin = blockIdx.y * a.sph_per_split;
  const int s_end = (int)min<int64_t>(a.nb, (int64_t)s_begin + a.sph_per_split);

  int64_t g[TPL];
  int tsph[TPL];
  bool valid[TPL];
  double at[TPL];
  R oxt[TPL][3];
  R tot[TPL][3], comp[TPL][3];
  double cpl[TPL][3];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    g[k] = (int64_t)blockIdx.x * 256 * TPL + k * 256 + tid;
    valid[k] = g[k] < a.N;
    const int64_t gg = valid[k] ? g[k] : 0;
    tsph[k] = (int)(gg / P);
    at[k] = RADII ? a.radius[tsph[k]] : 1.0;
    const int li = (int)(gg - (int64_t)tsph[k] * P);
    const R4<R> o = og[li];
    oxt[k][0] = o.x;
    oxt[k][1] = o.y;
    oxt[k][2] = o.z;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      tot[k][d] = 0;
      comp[k][d] = 0;
      cpl[k][d] = 0.0;
    }
  }

  for (int s = s_begin; s < s_end; ++s) {
    if (SRC == 0) {
      __syncthreads();
      for (int i = tid; i < P; i += 256) sm[2 * i + 1] = qg[(int64_t)s * P + i];
    }
    const double csx = a.centres4[4 * s], csy = a.centres4[4 * s + 1], csz = a.centres4[4 * s + 2];
    const double as = RADII ? a.radius[s] : 1.0;
    const double ias = RADII ? 1.0 / as : 1.0;
    R px[TPL], py[TPL], pz[TPL], K[TPL], K3[TPL], tcv[TPL];
    bool skip[TPL];
    bool any = false;
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      const uint32_t bits = a.excl[(int64_t)tsph[k] * a.nwords + (s >> 5)];
      skip[k] = !valid[k] || ((bits >> (s & 31)) & 1u);
      const double dx = a.centres4[4 * tsph[k]] - csx;
      const double dy = a.centres4[4 * tsph[k] + 1] - csy;
      const double dz = a.centres4[4 * tsph[k] + 2] - csz;
      if (RADII) {
        px[k] = (R)((dx + at[k] * (double)oxt[k][0]) * ias);
        py[k] = (R)((dy + at[k] * (double)oxt[k][1]) * ias);
        pz[k] = (R)((dz + at[k] * (double)oxt[k][2]) * ias);
        // a VGPR copy of the per-sphere constant: a VALU operand read from an SGPR halves
        // the float32 issue rate (measured), and 0 * p keeps the value per lane
        tcv[k] = fma(px[k], (R)0, (R)(as - 3.0));
      } else {
        px[k] = (R)dx + oxt[k][0];
        py[k] = (R)dy + oxt[k][1];
        pz[k] = (R)dz + oxt[k][2];
        tcv[k] = (R)-2;
      }
      K[k] = fma(px[k], px[k], fma(py[k], py[k], fma(pz[k], pz[k], (R)(KIND == 2 ? -1 : 1))));
      if (KIND == 4)
        K3[k] = fma(px[k], oxt[k][0], fma(py[k], oxt[k][1], pz[k] * oxt[k][2]));
      else
        K3[k] = (R)3 * fma(px[k], px[k], fma(py[k], py[k], fma(pz[k], pz[k], (R)-1)));
      any = any || !skip[k];
      if (a.completion && valid[k]) {
        // Stokeslet of strength F_s and rotlet of torque T_s at c_s, in float64
        const double qx = dx + at[k] * (double)oxt[k][0], qy = dy + at[k] * (double)oxt[k][1],
                     qz = dz + at[k] * (double)oxt[k][2];
        const double* mo = a.moments + 6 * (int64_t)s;
        const double r2 = qx * qx + qy * qy + qz * qz;
        const double ir = rsqrt_r<double>(r2);   // refined estimate: 1.0-1.3% faster than 1/sqrt (measured)
        const double ir3 = ir * ir * ir;
        const double rf = qx * mo[0] + qy * mo[1] + qz * mo[2];
        cpl[k][0] += mo[0] * ir + qx * rf * ir3 + (mo[4] * qz - mo[5] * qy) * ir3;
        cpl[k][1] += mo[1] * ir + qy * rf * ir3 + (mo[5] * qx - mo[3] * qz) * ir3;
        cpl[k][2] += mo[2] * ir + qz * rf * ir3 + (mo[3] * qy - mo[4] * qx) * ir3;
      }
    }
    if (SRC == 0) __syncthreads();
    // skip the sphere when every lane of the wave excludes it (self / near / padding)
    if (__any(any ? 1 : 0) == 0) continue;
    R C[TPL], Cx[TPL], Cy[TPL], Cz[TPL], Qx[TPL], Qy[TPL], Qz[TPL];
#pragma unroll
    for (int k = 0; k < TPL; ++k) C[k] = Cx[k] = Cy[k] = Cz[k] = Qx[k] = Qy[k] = Qz[k] = 0;
    // source unroll: 2 for the float32 S+D kernel (95 VGPRs, 5 waves per SIMD; 4 needs
    // 117 VGPRs and was 8% slower), 4 elsewhere (equal or better there, measured)
    constexpr int UNR = (sizeof(R) == 4 && KIND == 3) ? 2 : 4;
#pragma unroll UNR
    for (int i = 0; i < P; ++i) {
      R4<R> o, qq;
      if (SRC == 0) {
        o = sm[2 * i];
        qq = sm[2 * i + 1];
      } else {
        const CR4& oo = oc[i];
        const CR4& q4 = qc[(int64_t)s * P + i];
        o = R4<R>{oo.x, oo.y, oo.z, oo.w};
        qq = R4<R>{q4.x, q4.y, q4.z, q4.w};
      }
#pragma unroll
      for (int k = 0; k < TPL; ++k)
        pair<R, KIND>(px[k], py[k], pz[k], K[k], K3[k], (R)0.5 * oxt[k][0], (R)0.5 * oxt[k][1], (R)0.5 * oxt[k][2],
                      tcv[k], o, qq, C[k], Cx[k], Cy[k], Cz[k], Qx[k], Qy[k], Qz[k]);
    }
#pragma unroll
    for (int k = 0; k < TPL; ++k) {
      if (skip[k]) continue;
      // sum c r = p C + Co~ / 2
      R part[3] = {fma(px[k], C[k], fma((R)0.5, Cx[k], Qx[k])), fma(py[k], C[k], fma((R)0.5, Cy[k], Qy[k])),
                   fma(pz[k], C[k], fma((R)0.5, Cz[k], Qz[k]))};
      if (RADII && KIND == 1) {
        part[0] *= (R)as;
        part[1] *= (R)as;
        part[2] *= (R)as;
      } else if (RADII && KIND == 3) {
        part[0] = fma(px[k], C[k], fma((R)as, Qx[k], (R)0.5 * Cx[k]));
        part[1] = fma(py[k], C[k], fma((R)as, Qy[k], (R)0.5 * Cy[k]));
        part[2] = fma(pz[k], C[k], fma((R)as, Qz[k], (R)0.5 * Cz[k]));
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        // Kahan-compensated accumulation of the per-sphere partial sum
        const R y = part[d] - comp[k][d];
        const R tt = tot[k][d] + y;
        comp[k][d] = (tt - tot[k][d]) - y;
        tot[k][d] = tt;
      }
    }
  }
  const double cs = KIND == 2 ? -0.5 * a.cscale : a.cscale;
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    if (!valid[k]) continue;
    double* out = a.partial + ((int64_t)blockIdx.y * a.N + g[k]) * 3;
    for (int d = 0; d < 3; ++d)
      out[d] = cs * ((double)tot[k][d] - (double)comp[k][d]) + (1.0 / (8.0 * M_PI)) * cpl[k][d];
  }
}

__global__ void reduce_partials(const double* partial, int nsplit, int64_t n3, double* u) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)k * n3 + i];
    u[i] += s;
  }
}

// Measured on MI355X (512 spheres, p = 12, S+D, 20-VALU pair form): float32 LDS 11.4 ms
// vs scalar 13.8 ms; float64 LDS 22.4 ms vs scalar 21.0 ms.  float32 stages sources in
// LDS, float64 reads them through the scalar cache (float64 VALU issues at one rate
// with or without SGPR operands).
// Capacity of the partial-sum buffer in source splits: up to 64 (at most one split per
// two spheres), so that the split count of a launch can make its last round of resident
// work-groups full (64 x N x 24 B: ~1 GB at 640,000 nodes).
int far_split_capacity(int64_t N, int64_t nb) {
  (void)N;
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, nb / 2));
}

// Source splits of one launch.  The work-groups (grid.x target blocks x splits, all of
// about equal work) run in rounds of `slots` resident ones; the count whose rounds are
// fullest is taken, the fewest splits among equals, between the count that gives ~6144
// work-groups and the capacity of the partial-sum buffer.
static int far_splits(int64_t nb, int64_t tblocks, int cap, int64_t slots) {
  const int lo = (int)std::max<int64_t>(1, std::min<int64_t>({(6144 + tblocks - 1) / tblocks, nb / 2, (int64_t)cap}));
  int best = lo;
  double best_eff = -1.0;
  for (int ns = lo; ns <= cap; ++ns) {
    const int64_t per = (nb + ns - 1) / ns;
    const int64_t used = (nb + per - 1) / per;
    const int64_t w = tblocks * used;
    const double eff = (double)w / (double)(((w + slots - 1) / slots) * slots);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = ns;
    }
  }
  return best;
}

template <typename R, int KIND, int SRC, bool RADII>
static int far_launch_one(bie_ctx* c, FarParams& a, int64_t tblocks, size_t sm) {
  constexpr int TPL = 2;
  int per_cu = 0;
  BIE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, far_kernel<R, KIND, TPL, SRC, RADII>, 256, sm));
  const int64_t slots = (int64_t)std::max(1, per_cu) * c->num_cus;
  const int ns = far_splits(c->nb, tblocks, c->nsplit, slots);
  a.sph_per_split = (int)((c->nb + ns - 1) / ns);
  const int used = (int)((c->nb + a.sph_per_split - 1) / a.sph_per_split);
  far_kernel<R, KIND, TPL, SRC, RADII><<<dim3((unsigned)tblocks, (unsigned)used), dim3(256), sm, c->stream>>>(a);
  return used;
}

template <typename R, int KIND>
static int far_launch(bie_ctx* c, FarParams& a, int64_t tblocks) {
  if constexpr (sizeof(R) == 8) {
    return c->poly ? far_launch_one<R, KIND, 1, true>(c, a, tblocks, 0)
                   : far_launch_one<R, KIND, 1, false>(c, a, tblocks, 0);
  } else {
    const size_t sm = 2 * (size_t)c->P * sizeof(R4<R>);
    return c->poly ? far_launch_one<R, KIND, 0, true>(c, a, tblocks, sm)
                   : far_launch_one<R, KIND, 0, false>(c, a, tblocks, sm);
  }
}

void launch_far(bie_ctx* c, int precision, const OpSpec& spec, double* u) {
  constexpr int TPL = 2;
  FarParams a{};
  const bool f32 = precision == BIE_MIXED;
  a.q = c->q.ptr;
  a.otab = f32 ? c->otab_f.ptr : c->otab.ptr;
  a.osrc = f32 ? c->osrc_f.ptr : c->osrc.ptr;
  a.centres4 = c->centres4.as<double>();
  a.excl = c->excl.as<uint32_t>();
  a.moments = c->moments.as<double>();
  a.radius = c->poly ? c->radius_d.as<double>() : nullptr;
  a.partial = c->partial.as<double>();
  a.N = c->N;
  a.nb = c->nb;
  a.P = c->P;
  a.nwords = c->nwords;
  a.completion = spec.completion ? 1 : 0;
  const int kind = spec.traction ? 4 : (spec.a_s != 0.0 ? 1 : 0) + (spec.a_d != 0.0 ? 2 : 0);
  a.cscale = (kind == 2) ? 3.0 / (4.0 * M_PI) : (kind == 4) ? -3.0 / (4.0 * M_PI) : 1.0 / (8.0 * M_PI);
  const int64_t tblocks = (c->N + 256 * TPL - 1) / (256 * TPL);
  if (kind == 0) throw Error{BIE_EINVAL, "empty far-field kernel"};
  int nsplit = 1;
  if (f32) {
    if (kind == 1) nsplit = far_launch<float, 1>(c, a, tblocks);
    if (kind == 2) nsplit = far_launch<float, 2>(c, a, tblocks);
    if (kind == 3) nsplit = far_launch<float, 3>(c, a, tblocks);
    if (kind == 4) nsplit = far_launch<float, 4>(c, a, tblocks);
  } else {
    if (kind == 1) nsplit = far_launch<double, 1>(c, a, tblocks);
    if (kind == 2) nsplit = far_launch<double, 2>(c, a, tblocks);
    if (kind == 3) nsplit = far_launch<double, 3>(c, a, tblocks);
    if (kind == 4) nsplit = far_launch<double, 4>(c, a, tblocks);
  }
  BIE_HIP(hipGetLastError());
  const int64_t n3 = 3 * c->N;
  const int blocks = (int)std::min<int64_t>((n3 + 255) / 256, 4096);
  reduce_partials<<<dim3(blocks), dim3(256), 0, c->stream>>>(c->partial.as<double>(), nsplit, n3, u);
  BIE_HIP(hipGetLastError());
}

}  // namespace bie
