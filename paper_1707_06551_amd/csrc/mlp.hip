// The per-pair MLP of the learned coarse correction: forward / backward / Adam kernels,
// the training loss, training and inference.  float32 throughout.
//
// Network: features (8) -> tanh(64) -> tanh(64) -> linear(278) = (theta_off, theta_self);
// weights flattened W1 (8 x 64, in x out), b1, W2 (64 x 64), b2, W3 (64 x 278), b3.
// Loss over configurations with n_rhs samples each (xi = low-mode coefficients of a
// right-hand side b = P xi, t = R x - R M0 b for A x = b):
//   L = sum |t - zeta(xi)|^2 / sum |t|^2,
//   zeta_i = sum_{pairs (i,j)} rot^T [K_off rot xi_j + K_self rot xi_i].
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "bie_internal.h"
#include "coarse.h"

namespace bie {

static constexpr int kNIn = kNFeat, kH = kHidden, kNOut = kNTheta2;
static constexpr int64_t kNW = (int64_t)kNIn * kH + kH + (int64_t)kH * kH + kH + (int64_t)kH * kNOut + kNOut;
static constexpr int64_t kOffW1 = 0, kOffB1 = kNIn * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
                         kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + (int64_t)kH * kNOut;

// Y[b, o] = act(sum_k X[b, k] W[k, o] + bias[o])
__global__ void k_dense_fwd(const float* X, const float* W, const float* bias, int B, int nin, int nout, int tanh_act,
                            float* Y) {
  const int64_t n = (int64_t)B * nout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / nout), o = (int)(e - (int64_t)b * nout);
    float s = bias[o];
    const float* x = X + (int64_t)b * nin;
    for (int k = 0; k < nin; ++k) s = fmaf(x[k], W[(int64_t)k * nout + o], s);
    Y[e] = tanh_act ? tanhf(s) : s;
  }
}

// dZ = dY * (1 - Y^2) in place (tanh layer)
__global__ void k_tanh_bwd(const float* Y, float* dY, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dY[e] *= (1.0f - Y[e] * Y[e]);
}

// dX[b, k] = sum_o dZ[b, o] W[k, o]
__global__ void k_dense_bwd_in(const float* dZ, const float* W, int B, int nin, int nout, float* dX) {
  const int64_t n = (int64_t)B * nin;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / nin), k = (int)(e - (int64_t)b * nin);
    const float* dz = dZ + (int64_t)b * nout;
    const float* w = W + (int64_t)k * nout;
    float s = 0.0f;
    for (int o = 0; o < nout; ++o) s = fmaf(dz[o], w[o], s);
    dX[e] = s;
  }
}

// partial[chunk][k * nout + o] = sum_{b in chunk} X[b, k] dZ[b, o]; bias grads in row nin
__global__ void k_dense_bwd_w(const float* X, const float* dZ, int B, int nin, int nout, int rows_per_chunk,
                              float* partial) {
  const int chunk = blockIdx.y;
  const int64_t nw = (int64_t)(nin + 1) * nout;
  const int b0 = chunk * rows_per_chunk, b1 = min(B, b0 + rows_per_chunk);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / nout), o = (int)(e - (int64_t)k * nout);
    float s = 0.0f;
    if (k < nin)
      for (int b = b0; b < b1; ++b) s = fmaf(X[(int64_t)b * nin + k], dZ[(int64_t)b * nout + o], s);
    else
      for (int b = b0; b < b1; ++b) s += dZ[(int64_t)b * nout + o];
    partial[(int64_t)chunk * nw + e] = s;
  }
}

// grad[W] = sum over chunks (row nin of the partials is the bias gradient)
__global__ void k_sum_chunks(const float* partial, int nchunk, int nin, int nout, float* gW, float* gb) {
  const int64_t nw = (int64_t)(nin + 1) * nout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)c * nw + e];
    const int k = (int)(e / nout);
    if (k < nin)
      gW[e] = s;
    else
      gb[e - (int64_t)nin * nout] = s;
  }
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// contrib[(e, r)] = rot^T (K_off rot xi_j + K_self rot xi_i), one thread per (pair, rhs)
__global__ void k_pair_contrib(const float* theta, const float* frames, const int* pi, const int* pj, int np, int nrhs,
                               const float* xi, float* contrib) {
  const int64_t n = (int64_t)np * nrhs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / nrhs), r = (int)(e - (int64_t)p * nrhs);
    const float* fr = frames + (int64_t)p * kFrame;
    float y[25], x[25], c[25], out[25];
    rot25_apply<float>(fr, xi + ((int64_t)pj[p] * nrhs + r) * 25, y, false);
    rot25_apply<float>(fr, xi + ((int64_t)pi[p] * nrhs + r) * 25, x, false);
    for (int m = 0; m < 25; ++m) c[m] = 0.0f;
    apply_K<float, float>(theta + (int64_t)p * kNTheta2, y, c);
    apply_K<float, float>(theta + (int64_t)p * kNTheta2 + kNTheta, x, c);
    rot25_apply<float>(fr, c, out, true);
    for (int m = 0; m < 25; ++m) contrib[e * 25 + m] = out[m];
  }
}

// per (sphere, rhs): res = t - sum_pairs contrib; gpred = -2 res / den; loss partial
__global__ void k_sphere_res(const int* sph_ptr, int ns, int nrhs, int pbase, const float* contrib,
                             const float* target, float inv_den, float* gpred, double* loss_part) {
  const int64_t n = (int64_t)ns * nrhs;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(e / nrhs), r = (int)(e - (int64_t)s * nrhs);
    float pred[25];
    for (int m = 0; m < 25; ++m) pred[m] = 0.0f;
    for (int p = sph_ptr[s]; p < sph_ptr[s + 1]; ++p)
      for (int m = 0; m < 25; ++m) pred[m] += contrib[((int64_t)(p - pbase) * nrhs + r) * 25 + m];
    for (int m = 0; m < 25; ++m) {
      const float res = target[e * 25 + m] - pred[m];
      acc += (double)res * res;
      gpred[e * 25 + m] = -2.0f * res * inv_den;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0] * (double)inv_den;
}

// dtheta[p] = sum_r dK(u = rot gpred_i, v = rot xi_j) (off) and (u, rot xi_i) (self)
__global__ void k_pair_grad(const float* frames, const int* pi, const int* pj, int np, int nrhs, const float* xi,
                            const float* gpred, float* dtheta) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    float* go = dtheta + p * kNTheta2;
    for (int t = 0; t < kNTheta2; ++t) go[t] = 0.0f;
    const float* fr = frames + p * kFrame;
    for (int r = 0; r < nrhs; ++r) {
      float u[25], y[25], x[25];
      rot25_apply<float>(fr, gpred + ((int64_t)pi[p] * nrhs + r) * 25, u, false);
      rot25_apply<float>(fr, xi + ((int64_t)pj[p] * nrhs + r) * 25, y, false);
      rot25_apply<float>(fr, xi + ((int64_t)pi[p] * nrhs + r) * 25, x, false);
      K_grad_outer<float>(u, y, go);
      K_grad_outer<float>(u, x, go + kNTheta);
    }
  }
}

static int g1d(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

namespace {

struct DevF {
  float* p = nullptr;
  size_t n = 0;
  void alloc(size_t k) {
    release();
    if (k == 0) k = 1;
    if (hipMalloc(&p, k * sizeof(float)) != hipSuccess) {
      p = nullptr;
      throw Error{BIE_ENOMEM, "hipMalloc failed (mlp)"};
    }
    n = k;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DevF() { release(); }
};

// Device-side MLP workspace for a batch of up to Bmax pairs.
struct Net {
  DevF w, g, m, v, h1, h2, y, d2, d1, dx, part;
  int Bmax = 0;
  hipStream_t st = nullptr;
  void init(int bmax, hipStream_t s) {
    Bmax = bmax;
    st = s;
    w.alloc(kNW);
    g.alloc(kNW);
    m.alloc(kNW);
    v.alloc(kNW);
    h1.alloc((size_t)bmax * kH);
    h2.alloc((size_t)bmax * kH);
    y.alloc((size_t)bmax * kNOut);
    d2.alloc((size_t)bmax * kH);
    d1.alloc((size_t)bmax * kH);
    dx.alloc((size_t)bmax * kNIn);
    part.alloc((size_t)64 * (kH + 1) * kNOut);
    BIE_HIP(hipMemsetAsync(m.p, 0, kNW * sizeof(float), st));
    BIE_HIP(hipMemsetAsync(v.p, 0, kNW * sizeof(float), st));
  }
  void forward(const float* X, int B) {
    k_dense_fwd<<<g1d((int64_t)B * kH), 256, 0, st>>>(X, w.p + kOffW1, w.p + kOffB1, B, kNIn, kH, 1, h1.p);
    k_dense_fwd<<<g1d((int64_t)B * kH), 256, 0, st>>>(h1.p, w.p + kOffW2, w.p + kOffB2, B, kH, kH, 1, h2.p);
    k_dense_fwd<<<g1d((int64_t)B * kNOut), 256, 0, st>>>(h2.p, w.p + kOffW3, w.p + kOffB3, B, kH, kNOut, 0, y.p);
    BIE_HIP(hipGetLastError());
  }
  void wgrad(const float* Xin, const float* dZ, int B, int nin, int nout, float* gW, float* gb) {
    const int nchunk = std::max(1, std::min(64, (B + 255) / 256));
    const int rows = (B + nchunk - 1) / nchunk;
    k_dense_bwd_w<<<dim3(g1d((int64_t)(nin + 1) * nout), nchunk), 256, 0, st>>>(Xin, dZ, B, nin, nout, rows, part.p);
    k_sum_chunks<<<g1d((int64_t)(nin + 1) * nout), 256, 0, st>>>(part.p, nchunk, nin, nout, gW, gb);
  }
  // dY (B x 278) -> weight gradient g
  void backward(const float* X, float* dY, int B) {
    wgrad(h2.p, dY, B, kH, kNOut, g.p + kOffW3, g.p + kOffB3);
    k_dense_bwd_in<<<g1d((int64_t)B * kH), 256, 0, st>>>(dY, w.p + kOffW3, B, kH, kNOut, d2.p);
    k_tanh_bwd<<<g1d((int64_t)B * kH), 256, 0, st>>>(h2.p, d2.p, (int64_t)B * kH);
    wgrad(h1.p, d2.p, B, kH, kH, g.p + kOffW2, g.p + kOffB2);
    k_dense_bwd_in<<<g1d((int64_t)B * kH), 256, 0, st>>>(d2.p, w.p + kOffW2, B, kH, kH, d1.p);
    k_tanh_bwd<<<g1d((int64_t)B * kH), 256, 0, st>>>(h1.p, d1.p, (int64_t)B * kH);
    wgrad(X, d1.p, B, kNIn, kH, g.p + kOffW1, g.p + kOffB1);
    BIE_HIP(hipGetLastError());
  }
};

template <typename T>
void up(DevF& d, const T* src, size_t n) {
  static_assert(sizeof(T) == sizeof(float), "float data");
  d.alloc(n);
  BIE_HIP(hipMemcpy(d.p, src, n * sizeof(float), hipMemcpyHostToDevice));
}

struct Data {
  DevF feats, frames, xi, target, contrib, gpred, dtheta;
  int* pi = nullptr;
  int* pj = nullptr;
  int* sptr = nullptr;
  double* loss_part = nullptr;
  double den = 0.0;
  ~Data() {
    if (pi) (void)hipFree(pi);
    if (pj) (void)hipFree(pj);
    if (sptr) (void)hipFree(sptr);
    if (loss_part) (void)hipFree(loss_part);
  }
};

void check_data(const bie_mlp_data* d) {
  if (!d || d->n_pairs < 0 || d->n_spheres <= 0 || d->n_rhs <= 0 || d->n_configs <= 0 || !d->feats || !d->frames ||
      !d->pair_i || !d->pair_j || !d->sph_ptr || !d->xi || !d->target || !d->cfg_sph || !d->cfg_pair)
    throw Error{BIE_EINVAL, "incomplete bie_mlp_data"};
  if (d->sph_ptr[0] != 0 || d->sph_ptr[d->n_spheres] != d->n_pairs) throw Error{BIE_EINVAL, "bad sph_ptr"};
  for (int64_t p = 0; p < d->n_pairs; ++p)
    if (d->pair_i[p] < 0 || d->pair_i[p] >= d->n_spheres || d->pair_j[p] < 0 || d->pair_j[p] >= d->n_spheres)
      throw Error{BIE_EINVAL, "pair index out of range"};
  for (int64_t s = 0; s < d->n_spheres; ++s)
    for (int p = d->sph_ptr[s]; p < d->sph_ptr[s + 1]; ++p)
      if (d->pair_i[p] != s) throw Error{BIE_EINVAL, "pairs must be grouped by target sphere"};
  if (d->cfg_sph[0] != 0 || d->cfg_sph[d->n_configs] != d->n_spheres || d->cfg_pair[0] != 0 ||
      d->cfg_pair[d->n_configs] != d->n_pairs)
    throw Error{BIE_EINVAL, "bad configuration offsets"};
}

void upload_data(const bie_mlp_data* d, Data& D) {
  up(D.feats, d->feats, (size_t)d->n_pairs * kNFeat);
  up(D.frames, d->frames, (size_t)d->n_pairs * kFrame);
  up(D.xi, d->xi, (size_t)d->n_spheres * d->n_rhs * 25);
  up(D.target, d->target, (size_t)d->n_spheres * d->n_rhs * 25);
  D.contrib.alloc((size_t)std::max<int64_t>(1, d->n_pairs) * d->n_rhs * 25);
  D.gpred.alloc((size_t)d->n_spheres * d->n_rhs * 25);
  D.dtheta.alloc((size_t)std::max<int64_t>(1, d->n_pairs) * kNTheta2);
  auto upi = [](int*& dst, const int32_t* src, size_t n) {
    if (hipMalloc(&dst, std::max<size_t>(1, n) * sizeof(int)) != hipSuccess) throw Error{BIE_ENOMEM, "hipMalloc"};
    BIE_HIP(hipMemcpy(dst, src, n * sizeof(int), hipMemcpyHostToDevice));
  };
  upi(D.pi, d->pair_i, d->n_pairs);
  upi(D.pj, d->pair_j, d->n_pairs);
  upi(D.sptr, d->sph_ptr, d->n_spheres + 1);
  if (hipMalloc(&D.loss_part, 16384 * sizeof(double)) != hipSuccess) throw Error{BIE_ENOMEM, "hipMalloc"};
  double den = 0.0;
  for (int64_t e = 0; e < d->n_spheres * d->n_rhs * 25; ++e) den += (double)d->target[e] * d->target[e];
  D.den = den > 0 ? den : 1.0;
}

// Loss and weight gradient of the configurations [c0, c1) (pairs and spheres contiguous).
double loss_grad_batch(const bie_mlp_data* d, Data& D, Net& net, int c0, int c1) {
  const int p0 = d->cfg_pair[c0], p1 = d->cfg_pair[c1];
  const int s0 = d->cfg_sph[c0], s1 = d->cfg_sph[c1];
  const int np = p1 - p0, ns = s1 - s0, nr = d->n_rhs;
  hipStream_t st = net.st;
  if (np == 0) {
    BIE_HIP(hipMemsetAsync(net.g.p, 0, kNW * sizeof(float), st));
    return 0.0;
  }
  // sphere-local views: pair indices are global; rebase them to this batch
  net.forward(D.feats.p + (size_t)p0 * kNFeat, np);
  k_pair_contrib<<<g1d((int64_t)np * nr), 256, 0, st>>>(net.y.p, D.frames.p + (size_t)p0 * kFrame, D.pi + p0,
                                                        D.pj + p0, np, nr, D.xi.p, D.contrib.p);
  // sph_ptr holds global pair indices; contrib is indexed by (pair - p0)
  const int blocks = std::min(g1d((int64_t)ns * nr), 16384);
  k_sphere_res<<<blocks, 256, 0, st>>>(D.sptr + s0, ns, nr, p0, D.contrib.p,
                                       D.target.p + (size_t)s0 * nr * 25, (float)(1.0 / D.den),
                                       D.gpred.p + (size_t)s0 * nr * 25, D.loss_part);
  k_pair_grad<<<g1d(np), 256, 0, st>>>(D.frames.p + (size_t)p0 * kFrame, D.pi + p0, D.pj + p0, np, nr, D.xi.p,
                                        D.gpred.p, D.dtheta.p);
  BIE_HIP(hipGetLastError());
  net.backward(D.feats.p + (size_t)p0 * kNFeat, D.dtheta.p, np);
  std::vector<double> lp(blocks);
  BIE_HIP(hipMemcpyAsync(lp.data(), D.loss_part, blocks * sizeof(double), hipMemcpyDeviceToHost, st));
  BIE_HIP(hipStreamSynchronize(st));
  double L = 0.0;
  for (double x : lp) L += x;
  return L;
}

int max_batch_pairs(const bie_mlp_data* d, int cfg_per_batch) {
  int mx = 1;
  for (int c = 0; c < d->n_configs; c += cfg_per_batch) {
    const int c1 = std::min<int>((int)d->n_configs, c + cfg_per_batch);
    mx = std::max(mx, d->cfg_pair[c1] - d->cfg_pair[c]);
  }
  return mx;
}

}  // namespace

int64_t mlp_n_weights() { return kNW; }

double mlp_eval(const bie_mlp_data* d, const float* weights, float* grad) {
  check_data(d);
  Data D;
  upload_data(d, D);
  Net net;
  net.init((int)std::max<int64_t>(1, d->n_pairs), nullptr);
  BIE_HIP(hipMemcpy(net.w.p, weights, kNW * sizeof(float), hipMemcpyHostToDevice));
  const double L = loss_grad_batch(d, D, net, 0, (int)d->n_configs);
  BIE_HIP(hipMemcpy(grad, net.g.p, kNW * sizeof(float), hipMemcpyDeviceToHost));
  return L;
}

void mlp_train(const bie_mlp_data* d, float* weights, int epochs, int cfg_per_batch, double lr, double* loss_hist) {
  check_data(d);
  if (epochs < 0 || cfg_per_batch <= 0 || !(lr > 0)) throw Error{BIE_EINVAL, "bad training options"};
  Data D;
  upload_data(d, D);
  Net net;
  net.init(max_batch_pairs(d, cfg_per_batch), nullptr);
  BIE_HIP(hipMemcpy(net.w.p, weights, kNW * sizeof(float), hipMemcpyHostToDevice));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  int64_t step = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    double Lsum = 0.0;
    for (int c = 0; c < d->n_configs; c += cfg_per_batch) {
      const int c1 = std::min<int>((int)d->n_configs, c + cfg_per_batch);
      Lsum += loss_grad_batch(d, D, net, c, c1);
      ++step;
      const float c1f = 1.0f - std::pow(b1, (float)step), c2f = 1.0f - std::pow(b2, (float)step);
      k_adam<<<g1d(kNW), 256, 0, net.st>>>(net.w.p, net.g.p, net.m.p, net.v.p, kNW, (float)lr, b1, b2, c1f, c2f, eps);
      BIE_HIP(hipGetLastError());
    }
    if (loss_hist) loss_hist[ep] = Lsum;
  }
  BIE_HIP(hipMemcpy(weights, net.w.p, kNW * sizeof(float), hipMemcpyDeviceToHost));
}

// Inference on a context: theta for every directed close pair from the stored features.
void mlp_infer(bie_ctx* c, const float* weights) {
  const int64_t np = (int64_t)c->close_idx.size();
  c->mlp_theta.alloc((size_t)std::max<int64_t>(1, np) * kNTheta2 * sizeof(float));
  c->theta_ready = false;
  if (np == 0) {
    c->theta_ready = true;
    return;
  }
  for (int64_t i = 0; i < kNW; ++i)
    if (!std::isfinite(weights[i])) throw Error{BIE_EINVAL, "non-finite MLP weight"};
  Net net;
  net.init((int)np, c->stream);
  BIE_HIP(hipMemcpyAsync(net.w.p, weights, kNW * sizeof(float), hipMemcpyHostToDevice, c->stream));
  DevF X;
  X.alloc((size_t)np * kNFeat);
  BIE_HIP(hipMemcpyAsync(X.p, c->pair_feat.data(), (size_t)np * kNFeat * sizeof(float), hipMemcpyHostToDevice,
                         c->stream));
  net.forward(X.p, (int)np);
  BIE_HIP(hipMemcpyAsync(c->mlp_theta.ptr, net.y.p, (size_t)np * kNTheta2 * sizeof(float), hipMemcpyDeviceToDevice,
                         c->stream));
  BIE_HIP(hipStreamSynchronize(c->stream));
  c->theta_ready = true;
}

}  // namespace bie
