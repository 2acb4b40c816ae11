// Learned block screener: a 3-layer perceptron x (F) -> H -> H -> 1 (ReLU)
// that predicts log10 of the Frobenius norm of a chi output block (c, c', tau)
// from cheap features of the inputs, trained on the GPU with these kernels:
//   forward (FP16 weights, FP32 math)       mlp_forward_kernel
//   training forward + backprop per sample  mlp_train_fwd_kernel
//   deterministic gradient sums             mlp_grad_kernel (one thread per
//                                           parameter, fixed sample order)
//   Adam (Kingma & Ba, ICLR 2015)           mlp_adam_kernel
// Loss: mean of w(r) r^2 with r = prediction - target, w = 1 for r >= 0 and
// alpha for r < 0 (under-prediction is the unsafe direction for screening).
// Parameters are packed [w1 H*F][b1 H][w2 H*H][b2 H][w3 H][b3 1] in FP32
// (master copy, Adam moments) with an FP16 copy used for inference.
#include <hip/hip_fp16.h>

#include <cmath>
#include <vector>

#include "gw_internal.hpp"

namespace gw {
namespace {

constexpr int kMaxF = 16, kH = 64;

struct Layout {
  int F, H;
  __host__ __device__ int w1() const { return 0; }
  __host__ __device__ int b1() const { return H * F; }
  __host__ __device__ int w2() const { return H * F + H; }
  __host__ __device__ int b2() const { return H * F + H + H * H; }
  __host__ __device__ int w3() const { return H * F + 2 * H + H * H; }
  __host__ __device__ int b3() const { return H * F + 3 * H + H * H; }
  __host__ __device__ int total() const { return H * F + 3 * H + H * H + 1; }
};

// parameters to LDS as float (from the FP16 copy or the FP32 master)
template <class T>
__device__ void load_params(const T* src, float* dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = (float)src[i];
  __syncthreads();
}

__device__ inline float dense_relu_row(const float* w, const float* b, const float* in, int n_in, int j) {
  float a = b[j];
  for (int i = 0; i < n_in; ++i) a += w[j * n_in + i] * in[i];
  return a;
}

template <class T>
__global__ void mlp_forward_kernel(const T* __restrict__ prm, int F, int64_t n,
                                   const float* __restrict__ x, float* __restrict__ y) {
  const Layout L{F, kH};
  extern __shared__ float sp[];
  load_params(prm, sp, L.total());
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    float xin[kMaxF], h1[kH];
    for (int f = 0; f < F; ++f) xin[f] = x[s * F + f];
    for (int j = 0; j < kH; ++j) h1[j] = fmaxf(dense_relu_row(sp + L.w1(), sp + L.b1(), xin, F, j), 0.f);
    float out = sp[L.b3()];
    for (int j = 0; j < kH; ++j) {
      const float h2 = fmaxf(dense_relu_row(sp + L.w2(), sp + L.b2(), h1, kH, j), 0.f);
      out += sp[L.w3() + j] * h2;
    }
    y[s] = out;
  }
}

// per sample: activations and backpropagated signals for the gradient sums
__global__ void mlp_train_fwd_kernel(const float* __restrict__ prm, int F, int n,
                                     const float* __restrict__ x, const float* __restrict__ t,
                                     float alpha, float* __restrict__ h1o, float* __restrict__ h2o,
                                     float* __restrict__ da1o, float* __restrict__ da2o,
                                     float* __restrict__ dyo, float* __restrict__ lo) {
  const Layout L{F, kH};
  extern __shared__ float sp[];
  load_params(prm, sp, L.total());
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  float xin[kMaxF], h1[kH], h2[kH], da2[kH];
  for (int f = 0; f < F; ++f) xin[f] = x[(int64_t)s * F + f];
  for (int j = 0; j < kH; ++j) h1[j] = fmaxf(dense_relu_row(sp + L.w1(), sp + L.b1(), xin, F, j), 0.f);
  float y = sp[L.b3()];
  for (int j = 0; j < kH; ++j) {
    h2[j] = fmaxf(dense_relu_row(sp + L.w2(), sp + L.b2(), h1, kH, j), 0.f);
    y += sp[L.w3() + j] * h2[j];
  }
  const float r = y - t[s];
  const float w = r >= 0.f ? 1.f : alpha;
  const float dy = 2.f * w * r / (float)n;
  for (int j = 0; j < kH; ++j) da2[j] = h2[j] > 0.f ? dy * sp[L.w3() + j] : 0.f;
  for (int i = 0; i < kH; ++i) {
    float d = 0.f;
    for (int j = 0; j < kH; ++j) d += da2[j] * sp[L.w2() + j * kH + i];
    da1o[(int64_t)s * kH + i] = h1[i] > 0.f ? d : 0.f;
    h1o[(int64_t)s * kH + i] = h1[i];
    h2o[(int64_t)s * kH + i] = h2[i];
    da2o[(int64_t)s * kH + i] = da2[i];
  }
  dyo[s] = dy;
  lo[s] = w * r * r / (float)n;
}

// one thread per parameter (+ one for the loss), samples summed in order
__global__ void mlp_grad_kernel(int F, int n, const float* __restrict__ x,
                                const float* __restrict__ h1, const float* __restrict__ h2,
                                const float* __restrict__ da1, const float* __restrict__ da2,
                                const float* __restrict__ dy, const float* __restrict__ ls,
                                float* __restrict__ g, float* __restrict__ loss) {
  const Layout L{F, kH};
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = L.total();
  if (p > P) return;
  float acc = 0.f;
  if (p == P) {
    for (int s = 0; s < n; ++s) acc += ls[s];
    *loss = acc;
    return;
  }
  if (p < L.b1()) {
    const int j = p / F, f = p % F;
    for (int s = 0; s < n; ++s) acc += da1[(int64_t)s * kH + j] * x[(int64_t)s * F + f];
  } else if (p < L.w2()) {
    const int j = p - L.b1();
    for (int s = 0; s < n; ++s) acc += da1[(int64_t)s * kH + j];
  } else if (p < L.b2()) {
    const int q = p - L.w2(), j = q / kH, i = q % kH;
    for (int s = 0; s < n; ++s) acc += da2[(int64_t)s * kH + j] * h1[(int64_t)s * kH + i];
  } else if (p < L.w3()) {
    const int j = p - L.b2();
    for (int s = 0; s < n; ++s) acc += da2[(int64_t)s * kH + j];
  } else if (p < L.b3()) {
    const int j = p - L.w3();
    for (int s = 0; s < n; ++s) acc += dy[s] * h2[(int64_t)s * kH + j];
  } else {
    for (int s = 0; s < n; ++s) acc += dy[s];
  }
  g[p] = acc;
}

__global__ void mlp_adam_kernel(int P, float* __restrict__ prm, __half* __restrict__ prm16,
                                float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float mi = b1 * m[p] + (1.f - b1) * g[p];
  const float vi = b2 * v[p] + (1.f - b2) * g[p] * g[p];
  m[p] = mi;
  v[p] = vi;
  const float w = prm[p] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  prm[p] = w;
  prm16[p] = __float2half(w);
}

__global__ void to_half_kernel(int P, const float* __restrict__ a, __half* __restrict__ b) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) b[p] = __float2half(a[p]);
}

__global__ void features_kernel(int n_tau, int na, const double* __restrict__ tau,
                                const float* __restrict__ dist, const float* __restrict__ tnorm,
                                const float* __restrict__ dno, const float* __restrict__ dnv,
                                float* __restrict__ feat) {
  const int64_t total = (int64_t)n_tau * na * na;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / ((int64_t)na * na));
    const int c = (int)((e / na) % na), c2 = (int)(e % na);
    float* f = feat + e * 6;
    f[0] = dist[(int64_t)c * na + c2] * 0.1f;
    f[1] = (float)log10(tau[j] + 1e-30);
    f[2] = log10f(tnorm[c] + 1e-30f);
    f[3] = log10f(tnorm[c2] + 1e-30f);
    f[4] = log10f(dno[e] + 1e-30f);
    f[5] = log10f(dnv[e] + 1e-30f);
  }
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" gw_status gw_chi_block_features(const gw_system* s, const double* d_occ,
                                           const double* d_vir, int32_t n_tau, const double* tau,
                                           double filter_eps, float* feat, hipStream_t st) {
  clear_error();
  gw_status rc = check_system(s);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(!s->ao_off && !s->ri_off, "the block screener takes systems without per-atom offsets");
  GW_CHECK_ARG(d_occ && d_vir && tau && feat, "null argument");
  GW_CHECK_ARG(s->xyz, "block features need the atom coordinates (gw_system.xyz)");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
  GW_CHECK_ARG(std::isfinite(filter_eps) && filter_eps >= 0, "filter_eps must be >= 0");
  const int na = s->n_atoms, NA = s->ao_per_atom;
  Scratch sc(st);
  BrickGroups G;
  if ((rc = build_groups(s, filter_eps, st, sc, G)) != GW_OK) return rc;
  // norm of the kept tensor restricted to each RI atom
  const int64_t bs = (int64_t)NA * NA * s->ri_per_atom;
  double* d_bn = nullptr;
  if ((rc = sc.alloc(&d_bn, (size_t)std::max<int64_t>(s->n_trip, 1))) != GW_OK) return rc;
  GW_HIP(brick_norms(s->t3c, s->n_trip, bs, d_bn, st));
  std::vector<double> bn(s->n_trip);
  if (s->n_trip) {
    GW_HIP(hipMemcpyAsync(bn.data(), d_bn, sizeof(double) * s->n_trip, hipMemcpyDeviceToHost, st));
    GW_HIP(hipStreamSynchronize(st));
  }
  std::vector<double> tn2(na, 0.0);
  for (int64_t i : G.seg_brick) tn2[s->trip[3 * i + 2]] += bn[i] * bn[i];
  std::vector<float> tnorm(na), dist((size_t)na * na, 0.f);
  for (int c = 0; c < na; ++c) tnorm[c] = (float)std::sqrt(tn2[c]);
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < na; ++b) {
      double d2 = 0;
      for (int k = 0; k < 3; ++k) {
        const double d = s->xyz[3 * a + k] - s->xyz[3 * b + k];
        d2 += d * d;
      }
      dist[(size_t)a * na + b] = (float)std::sqrt(d2);
    }
  float *d_tn, *d_dist, *dno, *dnv;
  double* d_tau;
  if ((rc = sc.upload(&d_tn, tnorm)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_dist, dist)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_tau, std::vector<double>(tau, tau + n_tau))) != GW_OK) return rc;
  if ((rc = sc.alloc(&dno, (size_t)n_tau * na * na)) != GW_OK) return rc;
  if ((rc = sc.alloc(&dnv, (size_t)n_tau * na * na)) != GW_OK) return rc;
  GW_HIP(block_norms_f32(d_occ, n_tau, na, NA, 0, dno, st));
  GW_HIP(block_norms_f32(d_vir, n_tau, na, NA, 0, dnv, st));
  const int64_t total = (int64_t)n_tau * na * na;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)),
                     dim3(256), 0, st, n_tau, na, d_tau, d_dist, d_tn, dno, dnv, feat);
  GW_HIP(hipGetLastError());
  return GW_OK;
}

extern "C" gw_status gw_chi_block_lognorms(const gw_system* s, const double* chi, int32_t n_tau,
                                           float* out, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(s && s->n_atoms > 0 && s->ri_per_atom > 0, "bad system");
  GW_CHECK_ARG(!s->ao_off && !s->ri_off, "block norms take systems without per-atom offsets");
  GW_CHECK_ARG(chi && out && n_tau >= 1, "bad arguments");
  GW_HIP(block_norms_f32(chi, n_tau, s->n_atoms, s->ri_per_atom, 1, out, st));
  return GW_OK;
}

extern "C" int64_t gw_mlp_param_count(int32_t n_features, int32_t hidden) {
  if (n_features < 1 || n_features > kMaxF || hidden != kH) return -1;
  return Layout{n_features, hidden}.total();
}

extern "C" gw_status gw_mlp_forward(const gw_mlp* net, int64_t n, const float* x, float* y,
                                    int32_t use_fp16, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(net && net->params && net->params16 && x && y, "null argument");
  GW_CHECK_ARG(net->n_features >= 1 && net->n_features <= kMaxF && net->hidden == kH,
               "network shape must be F <= 16, H = 64");
  if (n <= 0) return GW_OK;
  const Layout L{net->n_features, kH};
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  const size_t lds = sizeof(float) * L.total();
  if (use_fp16)
    hipLaunchKernelGGL(mlp_forward_kernel<__half>, dim3(blocks), dim3(256), lds, st,
                       (const __half*)net->params16, net->n_features, n, x, y);
  else
    hipLaunchKernelGGL(mlp_forward_kernel<float>, dim3(blocks), dim3(256), lds, st,
                       (const float*)net->params, net->n_features, n, x, y);
  GW_HIP(hipGetLastError());
  return GW_OK;
}

extern "C" gw_status gw_mlp_gradient(const gw_mlp* net, int32_t n, const float* x, const float* t,
                                     float alpha, float* grad, float* loss_dev, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(net && net->params && x && t && grad && loss_dev, "null argument");
  GW_CHECK_ARG(net->n_features >= 1 && net->n_features <= kMaxF && net->hidden == kH,
               "network shape must be F <= 16, H = 64");
  GW_CHECK_ARG(n >= 1 && n <= (1 << 20), "batch size must be in [1, 2^20]");
  GW_CHECK_ARG(std::isfinite(alpha) && alpha > 0, "alpha must be positive");
  const Layout L{net->n_features, kH};
  Scratch sc(st);
  float *h1, *h2, *da1, *da2, *dy, *ls;
  gw_status rc;
  if ((rc = sc.alloc(&h1, (size_t)n * kH)) != GW_OK) return rc;
  if ((rc = sc.alloc(&h2, (size_t)n * kH)) != GW_OK) return rc;
  if ((rc = sc.alloc(&da1, (size_t)n * kH)) != GW_OK) return rc;
  if ((rc = sc.alloc(&da2, (size_t)n * kH)) != GW_OK) return rc;
  if ((rc = sc.alloc(&dy, (size_t)n)) != GW_OK) return rc;
  if ((rc = sc.alloc(&ls, (size_t)n)) != GW_OK) return rc;
  const size_t lds = sizeof(float) * L.total();
  hipLaunchKernelGGL(mlp_train_fwd_kernel, dim3((n + 127) / 128), dim3(128), lds, st, net->params,
                     net->n_features, n, x, t, alpha, h1, h2, da1, da2, dy, ls);
  GW_HIP(hipGetLastError());
  const int P = L.total();
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((P + 1 + 127) / 128), dim3(128), 0, st, net->n_features,
                     n, x, h1, h2, da1, da2, dy, ls, grad, loss_dev);
  GW_HIP(hipGetLastError());
  return GW_OK;
}

extern "C" gw_status gw_mlp_train_step(gw_mlp* net, int32_t n, const float* x, const float* t,
                                       float alpha, float lr, float* loss_dev, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(net && net->params && net->params16 && net->adam_m && net->adam_v && net->grad,
               "network buffers must be set");
  GW_CHECK_ARG(std::isfinite(lr) && lr > 0, "learning rate must be positive");
  gw_status rc = gw_mlp_gradient(net, n, x, t, alpha, net->grad, loss_dev, st);
  if (rc != GW_OK) return rc;
  net->step += 1;
  const int P = Layout{net->n_features, kH}.total();
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((P + 255) / 256), dim3(256), 0, st, P, net->params,
                     (__half*)net->params16, net->adam_m, net->adam_v, net->grad, lr, b1, b2,
                     1e-8f, c1, c2);
  GW_HIP(hipGetLastError());
  return GW_OK;
}

extern "C" gw_status gw_mlp_sync_half(gw_mlp* net, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(net && net->params && net->params16, "network buffers must be set");
  const int P = Layout{net->n_features, kH}.total();
  hipLaunchKernelGGL(to_half_kernel, dim3((P + 255) / 256), dim3(256), 0, st, P, net->params,
                     (__half*)net->params16);
  GW_HIP(hipGetLastError());
  return GW_OK;
}
