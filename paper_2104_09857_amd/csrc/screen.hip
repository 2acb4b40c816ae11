// Screening (Eqs. 5-9), FP64.  RI overlap metric S = 1 (chi~ = chi).
//   chi(i w_k)   = 2 s sum_j c_kj chi(tau_j)                 stack transform
//   V = L L^T                                                 Cholesky (Eq. 8)
//   A_k = L^T chi(i w_k) L,  eps_k = 1 - A_k                  (Eq. 7)
//   W^c(i w_k) = L [eps_k^-1 - 1] L^T = L (eps_k^-1 A_k) L^T  (Eq. 9)
//   W^c(tau_j) = 1/2 sum_k d_jk W^c(i w_k)                    stack transform
// eps_k^-1 A_k is obtained from the Cholesky factor of eps_k (two triangular
// solves).  With an RI overlap metric S (Eq. 5; W~^c and V~ of Eqs. 10-11),
// S^-1 enters only through M = S^-1 L:
//   L^T (S^-1 chi S^-1) L = M^T chi M,  S^-1 L Y L^T S^-1 = M Y M^T,
//   V~ = S^-1 L L^T S^-1 = M M^T,
// so the metric form runs the same steps with M (general, two GEMMs) in place
// of the triangular L, after one Cholesky factorization of S and one solve.  Dense FP64 factorizations and triangular products come from
// rocSOLVER / rocBLAS; the stack transforms and the shift are HBM-bound
// kernels here.  All matrices except L are symmetric, so the row-major
// buffers are handed to the column-major libraries unchanged.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "gw_internal.hpp"

namespace gw {
namespace {

constexpr int kMaxStack = 32;

// out[k][e] = sum_j coef[k][j] in[j][e] for a stack of n_in matrices of n2 elements
// out[k] = sum_j coef[k][j] (in[j] + in2[j]) (in2 may be null)
__global__ void stack_transform_kernel(const double* __restrict__ in, const double* __restrict__ in2,
                                       double* __restrict__ out, const double* __restrict__ coef,
                                       int n_in, int n_out, int64_t n2) {
  extern __shared__ double cs[];
  for (int i = threadIdx.x; i < n_in * n_out; i += blockDim.x) cs[i] = coef[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v[kMaxStack];
#pragma unroll
    for (int j = 0; j < kMaxStack; ++j)
      v[j] = j < n_in ? in[(int64_t)j * n2 + e] + (in2 ? in2[(int64_t)j * n2 + e] : 0.0) : 0.0;
    for (int k = 0; k < n_out; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxStack; ++j)
        if (j < n_in) s += cs[k * n_in + j] * v[j];
      out[(int64_t)k * n2 + e] = s;
    }
  }
}

// b = 1 - a (n x n)
__global__ void one_minus_kernel(const double* __restrict__ a, double* __restrict__ b, int n) {
  const int64_t n2 = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e % n;
    b[e] = (r == c ? 1.0 : 0.0) - a[e];
  }
}

// m = lower triangle of l (column-major n x n), zeros above the diagonal
__global__ void lower_part_kernel(const double* __restrict__ l, double* __restrict__ m, int n) {
  const int64_t n2 = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t col = e / n, row = e % n;
    m[e] = row >= col ? l[e] : 0.0;
  }
}

hipError_t stack_transform(const double* in, const double* in2, double* out, const double* coef_dev,
                           int n_in, int n_out, int64_t n2, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<int64_t>((n2 + 255) / 256, 16384);
  hipLaunchKernelGGL(stack_transform_kernel, dim3(blocks), dim3(256),
                     sizeof(double) * n_in * n_out, st, in, in2, out, coef_dev, n_in, n_out, n2);
  return hipGetLastError();
}

std::mutex g_handle_mu;
rocblas_handle g_handle[64] = {};

gw_status get_handle(hipStream_t st, rocblas_handle* h) {
  int dev = 0;
  GW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return GW_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_handle_mu);
  if (!g_handle[dev]) {
    if (rocblas_create_handle(&g_handle[dev]) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return GW_ERR_BLAS;
    }
  }
  if (rocblas_set_stream(g_handle[dev], st) != rocblas_status_success) {
    set_error("rocblas_set_stream failed");
    return GW_ERR_BLAS;
  }
  *h = g_handle[dev];
  return GW_OK;
}

}  // namespace
}  // namespace gw

// Releases the per-device rocBLAS / rocSOLVER handles the screening calls
// keep between calls; later calls create them again.
extern "C" gw_status gw_finalize(void) {
  gw::clear_error();
  std::lock_guard<std::mutex> lk(gw::g_handle_mu);
  int cur = 0;
  GW_HIP(hipGetDevice(&cur));
  gw_status rc = GW_OK;
  for (int dev = 0; dev < 64; ++dev) {
    if (!gw::g_handle[dev]) continue;
    if (hipSetDevice(dev) != hipSuccess || rocblas_destroy_handle(gw::g_handle[dev]) != rocblas_status_success) {
      gw::set_error("releasing the rocBLAS handle of device " + std::to_string(dev) + " failed");
      rc = GW_ERR_BLAS;
    }
    gw::g_handle[dev] = nullptr;
  }
  GW_HIP(hipSetDevice(cur));
  return rc;
}

namespace gw {
namespace {

#define GW_BLAS(call)                                                          \
  do {                                                                         \
    rocblas_status s_ = (call);                                                \
    if (s_ != rocblas_status_success) {                                        \
      ::gw::set_error(std::string("rocBLAS/rocSOLVER error in ") + #call +     \
                      ": " + rocblas_status_to_string(s_));                    \
      return GW_ERR_BLAS;                                                      \
    }                                                                          \
  } while (0)

}  // namespace
}  // namespace gw

using namespace gw;

namespace {
// W^c from chi + chi2 (chi2 may be null), spin factor `spin` (Eqs. 5-9); with
// an RI overlap Smet (may be null: S = 1) the output is W~^c and v_tilde (may
// be null) receives V~
gw_status screen_impl(const gw_system* s, const double* chi, const double* chi2, const double* V,
                      const double* Smet, int32_t n_tau, int32_t n_w, const double* cos_w,
                      const double* icos_w, double spin, double* wc, double* v_tilde,
                      hipStream_t st) {
  gw_status rc0 = check_system_sizes(s);
  if (rc0 != GW_OK) return rc0;
  const int64_t n64 = sys_n_ri(s);   // the screening is dense over the RI functions
  GW_CHECK_ARG(n64 < 46341, "n_ri too large for 32-bit BLAS indexing");
  const int n = (int)n64;
  GW_CHECK_ARG(chi && V && wc && cos_w && icos_w, "null pointer argument");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= kMaxStack && n_w >= 1 && n_w <= kMaxStack,
               "n_tau and n_w must be in [1, 32]");
  GW_CHECK_ARG(std::isfinite(spin) && spin > 0, "spin factor must be positive");
  for (int i = 0; i < n_tau * n_w; ++i)
    GW_CHECK_ARG(std::isfinite(cos_w[i]) && std::isfinite(icos_w[i]), "non-finite transform weight");

  rocblas_handle h;
  gw_status rc = get_handle(st, &h);
  if (rc != GW_OK) return rc;

  const int64_t n2 = (int64_t)n * n;
  Scratch sc(st);
  double *L, *S, *T1, *T2, *coef, *M = nullptr, *LS = nullptr;
  rocblas_int* info;
  if ((rc = sc.alloc(&L, n2)) != GW_OK) return rc;
  if ((rc = sc.alloc(&S, n2 * n_w)) != GW_OK) return rc;
  if ((rc = sc.alloc(&T1, n2)) != GW_OK) return rc;
  if ((rc = sc.alloc(&T2, n2)) != GW_OK) return rc;
  if ((rc = sc.alloc(&info, n_w + 2)) != GW_OK) return rc;
  if (Smet) {
    if ((rc = sc.alloc(&M, n2)) != GW_OK) return rc;
    if ((rc = sc.alloc(&LS, n2)) != GW_OK) return rc;
  }
  std::vector<double> cf((size_t)n_w * n_tau), icf((size_t)n_tau * n_w);
  for (int k = 0; k < n_w; ++k)
    for (int j = 0; j < n_tau; ++j) cf[(size_t)k * n_tau + j] = 2.0 * spin * cos_w[k * n_tau + j];
  for (int j = 0; j < n_tau; ++j)
    for (int k = 0; k < n_w; ++k) icf[(size_t)j * n_w + k] = 0.5 * icos_w[j * n_w + k];
  std::vector<double> both(cf);
  both.insert(both.end(), icf.begin(), icf.end());
  if ((rc = sc.upload(&coef, both)) != GW_OK) return rc;
  GW_HIP(hipMemsetAsync(info, 0, sizeof(rocblas_int) * (n_w + 2), st));

  // V = L L^T
  GW_HIP(hipMemcpyAsync(L, V, sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
  GW_BLAS(rocsolver_dpotrf(h, rocblas_fill_lower, n, L, n, info + n_w));
  const double zero = 0.0;
  const unsigned eb = (unsigned)std::min<int64_t>((n2 + 255) / 256, 16384);
  if (Smet) {
    // M = S^-1 L: S = R R^T, two triangular solves on the lower part of L
    hipLaunchKernelGGL(lower_part_kernel, dim3(eb), dim3(256), 0, st, L, M, n);
    GW_HIP(hipGetLastError());
    GW_HIP(hipMemcpyAsync(LS, Smet, sizeof(double) * n2, hipMemcpyDeviceToDevice, st));
    GW_BLAS(rocsolver_dpotrf(h, rocblas_fill_lower, n, LS, n, info + n_w + 1));
    GW_BLAS(rocsolver_dpotrs(h, rocblas_fill_lower, n, n, LS, n, M, n));
  }

  // chi(i w_k) for all k
  GW_HIP(stack_transform(chi, chi2, S, coef, n_tau, n_w, n2, st));
  const double one = 1.0;
  for (int k = 0; k < n_w; ++k) {
    double* X = S + (int64_t)k * n2;
    // A = L^T X L, or M^T X M with the metric (into T2)
    if (Smet) {
      GW_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, X, n,
                            M, n, &zero, T1, n));
      GW_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one,
                            M, n, T1, n, &zero, T2, n));
    } else {
      GW_BLAS(rocblas_dtrmm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_transpose,
                            rocblas_diagonal_non_unit, n, n, &one, L, n, X, n, T1, n));
      GW_BLAS(rocblas_dtrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                            rocblas_diagonal_non_unit, n, n, &one, L, n, T1, n, T2, n));
    }
    // eps = 1 - A, Cholesky
    hipLaunchKernelGGL(one_minus_kernel, dim3(eb), dim3(256), 0, st, T2, T1, n);
    GW_HIP(hipGetLastError());
    GW_BLAS(rocsolver_dpotrf(h, rocblas_fill_lower, n, T1, n, info + k));
    // Y = eps^-1 A (in T2)
    GW_BLAS(rocsolver_dpotrs(h, rocblas_fill_lower, n, n, T1, n, T2, n));
    // W^c(i w_k) = L Y L^T, or W~^c = M Y M^T with the metric (into X)
    if (Smet) {
      GW_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n, n, n, &one, M, n,
                            T2, n, &zero, T1, n));
      GW_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one,
                            T1, n, M, n, &zero, X, n));
    } else {
      GW_BLAS(rocblas_dtrmm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                            rocblas_diagonal_non_unit, n, n, &one, L, n, T2, n, T1, n));
      GW_BLAS(rocblas_dtrmm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                            rocblas_diagonal_non_unit, n, n, &one, L, n, T1, n, X, n));
    }
  }
  // V~ = M M^T
  if (Smet && v_tilde)
    GW_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, M,
                          n, M, n, &zero, v_tilde, n));
  // W^c(tau_j)
  GW_HIP(stack_transform(S, nullptr, wc, coef + (size_t)n_w * n_tau, n_w, n_tau, n2, st));

  std::vector<rocblas_int> hinfo(n_w + 2);
  GW_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * (n_w + 2), hipMemcpyDeviceToHost, st));
  GW_HIP(hipStreamSynchronize(st));
  if (hinfo[n_w] != 0) {
    set_error("V is not positive definite (potrf info " + std::to_string(hinfo[n_w]) + ")");
    return GW_ERR_NOT_SPD;
  }
  if (hinfo[n_w + 1] != 0) {
    set_error("S is not positive definite (potrf info " + std::to_string(hinfo[n_w + 1]) + ")");
    return GW_ERR_NOT_SPD;
  }
  for (int k = 0; k < n_w; ++k)
    if (hinfo[k] != 0) {
      set_error("epsilon(i w_" + std::to_string(k) + ") is not positive definite (potrf info " +
                std::to_string(hinfo[k]) + ")");
      return GW_ERR_NOT_SPD;
    }
  return GW_OK;
}
}  // namespace

extern "C" gw_status gw_screen_w(const gw_system* s, const double* chi, const double* V,
                                 int32_t n_tau, int32_t n_w, const double* cos_w,
                                 const double* icos_w, double spin, double* wc, hipStream_t st) {
  clear_error();
  return screen_impl(s, chi, nullptr, V, nullptr, n_tau, n_w, cos_w, icos_w, spin, wc, nullptr, st);
}

extern "C" gw_status gw_screen_w_metric(const gw_system* s, const double* chi, const double* V,
                                        const double* S_ri, int32_t n_tau, int32_t n_w,
                                        const double* cos_w, const double* icos_w, double spin,
                                        double* wc_tilde, double* v_tilde, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(S_ri != nullptr, "null pointer argument");
  return screen_impl(s, chi, nullptr, V, S_ri, n_tau, n_w, cos_w, icos_w, spin, wc_tilde, v_tilde,
                     st);
}

extern "C" gw_status gw_screen_w_spins(const gw_system* s, const double* chi_up,
                                       const double* chi_dn, const double* V, int32_t n_tau,
                                       int32_t n_w, const double* cos_w, const double* icos_w,
                                       double* wc, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(chi_up && chi_dn, "null pointer argument");
  return screen_impl(s, chi_up, chi_dn, V, nullptr, n_tau, n_w, cos_w, icos_w, 1.0, wc, nullptr, st);
}

extern "C" gw_status gw_screen_w_spins_metric(const gw_system* s, const double* chi_up,
                                              const double* chi_dn, const double* V,
                                              const double* S_ri, int32_t n_tau, int32_t n_w,
                                              const double* cos_w, const double* icos_w,
                                              double* wc_tilde, double* v_tilde, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(chi_up && chi_dn && S_ri, "null pointer argument");
  return screen_impl(s, chi_up, chi_dn, V, S_ri, n_tau, n_w, cos_w, icos_w, 1.0, wc_tilde, v_tilde,
                     st);
}

// ---------------------------------------------------------------------------
// Periodic Coulomb matrix (Eq. 8 for a periodic Gamma-point cell, obtained by
// Ewald summation).  RI functions are normalized Gaussian charges (exponent
// a_P, centre R_P) in an orthorhombic cell of volume Omega with a
// neutralizing background (G = 0 left out).  With 1/mu = 1/a_P + 1/a_Q and a
// splitting parameter eta < sqrt(mu) for every pair:
//   V_PQ = sum_images [erf(sqrt(mu) r) - erf(eta r)] / r             (real)
//        + (4 pi / Omega) sum_{G != 0} exp(-G^2/(4 eta^2)) cos(G.R_PQ)/G^2
//        - (pi / Omega) (1/eta^2 - 1/mu)                              (background)
// The reciprocal sum is separable: with F_P = sqrt(w_G) [cos G.R_P, sin G.R_P]
// over the half space of G (w_G = 2 (4 pi/Omega) e^{-G^2/4eta^2}/G^2), it is
// F F^T, a dense FP64 GEMM on the matrix cores; the real-space sum is an
// elementwise kernel over the lattice images within the cutoff.  eta trades
// one for the other and is chosen by a cost model unless given.
namespace {

constexpr double kPi = 3.14159265358979323846;

__global__ void ewald_phase_kernel(const double* __restrict__ centres, const double* __restrict__ gw4,
                                   int n_ri, int n_g, double* __restrict__ F) {
  // F row-major [n_ri][2 n_g]: (P, g) -> sqrt(w_g) cos(G_g . R_P), (P, n_g + g) -> sin
  const int64_t total = (int64_t)n_ri * n_g;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / n_g;
    const int g = (int)(e % n_g);
    const double ph = gw4[4 * g] * centres[3 * p] + gw4[4 * g + 1] * centres[3 * p + 1] +
                      gw4[4 * g + 2] * centres[3 * p + 2];
    double s, c;
    sincos(ph, &s, &c);
    const double w = gw4[4 * g + 3];
    F[p * 2 * n_g + g] = w * c;
    F[p * 2 * n_g + n_g + g] = w * s;
  }
}

// [erf(sqrt(mu) r) - erf(eta r)] / r, accurate at small and large r
__device__ inline double short_range(double smu, double eta, double r) {
  if (r < 1e-10) return 2.0 * (smu - eta) * 0.56418958354775628695;   // 1/sqrt(pi)
  const double d = eta * r > 0.5 ? erfc(eta * r) - erfc(smu * r) : erf(smu * r) - erf(eta * r);
  return d / r;
}

// images: n_img lattice vectors (x, y, z) whose distance to the box of
// minimum-image displacements is within r_cut (the only ones that can be)
__global__ void ewald_real_kernel(const double* __restrict__ centres, const double* __restrict__ alpha,
                                  int n_ri, double lx, double ly, double lz,
                                  const double* __restrict__ images, int n_img, double eta,
                                  double r_cut, double inv_omega, double* __restrict__ V) {
  // the real-space part is symmetric in (P, Q): element (p, q >= p) adds
  // to V_pq and V_qp (each pair owned by one thread)
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= n_ri || q < p) return;
  const double ap = alpha[p], aq = alpha[q];
  const double mu = ap * aq / (ap + aq);
  const double smu = sqrt(mu);
  double dx = centres[3 * p] - centres[3 * q];
  double dy = centres[3 * p + 1] - centres[3 * q + 1];
  double dz = centres[3 * p + 2] - centres[3 * q + 2];
  dx -= lx * rint(dx / lx);
  dy -= ly * rint(dy / ly);
  dz -= lz * rint(dz / lz);
  const double rc2 = r_cut * r_cut;
  double acc = 0.0;
  for (int m = 0; m < n_img; ++m) {
    const double x = dx + images[3 * m], y = dy + images[3 * m + 1], z = dz + images[3 * m + 2];
    const double r2 = x * x + y * y + z * z;
    if (r2 <= rc2) acc += short_range(smu, eta, sqrt(r2));
  }
  acc -= kPi * inv_omega * (1.0 / (eta * eta) - 1.0 / mu);
  V[(int64_t)p * n_ri + q] += acc;
  if (q != p) V[(int64_t)q * n_ri + p] += acc;
}

// x with erfc(x) <= tol
double erfc_root(double tol) {
  double lo = 0.0, hi = 30.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    (std::erfc(mid) > tol ? lo : hi) = mid;
  }
  return hi;
}

struct EwaldPlan {
  double eta, r_cut, g_cut;
  int nx, ny, nz;
  int64_t n_img, n_g_est;
};

EwaldPlan ewald_plan(double eta, const double* cell, double omega, double tol) {
  EwaldPlan pl;
  pl.eta = eta;
  pl.r_cut = erfc_root(tol) / eta;
  // reciprocal cutoff: (4 pi/Omega) e^{-G^2/(4 eta^2)} / G^2 <= tol
  double g = 2.0 * eta * std::sqrt(std::log(1.0 / tol));
  for (int it = 0; it < 3; ++it) {
    const double arg = 4.0 * kPi / (omega * tol * std::max(g * g, 1e-300));
    g = 2.0 * eta * std::sqrt(std::max(std::log(std::max(arg, 1.0)), 0.0));
  }
  pl.g_cut = g * 1.02;
  // images per direction, clamped before the int conversion (the caller
  // rejects boxes beyond its bound)
  auto n_img_dir = [&](double l) { return (int)std::min(std::ceil(pl.r_cut / l + 0.5), 1.0e6); };
  pl.nx = n_img_dir(cell[0]);
  pl.ny = n_img_dir(cell[1]);
  pl.nz = n_img_dir(cell[2]);
  const double ball = 4.0 / 3.0 * kPi * pl.r_cut * pl.r_cut * pl.r_cut;
  pl.n_img = std::min<int64_t>((int64_t)(2 * pl.nx + 1) * (2 * pl.ny + 1) * (2 * pl.nz + 1),
                               (int64_t)(ball / omega) + 1);
  pl.n_g_est = (int64_t)(4.0 / 3.0 * kPi * std::pow(pl.g_cut, 3) * omega / std::pow(2.0 * kPi, 3) / 2.0) + 1;
  return pl;
}

}  // namespace

extern "C" gw_status gw_coulomb_periodic(int32_t n_ri, const double* centres, const double* alpha,
                                         const double* cell, double eta, double tol, double* V,
                                         gw_coulomb_info* info, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(n_ri >= 1 && n_ri < 46341, "n_ri must be in [1, 46340]");
  GW_CHECK_ARG(centres && alpha && cell && V, "null pointer argument");
  GW_CHECK_ARG(std::isfinite(tol) && tol > 0.0 && tol <= 1e-6, "tol must be in (0, 1e-6]");
  for (int i = 0; i < 3; ++i) GW_CHECK_ARG(std::isfinite(cell[i]) && cell[i] > 0.0, "bad cell");
  double a_min = INFINITY;
  for (int p = 0; p < n_ri; ++p) {
    GW_CHECK_ARG(std::isfinite(alpha[p]) && alpha[p] > 0.0, "exponents must be positive");
    for (int i = 0; i < 3; ++i) GW_CHECK_ARG(std::isfinite(centres[3 * p + i]), "non-finite centre");
    a_min = std::min(a_min, alpha[p]);
  }
  const double omega = cell[0] * cell[1] * cell[2];
  const double smu_min = std::sqrt(0.5 * a_min);
  GW_CHECK_ARG(eta == 0.0 || (std::isfinite(eta) && eta > 0.0 && eta < smu_min),
               "eta must be 0 (automatic) or in (0, sqrt(min alpha / 2))");
  EwaldPlan pl;
  if (eta > 0.0) {
    pl = ewald_plan(eta, cell, omega, tol);
  } else {
    // cost per pair: ~60 ALU flops per image in range, ~4 matrix-core flops
    // (at ~10x the vector rate) plus the phase build per half-space G
    double best = INFINITY;
    for (int i = 0; i < 48; ++i) {
      const double e = smu_min * (0.05 + 0.9 * i / 47.0);
      EwaldPlan c = ewald_plan(e, cell, omega, tol);
      const double cost = 60.0 * (double)c.n_img + 0.4 * (double)c.n_g_est;
      if (cost < best) best = cost, pl = c;
    }
  }
  // bounded work: the image box each thread walks and the G list
  const int64_t box = (int64_t)(2 * pl.nx + 1) * (2 * pl.ny + 1) * (2 * pl.nz + 1);
  GW_CHECK_ARG(box <= 1000000, "real-space image box too large (give a larger eta)");
  GW_CHECK_ARG(pl.n_g_est <= 20000000, "reciprocal sum too large (give a smaller eta)");
  // half-space G list: (i, j, k) > 0 lexicographically, |G| <= g_cut
  const double b[3] = {2.0 * kPi / cell[0], 2.0 * kPi / cell[1], 2.0 * kPi / cell[2]};
  const int m[3] = {(int)std::ceil(pl.g_cut / b[0]), (int)std::ceil(pl.g_cut / b[1]),
                    (int)std::ceil(pl.g_cut / b[2])};
  std::vector<double> gw4;
  const double gc2 = pl.g_cut * pl.g_cut;
  for (int i = 0; i <= m[0]; ++i)
    for (int j = (i == 0 ? 0 : -m[1]); j <= m[1]; ++j)
      for (int k = (i == 0 && j == 0 ? 1 : -m[2]); k <= m[2]; ++k) {
        const double gx = i * b[0], gy = j * b[1], gz = k * b[2];
        const double g2 = gx * gx + gy * gy + gz * gz;
        if (g2 > gc2) continue;
        const double w = 2.0 * 4.0 * kPi / omega * std::exp(-g2 / (4.0 * pl.eta * pl.eta)) / g2;
        gw4.insert(gw4.end(), {gx, gy, gz, std::sqrt(w)});
      }
  const int n_g = (int)(gw4.size() / 4);
  // lattice images that can lie within r_cut of a minimum-image displacement
  // (|d_i| <= l_i / 2): distance from the image to that box at most r_cut
  std::vector<double> img;
  const double l[3] = {cell[0], cell[1], cell[2]};
  for (int i = -pl.nx; i <= pl.nx; ++i)
    for (int j = -pl.ny; j <= pl.ny; ++j)
      for (int k = -pl.nz; k <= pl.nz; ++k) {
        const int n[3] = {i, j, k};
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          const double e = std::max(0.0, std::abs(n[a]) * l[a] - 0.5 * l[a]);
          d2 += e * e;
        }
        if (d2 <= pl.r_cut * pl.r_cut * (1.0 + 1e-12))
          img.insert(img.end(), {i * l[0], j * l[1], k * l[2]});
      }
  const int n_list = (int)(img.size() / 3);
  const int64_t f_elems = (int64_t)n_ri * 2 * std::max(n_g, 1);
  GW_CHECK_ARG(f_elems * 8 <= (int64_t)16 << 30,
               "reciprocal sum too large for the workspace (give a smaller eta)");
  if (info) {
    info->eta = pl.eta;
    info->r_cut = pl.r_cut;
    info->g_cut = pl.g_cut;
    info->n_g = n_g;
    info->n_img = n_list;
  }

  rocblas_handle h;
  gw_status rc = get_handle(st, &h);
  if (rc != GW_OK) return rc;
  Scratch sc(st);
  std::vector<double> cen(centres, centres + 3 * (size_t)n_ri), alp(alpha, alpha + n_ri);
  double *cen_d, *alp_d, *img_d, *gw_d = nullptr, *F = nullptr;
  if ((rc = sc.upload(&cen_d, cen)) != GW_OK) return rc;
  if ((rc = sc.upload(&alp_d, alp)) != GW_OK) return rc;
  if ((rc = sc.upload(&img_d, img)) != GW_OK) return rc;
  const int64_t n2 = (int64_t)n_ri * n_ri;
  if (n_g > 0) {
    if ((rc = sc.upload(&gw_d, gw4)) != GW_OK) return rc;
    if ((rc = sc.alloc(&F, f_elems)) != GW_OK) return rc;
    const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)n_ri * n_g + 255) / 256, 65536);
    hipLaunchKernelGGL(ewald_phase_kernel, dim3(blocks), dim3(256), 0, st, cen_d, gw_d, n_ri, n_g, F);
    GW_HIP(hipGetLastError());
    // row-major F [n_ri][2 n_g] is column-major [2 n_g][n_ri]: V = F^T F
    const double one = 1.0, zero = 0.0;
    GW_BLAS(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n_ri, n_ri,
                          2 * n_g, &one, F, 2 * n_g, F, 2 * n_g, &zero, V, n_ri));
  } else {
    GW_HIP(hipMemsetAsync(V, 0, sizeof(double) * n2, st));
  }
  // one block row per p; blocks entirely left of the diagonal exit at once
  hipLaunchKernelGGL(ewald_real_kernel, dim3((n_ri + 255) / 256, n_ri), dim3(256), 0, st, cen_d,
                     alp_d, n_ri, cell[0], cell[1], cell[2], img_d, n_list, pl.eta, pl.r_cut,
                     1.0 / omega, V);
  GW_HIP(hipGetLastError());
  GW_HIP(hipStreamSynchronize(st));
  return GW_OK;
}
