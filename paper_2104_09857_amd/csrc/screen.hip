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

#include <cmath>
#include <mutex>

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
  GW_CHECK_ARG(s != nullptr && s->n_atoms > 0 && s->ri_per_atom > 0, "bad system");
  const int64_t n64 = (int64_t)s->n_atoms * s->ri_per_atom;
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
