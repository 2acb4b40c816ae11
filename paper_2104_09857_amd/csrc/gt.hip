// Imaginary-time density matrices (Eq. 2) on FP64 MFMA:
//   D^occ(tau_j)_{mu nu} = sum_{i < n_occ} C_{i mu} exp(+(eps_i - mu_F) tau_j) C_{i nu}
//   D^vir(tau_j)_{mu nu} = sum_{a >= n_occ} C_{a mu} exp(-(eps_a - mu_F) tau_j) C_{a nu}
// One launch for all tau and both branches; the weight multiplies the A
// operand as it is staged.
#include <cmath>
#include <mutex>

#include "gw_internal.hpp"
#include "tile_gemm.hpp"

namespace gw {
namespace {

constexpr int G_WM = 4, G_WN = 2, G_NBW = 4;   // 128 x 128 tiles, 8 waves
constexpr int G_COLS = 16 * G_NBW * G_WN;

struct GtProblem {
  struct Tile : TileBase {
    int row0, col0, tau, branch;
  };
  static constexpr bool kAScale = true, kDot = false;
  static constexpr int kTabA = 0, kTabB = 0;
  const double* C;
  const double* w;          // [2][n_tau][n_ao] weights (zeros beyond the branch's K)
  double* out[2];
  int N, n_occ, n_tau, n_rt;

  __device__ bool tile(int bx, int by, int bz, Tile& t) const {
    t.row0 = (bx % n_rt) * 32 * G_WM;
    t.col0 = (bx / n_rt) * G_COLS;
    t.tau = by;
    t.branch = bz;
    if (out[bz] == nullptr) return false;
    t.K = bz == 0 ? n_occ : N - n_occ;
    t.rows = min(32 * G_WM, N - t.row0);
    t.cols = min(G_COLS, N - t.col0);
    return t.rows > 0 && t.cols > 0;
  }
  __device__ const double* kbase(const Tile& t) const {
    return C + (t.branch == 0 ? 0 : (int64_t)n_occ * N);
  }
  __device__ const double* abase(const Tile& t) const { return kbase(t) + t.row0; }
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ void fill(const Tile&, int*, int*, int, int) const {}
  __device__ int64_t akoff(const Tile&, int k, const int*) const { return (int64_t)k * N; }
  __device__ double ascale(const Tile& t, int k) const {
    return w[((int64_t)t.branch * n_tau + t.tau) * N + k];
  }
  __device__ const double* bbase(const Tile& t) const { return kbase(t) + t.col0; }
  __device__ int64_t bkoff(const Tile&, int k, const int*) const { return (int64_t)k * N; }
  __device__ double* obase(const Tile& t) const {
    return out[t.branch] + (int64_t)t.tau * N * N + (int64_t)t.row0 * N + t.col0;
  }
  __device__ int64_t rowoff(const Tile&, int r) const { return (int64_t)r * N; }
  __device__ int64_t coloff(const Tile&, int c) const { return c; }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

// Staging array of gw_build_gt_noalloc: weights of up to kGtStage / 2
// (tau, MO) pairs per branch, 8 MiB on every device the library runs on.
constexpr int64_t kGtStage = 1 << 20;
__device__ __align__(256) double scratch[kGtStage];

std::mutex g_stage_mu;
double* g_stage_ptr[64] = {};

// device address of `scratch` on the current device (looked up once per device)
gw_status gt_stage_ptr(double** out) {
  int dev = 0;
  GW_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return GW_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_stage_mu);
  if (!g_stage_ptr[dev]) {
    void* ptr = nullptr;
    GW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_stage_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_stage_ptr[dev];
  return GW_OK;
}

gw_status check_gt_args(const gw_system* s, const double* C, const double* eps, double mu_f,
                        int32_t n_tau, const double* tau, const double* d_occ, const double* d_vir) {
  gw_status rc = check_system_sizes(s);
  if (rc != GW_OK) return rc;
  const int N = (int)sys_n_ao(s);     // D is dense over the AO functions
  GW_CHECK_ARG(C && eps && tau, "C, eps and tau must be non-null");
  GW_CHECK_ARG(d_occ || d_vir, "at least one output is required");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
  GW_CHECK_ARG(std::isfinite(mu_f), "mu_f must be finite");
  for (int i = 0; i < N; ++i) {
    GW_CHECK_ARG(std::isfinite(eps[i]), "eps must be finite");
    GW_CHECK_ARG(i < s->n_occ ? eps[i] < mu_f : eps[i] > mu_f,
                 "occupied levels must lie below mu_f and virtual levels above it");
  }
  for (int j = 0; j < n_tau; ++j) GW_CHECK_ARG(std::isfinite(tau[j]) && tau[j] >= 0.0, "tau must be finite and >= 0");
  return GW_OK;
}

gw_status build_gt_launch(const gw_system* s, const double* C, const double* eps, double mu_f,
                          int32_t n_tau, const double* tau, double* d_occ, double* d_vir,
                          double* d_w, hipStream_t st);

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" gw_status gw_build_gt(const gw_system* s, const double* C, const double* eps,
                                 double mu_f, int32_t n_tau, const double* tau, double* d_occ,
                                 double* d_vir, hipStream_t st) {
  clear_error();
  gw_status rc0 = check_gt_args(s, C, eps, mu_f, n_tau, tau, d_occ, d_vir);
  if (rc0 != GW_OK) return rc0;
  Scratch sc(st);
  double* d_w = nullptr;
  gw_status rc = sc.alloc(&d_w, (size_t)2 * n_tau * sys_n_ao(s));
  if (rc != GW_OK) return rc;
  return build_gt_launch(s, C, eps, mu_f, n_tau, tau, d_occ, d_vir, d_w, st);
}

// The same without any allocation: the weights are staged in the library's
// per-device array (see gw_build_gt_noalloc in include/gw.h).
extern "C" gw_status gw_build_gt_noalloc(const gw_system* s, const double* C, const double* eps,
                                         double mu_f, int32_t n_tau, const double* tau,
                                         double* d_occ, double* d_vir, hipStream_t st) {
  clear_error();
  gw_status rc = check_gt_args(s, C, eps, mu_f, n_tau, tau, d_occ, d_vir);
  if (rc != GW_OK) return rc;
  const int64_t need = 2 * (int64_t)n_tau * sys_n_ao(s);
  if (need > kGtStage) {
    set_error("gw_build_gt_noalloc: 2 * n_tau * n_ao = " + std::to_string(need) +
              " weights exceed the staging array of " + std::to_string(kGtStage) +
              " (use gw_build_gt)");
    return GW_ERR_ARG;
  }
  double* d_w = nullptr;
  if ((rc = gt_stage_ptr(&d_w)) != GW_OK) return rc;
  return build_gt_launch(s, C, eps, mu_f, n_tau, tau, d_occ, d_vir, d_w, st);
}

namespace gw {
namespace {

// weights w[branch][tau][k] into the device buffer d_w (2 n_tau N doubles,
// zeros beyond the branch's K), then one launch for all tau and both branches
gw_status build_gt_launch(const gw_system* s, const double* C, const double* eps, double mu_f,
                          int32_t n_tau, const double* tau, double* d_occ, double* d_vir,
                          double* d_w, hipStream_t st) {
  const int N = (int)sys_n_ao(s);
  std::vector<double> w((size_t)2 * n_tau * N, 0.0);
  for (int j = 0; j < n_tau; ++j) {
    for (int i = 0; i < s->n_occ; ++i) w[(size_t)j * N + i] = std::exp((eps[i] - mu_f) * tau[j]);
    for (int a = s->n_occ; a < N; ++a)
      w[((size_t)n_tau + j) * N + (a - s->n_occ)] = std::exp(-(eps[a] - mu_f) * tau[j]);
  }
  // a copy from pageable host memory has consumed w when it returns
  GW_HIP(hipMemcpyAsync(d_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice, st));

  GtProblem p{};
  p.C = C;
  p.w = d_w;
  p.out[0] = d_occ;
  p.out[1] = d_vir;
  p.N = N;
  p.n_occ = s->n_occ;
  p.n_tau = n_tau;
  p.n_rt = (N + 32 * G_WM - 1) / (32 * G_WM);
  const int n_ct = (N + G_COLS - 1) / (G_COLS);
  GW_HIP((launch_tile_gemm<G_WM, G_WN, G_NBW, 16>(p, dim3((unsigned)(p.n_rt * n_ct), n_tau, 2), st)));
  return GW_OK;
}

}  // namespace
}  // namespace gw
