// Diagonal self-energy pieces (Eqs. 10-11) on FP64 MFMA.
//   B^n_{mu P} = sum_nu C_{n nu} (nu mu P)                (half transform, once)
//   Z^n_{P nu} = sum_Q W_PQ B^n_{nu Q}                     inner sum of Eq. 10
//   sig_occ_n  = sum_{mu nu} D^occ_{mu nu} sum_P B^n_{mu P} Z^n_{P nu}
//   sig_vir_n  = the same with D^vir (both dots in one pass)
//   sig_x_n    = - the same with W := V, D := D^occ(0)     (Eq. 11)
// B^n is block sparse: block (mu atom s, RI atom c) exists when a brick
// (f, s, c) is kept.  It is stored panel-dense over AO column panels (PGa
// atoms): panel q holds rows k = (RI atom in U_q, P) and columns (s, mu),
// U_q = RI atoms coupled to the panel.  The same panels feed both the W
// product (K = Q) and the final contraction (K = P).
#include <chrono>
#include <cmath>
#include <type_traits>

#include "gw_internal.hpp"
#include "tile_gemm.hpp"

namespace gw {
namespace {

constexpr int H_WN = 2, H_NBW = 6;  // half transform: rows n_gw (32*WM), cols 192
constexpr int Z_WM = 4, Z_WN = 2, Z_NBW = 5;   // W product / dot: 128 x 160 tiles, 8 waves
constexpr int Z_COLS = 16 * Z_NBW * Z_WN;

constexpr int kSegTab = 2048;     // max bricks per group
constexpr int kPanTab = 8192;     // max RI atoms per AO column panel (|U_q|: one table entry each)

struct HalfProblem {
  struct Tile : TileBase {
    int g, row0, col0, seg0, nseg, q, al, slot;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kSegTab, kTabB = kSegTab;
  const double* cg;         // [N][RS], RS = n_gw
  const double* t3c;
  double* fp;
  const int32_t* goff;
  const int32_t* seg_atom;
  const int64_t* seg_brick;
  const int32_t* gs;
  const int32_t* gslot;
  const int64_t* poff;
  int n_rt, n_ct, rows_pt, cols_pt;
  int RS, NA, NR, PGa, PCa;
  int64_t bs, FPS;
  FastDiv fdNA, fdNR;

  __device__ bool tile(int bx, int, int, Tile& t) const {
    const int per = n_rt * n_ct;
    t.g = bx / per;
    const int rem = bx % per;
    t.row0 = (rem % n_rt) * rows_pt;
    t.col0 = (rem / n_rt) * cols_pt;
    t.seg0 = goff[t.g];
    t.nseg = goff[t.g + 1] - t.seg0;
    t.K = NA * t.nseg;
    const int sa = gs[t.g];
    t.q = sa / PGa;
    t.al = sa % PGa;
    t.slot = gslot[t.g];
    t.rows = min(rows_pt, RS - t.row0);
    t.cols = min(cols_pt, NA * NR - t.col0);
    return t.rows > 0 && t.cols > 0;
  }
  __device__ void fill(const Tile& t, int* ta, int* tb, int tid, int nt) const {
    for (int i = tid; i < t.nseg; i += nt) {
      ta[i] = seg_atom[t.seg0 + i];
      tb[i] = (int)seg_brick[t.seg0 + i];
    }
  }
  __device__ const double* abase(const Tile& t) const { return cg + t.row0; }
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int64_t akoff(const Tile&, int k, const int* ta) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)(ta[sg] * NA + i) * RS;
  }
  __device__ const double* bbase(const Tile& t) const { return t3c + t.col0; }
  __device__ int64_t bkoff(const Tile&, int k, const int* tb) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)tb[sg] * bs + (int64_t)i * NA * NR;
  }
  __device__ double ascale(const Tile&, int) const { return 1.0; }
  // Fp[n][panel q][(slot, P)][(al, mu)]: row n, column (mu, P)
  __device__ double* obase(const Tile& t) const { return fp + poff[t.q] + t.al * NA; }
  __device__ int64_t rowoff(const Tile& t, int r) const { return (int64_t)(t.row0 + r) * FPS; }
  __device__ int64_t coloff(const Tile& t, int c) const {
    const int col = t.col0 + c, mul = (int)fdNR.div((uint32_t)col), P = col - mul * NR;
    return (int64_t)(t.slot * NR + P) * PCa + mul;
  }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

// Z[n][P][nu] = sum_{k in panel q} W[Q(k)][P] * Fp[n][q][k][nu - q*PCa]
// (operands and Z in T: double, or float in the FP32 form)
template <class T>
struct ZProblem {
  using In = T;
  using Out = T;
  struct Tile : TileBase {
    int row0, q, n, km0;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kPanTab, kTabB = 0;
  const T* w;               // [NRI][NRI] symmetric
  const T* fp;
  T* z;                     // [n_gw][NRI][N]
  const int32_t* kmap;
  const int32_t* km_off;
  const int32_t* ulen;
  const int64_t* poff;
  int n_rt, rows_pt, NRI, N, NR, PCa;
  int64_t FPS;
  FastDiv fdNR;

  __device__ bool tile(int bx, int, int bz, Tile& t) const {
    t.row0 = (bx % n_rt) * rows_pt;
    t.q = bx / n_rt;
    t.n = bz;
    t.rows = min(rows_pt, NRI - t.row0);
    t.cols = min(PCa, N - t.q * PCa);
    t.K = NR * ulen[t.q];
    t.km0 = km_off[t.q];
    return t.rows > 0 && t.cols > 0 && t.K > 0;
  }
  // one table entry per union RI atom j: its first function (NR each)
  __device__ void fill(const Tile& t, int* ta, int*, int tid, int nt) const {
    const int nu = t.K / NR;
    for (int j = tid; j < nu; j += nt) ta[j] = kmap[t.km0 + j * NR];
  }
  __device__ const T* abase(const Tile& t) const { return w + t.row0; }
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int64_t akoff(const Tile&, int k, const int* ta) const {
    const int j = (int)fdNR.div((uint32_t)k);
    return (int64_t)(ta[j] + k - j * NR) * NRI;
  }
  __device__ const T* bbase(const Tile& t) const { return fp + (int64_t)t.n * FPS + poff[t.q]; }
  __device__ int64_t bkoff(const Tile&, int k, const int*) const { return (int64_t)k * PCa; }
  __device__ T ascale(const Tile&, int) const { return T(1); }
  __device__ T* obase(const Tile& t) const {
    return z + ((int64_t)t.n * NRI + t.row0) * N + (int64_t)t.q * PCa;
  }
  __device__ int64_t rowoff(const Tile&, int r) const { return (int64_t)r * N; }
  __device__ int64_t coloff(const Tile&, int c) const { return c; }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

// sum_{nu mu} D[nu][mu] * sum_{k in panel q} Z[n][P(k)][nu] Fp[n][q][k][mu - q*PCa]
// (Z, Fp in T; the tile products meet D and are summed in FP64)
template <class T>
struct DotProblem {
  using In = T;
  struct Tile : TileBase {
    int row0, q, n, km0, tile_id;
  };
  static constexpr bool kAScale = false, kDot = true;
  static constexpr int kTabA = kPanTab, kTabB = 0;
  const T* z;
  const T* fp;
  const double* d0;         // [N][N]
  const double* d1;         // [N][N]
  double* partial;          // [n_gw][n_tiles][2]
  const int32_t* kmap;
  const int32_t* km_off;
  const int32_t* ulen;
  const int64_t* poff;
  int n_rt, n_tiles, rows_pt, NRI, N, NR, PCa;
  int64_t FPS;
  FastDiv fdNR;

  __device__ bool tile(int bx, int, int bz, Tile& t) const {
    t.row0 = (bx % n_rt) * rows_pt;
    t.q = bx / n_rt;
    t.n = bz;
    t.tile_id = bx;
    t.rows = min(rows_pt, N - t.row0);
    t.cols = min(PCa, N - t.q * PCa);
    t.K = NR * ulen[t.q];
    t.km0 = km_off[t.q];
    if (t.rows <= 0 || t.cols <= 0 || t.K <= 0) {
      // an empty tile still reports zero so that every partial is written
      if (threadIdx.x == 0) {
        partial[((int64_t)t.n * n_tiles + t.tile_id) * 2] = 0.0;
        partial[((int64_t)t.n * n_tiles + t.tile_id) * 2 + 1] = 0.0;
      }
      return false;
    }
    return true;
  }
  __device__ const T* abase(const Tile& t) const {
    return z + (int64_t)t.n * NRI * N + t.row0;
  }
  // one table entry per union RI atom j: its first function (NR each)
  __device__ void fill(const Tile& t, int* ta, int*, int tid, int nt) const {
    const int nu = t.K / NR;
    for (int j = tid; j < nu; j += nt) ta[j] = kmap[t.km0 + j * NR];
  }
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int64_t akoff(const Tile&, int k, const int* ta) const {
    const int j = (int)fdNR.div((uint32_t)k);
    return (int64_t)(ta[j] + k - j * NR) * N;
  }
  __device__ const T* bbase(const Tile& t) const { return fp + (int64_t)t.n * FPS + poff[t.q]; }
  __device__ int64_t bkoff(const Tile&, int k, const int*) const { return (int64_t)k * PCa; }
  __device__ T ascale(const Tile&, int) const { return T(1); }
  __device__ double* obase(const Tile&) const { return nullptr; }
  __device__ const double* dbase0(const Tile& t) const { return d0 + (int64_t)t.row0 * N + (int64_t)t.q * PCa; }
  __device__ const double* dbase1(const Tile& t) const { return d1 + (int64_t)t.row0 * N + (int64_t)t.q * PCa; }
  __device__ int64_t rowoff(const Tile&, int r) const { return (int64_t)r * N; }
  __device__ int64_t coloff(const Tile&, int c) const { return c; }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ void dot_out(const Tile& t, double s0, double s1) const {
    partial[((int64_t)t.n * n_tiles + t.tile_id) * 2] = s0;
    partial[((int64_t)t.n * n_tiles + t.tile_id) * 2 + 1] = s1;
  }
};

__global__ void gather_rows_kernel(const double* __restrict__ C, const int32_t* __restrict__ rows,
                                   double* __restrict__ cg, int N, int n_rows) {
  const int64_t total = (int64_t)N * n_rows;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int nu = (int)(e / n_rows), k = (int)(e % n_rows);
    cg[e] = C[(int64_t)rows[k] * N + nu];
  }
}

__global__ void round_f32_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
hipError_t round_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(round_f32_kernel, dim3(blocks), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

template <int WM>
hipError_t launch_half(HalfProblem hp, int n_groups, hipStream_t st) {
  hp.rows_pt = 32 * WM;
  hp.cols_pt = 16 * H_NBW * H_WN;
  hp.n_rt = (hp.RS + hp.rows_pt - 1) / hp.rows_pt;
  hp.n_ct = (hp.NA * hp.NR + hp.cols_pt - 1) / hp.cols_pt;
  return launch_tile_gemm<WM, H_WN, H_NBW, 16>(hp, dim3((unsigned)(n_groups * hp.n_rt * hp.n_ct)), st);
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" gw_status gw_contract_sigma_prec(const gw_system* s, int32_t n_gw, const int32_t* states,
                                            const double* C, const double* d_occ, const double* d_vir,
                                            const double* d_occ0, const double* wc, const double* V,
                                            int32_t n_tau, double filter_eps, int32_t prec,
                                            double* sig_occ, double* sig_vir, double* sig_x,
                                            gw_sigma_stats* stats, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(prec == GW_FP64 || prec == GW_FP32, "the Sigma contraction runs in FP64 or FP32");
  const bool f32 = prec == GW_FP32;
  const auto t_start = std::chrono::steady_clock::now();
  gw_status rc = check_system(s);
  if (rc != GW_OK) return rc;
  const int na = s->n_atoms, NA = s->ao_per_atom, NR = s->ri_per_atom;
  const int N = na * NA, NRI = na * NR;
  GW_CHECK_ARG(n_gw >= 1 && n_gw <= 128, "n_gw must be in [1, 128]");
  GW_CHECK_ARG(states != nullptr, "states is null");
  const int64_t n_mo = sys_n_ao(s);
  for (int i = 0; i < n_gw; ++i) GW_CHECK_ARG(states[i] >= 0 && states[i] < n_mo, "state index out of range");
  // d_occ0, V and sig_x all NULL: the exchange term is skipped (it does not
  // depend on tau; callers that contract one tau point at a time take it once)
  const bool with_x = d_occ0 || V || sig_x;
  GW_CHECK_ARG(!with_x || (d_occ0 && V && sig_x),
               "d_occ0, V and sig_x must be given together (or all be null)");
  GW_CHECK_ARG(C && d_occ && d_vir && wc, "null device pointer");
  GW_CHECK_ARG(sig_occ && sig_vir, "null output pointer");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
  GW_CHECK_ARG(std::isfinite(filter_eps) && filter_eps >= 0.0, "filter_eps must be finite and >= 0");
  GW_CHECK_ARG(NA <= Z_COLS, "ao_per_atom must be <= 160");
  if (s->ao_off || s->ri_off) {
    // per-atom sizes: the padded system (missing functions as zero functions)
    Scratch sp(st);
    PadMaps pm;
    if ((rc = pad_maps(s, sp, pm)) != GW_OK) return rc;
    double *pC, *po, *pv, *pw, *pd0 = nullptr, *pV = nullptr;
    if ((rc = sp.alloc(&pC, (size_t)pm.n_ao * pm.N)) != GW_OK) return rc;
    if ((rc = sp.alloc(&po, (size_t)n_tau * pm.N * pm.N)) != GW_OK) return rc;
    if ((rc = sp.alloc(&pv, (size_t)n_tau * pm.N * pm.N)) != GW_OK) return rc;
    if ((rc = sp.alloc(&pw, (size_t)n_tau * pm.NRI * pm.NRI)) != GW_OK) return rc;
    GW_HIP(scatter_cols(C, pm.n_ao, pm.n_ao, pC, pm.N, pm.ao, st));
    GW_HIP(scatter_square(d_occ, pm.n_ao, po, pm.N, pm.ao, n_tau, st));
    GW_HIP(scatter_square(d_vir, pm.n_ao, pv, pm.N, pm.ao, n_tau, st));
    GW_HIP(scatter_square(wc, pm.n_ri, pw, pm.NRI, pm.ri, n_tau, st));
    if (with_x) {
      if ((rc = sp.alloc(&pd0, (size_t)pm.N * pm.N)) != GW_OK) return rc;
      if ((rc = sp.alloc(&pV, (size_t)pm.NRI * pm.NRI)) != GW_OK) return rc;
      GW_HIP(scatter_square(d_occ0, pm.n_ao, pd0, pm.N, pm.ao, 1, st));
      GW_HIP(scatter_square(V, pm.n_ri, pV, pm.NRI, pm.ri, 1, st));
    }
    const gw_system ps = padded_view(s);
    return gw_contract_sigma_prec(&ps, n_gw, states, pC, po, pv, pd0, pw, pV, n_tau, filter_eps,
                                  prec, sig_occ, sig_vir, sig_x, stats, st);
  }
  if (stats) *stats = gw_sigma_stats{};

  Scratch sc(st);
  BrickGroups G;
  if ((rc = build_groups(s, filter_eps, st, sc, G)) != GW_OK) return rc;
  const int n_groups = G.n_groups();
  const int64_t bs = (int64_t)NA * NA * NR;

  // AO column panels (mu atoms); K atoms = RI atoms coupled through a kept brick
  const int PGa = std::max(1, (Z_COLS) / NA), PCa = PGa * NA;
  const Panels pan = build_panels(na, PGa, PCa, G.gs, G.gc, NR, 1);
  const int n_pan = pan.n_pan;
  const int64_t FPS = pan.off[n_pan];
  for (int g = 0; g < n_groups; ++g)
    GW_CHECK_ARG(G.goff[g + 1] - G.goff[g] <= kSegTab, "too many bricks in one (atom, RI atom) group");
  for (int q = 0; q < n_pan; ++q)
    GW_CHECK_ARG(pan.ulen[q] <= kPanTab, "too many RI atoms coupled to one AO column panel");

  double *dof, *dvf, *d0f, *cg, *fp, *z = nullptr, *partial;
  float *fp32 = nullptr, *z32 = nullptr, *w32 = nullptr;   // FP32 form
  int32_t* d_states;
  const size_t dsz = (size_t)n_tau * N * N;
  if ((rc = sc.alloc(&dof, dsz)) != GW_OK) return rc;
  if ((rc = sc.alloc(&dvf, dsz)) != GW_OK) return rc;
  if ((rc = sc.alloc(&d0f, (size_t)N * N)) != GW_OK) return rc;
  if ((rc = sc.alloc(&cg, (size_t)N * n_gw)) != GW_OK) return rc;
  if ((rc = sc.alloc(&fp, (size_t)n_gw * std::max<int64_t>(FPS, 1))) != GW_OK) return rc;
  if (f32) {
    if ((rc = sc.alloc(&fp32, (size_t)n_gw * std::max<int64_t>(FPS, 1))) != GW_OK) return rc;
    if ((rc = sc.alloc(&z32, (size_t)n_gw * NRI * N)) != GW_OK) return rc;
    if ((rc = sc.alloc(&w32, (size_t)NRI * NRI)) != GW_OK) return rc;
  } else {
    if ((rc = sc.alloc(&z, (size_t)n_gw * NRI * N)) != GW_OK) return rc;
  }
  const int z_rt = (NRI + 32 * Z_WM - 1) / (32 * Z_WM);
  const int y_rt = (N + 32 * Z_WM - 1) / (32 * Z_WM);
  const int n_tiles = y_rt * n_pan;
  const int n_slots = n_tau + (with_x ? 1 : 0);
  if ((rc = sc.alloc(&partial, (size_t)n_slots * n_gw * n_tiles * 2)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_states, std::vector<int32_t>(states, states + n_gw))) != GW_OK) return rc;
  int32_t *d_goff, *d_seg_atom, *d_gs, *d_gslot, *d_ulen, *d_kmap, *d_km_off;
  int64_t *d_seg_brick, *d_poff;
  if ((rc = sc.upload(&d_goff, G.goff)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_seg_atom, G.seg_atom)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_seg_brick, G.seg_brick)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_gs, G.gs)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_gslot, pan.gslot)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_ulen, pan.ulen)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_kmap, pan.kmap)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_km_off, pan.km_off)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_poff, pan.off)) != GW_OK) return rc;

  GW_HIP(filter_square_blocks(d_occ, dof, n_tau, na, NA, filter_eps, nullptr, st));
  GW_HIP(filter_square_blocks(d_vir, dvf, n_tau, na, NA, filter_eps, nullptr, st));
  if (with_x) GW_HIP(filter_square_blocks(d_occ0, d0f, 1, na, NA, filter_eps, nullptr, st));
  GW_HIP(hipMemsetAsync(fp, 0, sizeof(double) * (size_t)n_gw * std::max<int64_t>(FPS, 1), st));
  // panels without coupled RI atoms never write their Z columns; those stay 0
  if (f32) GW_HIP(hipMemsetAsync(z32, 0, sizeof(float) * (size_t)n_gw * NRI * N, st));
  else GW_HIP(hipMemsetAsync(z, 0, sizeof(double) * (size_t)n_gw * NRI * N, st));
  {
    const int64_t total = (int64_t)N * n_gw;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks), dim3(256), 0, st, C, d_states, cg, N, n_gw);
    GW_HIP(hipGetLastError());
  }

  // half transform B^n (all states at once)
  if (n_groups > 0) {
    HalfProblem hp{};
    hp.cg = cg; hp.t3c = s->t3c; hp.fp = fp; hp.goff = d_goff; hp.seg_atom = d_seg_atom;
    hp.seg_brick = d_seg_brick; hp.gs = d_gs; hp.gslot = d_gslot; hp.poff = d_poff;
    hp.RS = n_gw; hp.NA = NA; hp.NR = NR; hp.PGa = PGa; hp.PCa = PCa; hp.bs = bs; hp.FPS = FPS;
    hp.fdNA.set((uint32_t)NA);
    hp.fdNR.set((uint32_t)NR);
    hipError_t e = n_gw <= 64 ? launch_half<2>(hp, n_groups, st) : launch_half<4>(hp, n_groups, st);
    GW_HIP(e);
  }

  // per slot (tau_j, then the exchange slot with W := V, D := D^occ(0)): Z = W B^n
  // and the dots with D^occ / D^vir, in FP64 or, in the FP32 form, with W,
  // B^n and Z rounded to FP32 (FP32 products and tile sums, FP64 dot sums)
  auto slots = [&](auto tag, auto* fpx, auto* zx, auto* wx) -> gw_status {
    using T = decltype(tag);
    ZProblem<T> zp{};
    zp.fp = fpx; zp.z = zx; zp.kmap = d_kmap; zp.km_off = d_km_off; zp.ulen = d_ulen; zp.poff = d_poff;
    zp.n_rt = z_rt; zp.rows_pt = 32 * Z_WM; zp.NRI = NRI; zp.N = N; zp.NR = NR; zp.PCa = PCa;
    zp.FPS = FPS;
    zp.fdNR.set((uint32_t)NR);
    DotProblem<T> dp{};
    dp.z = zx; dp.fp = fpx; dp.kmap = d_kmap; dp.km_off = d_km_off; dp.ulen = d_ulen; dp.poff = d_poff;
    dp.n_rt = y_rt; dp.n_tiles = n_tiles; dp.rows_pt = 32 * Z_WM; dp.NRI = NRI; dp.N = N; dp.NR = NR;
    dp.PCa = PCa; dp.FPS = FPS;
    dp.fdNR.set((uint32_t)NR);
    for (int j = 0; j < n_slots; ++j) {
      const bool xslot = (j == n_tau);
      const double* w = xslot ? V : wc + (int64_t)j * NRI * NRI;
      if constexpr (std::is_same<T, float>::value) {
        GW_HIP(round_f32(w, wx, (int64_t)NRI * NRI, st));
        zp.w = wx;
      } else {
        zp.w = w;
      }
      GW_HIP((launch_tile_gemm<Z_WM, Z_WN, Z_NBW, 16>(zp, dim3((unsigned)(z_rt * n_pan), 1, n_gw), st)));
      dp.d0 = xslot ? d0f : dof + (int64_t)j * N * N;
      dp.d1 = xslot ? d0f : dvf + (int64_t)j * N * N;
      dp.partial = partial + (size_t)j * n_gw * n_tiles * 2;
      GW_HIP((launch_tile_gemm<Z_WM, Z_WN, Z_NBW, 16>(dp, dim3((unsigned)n_tiles, 1, n_gw), st)));
    }
    return GW_OK;
  };
  if (f32) {
    GW_HIP(round_f32(fp, fp32, (int64_t)n_gw * std::max<int64_t>(FPS, 1), st));
    if ((rc = slots(0.0f, fp32, z32, w32)) != GW_OK) return rc;
  } else {
    if ((rc = slots(0.0, fp, z, (double*)nullptr)) != GW_OK) return rc;
  }

  std::vector<double> hp((size_t)n_slots * n_gw * n_tiles * 2);
  GW_HIP(hipMemcpyAsync(hp.data(), partial, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
  GW_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < n_slots; ++j)
    for (int n = 0; n < n_gw; ++n) {
      double s0 = 0.0, s1 = 0.0;
      const double* p = hp.data() + ((size_t)j * n_gw + n) * n_tiles * 2;
      for (int t = 0; t < n_tiles; ++t) {
        s0 += p[2 * t];
        s1 += p[2 * t + 1];
      }
      if (j == n_tau) {
        sig_x[n] = -s0;
      } else {
        sig_occ[(size_t)n * n_tau + j] = s0;
        sig_vir[(size_t)n * n_tau + j] = s1;
      }
    }
  if (stats) {
    const double nnzb = (double)n_groups * NA * NR;
    const double half = 2.0 * n_gw * NA * (double)G.n_kept * bs;
    const double per_slot = n_gw * (2.0 * NRI * nnzb + 2.0 * N * nnzb + 4.0 * (double)N * N);
    stats->flops = half + per_slot * n_slots;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return GW_OK;
}

extern "C" gw_status gw_contract_sigma(const gw_system* s, int32_t n_gw, const int32_t* states,
                                       const double* C, const double* d_occ, const double* d_vir,
                                       const double* d_occ0, const double* wc, const double* V,
                                       int32_t n_tau, double filter_eps, double* sig_occ,
                                       double* sig_vir, double* sig_x, gw_sigma_stats* stats,
                                       hipStream_t st) {
  return gw_contract_sigma_prec(s, n_gw, states, C, d_occ, d_vir, d_occ0, wc, V, n_tau, filter_eps,
                                GW_FP64, sig_occ, sig_vir, sig_x, stats, st);
}
