// Block-sparse polarizability chi_PQ(tau) (Eq. 3) on FP64 MFMA.
//
// Eq. 3 is organised around a pivot AO atom b (sigma runs over b):
//   stage A  M_b[tau][sigma][c][mu][P] = sum_a sum_{l in a} D^occ_{l mu}(tau) (l sigma P)
//            for every RI atom c that has a brick (a, b, c) and every mu
//   stage B  N_b[tau][(a', c')][mu][Q][sigma] = sum_{a2} sum_{nu in a2}
//                 (nu mu Q) D^vir_{nu sigma}(tau)      (brick (a2, a', c'))
//   stage C  chi[tau][c][c'] -= sum_{sigma in b} sum_{mu} M_b[..][mu][P] N_b[..][mu][Q][sigma]
// Both half contractions use the same brick grouping: group (s, c) lists the
// bricks (f, s, c) and the contraction runs over the first index f.  Stage C
// is a GEMM per RI column panel p (PG consecutive RI atoms): its K range is
// (sigma, mu in U_p) with U_p the union of the AO atoms that couple to the
// panel, so N_b is written panel-dense (zeros where an atom does not couple).
// Only blocks with c <= c' are computed; the lower blocks are mirrored at
// the end (chi is symmetric).  The half-contracted tensors never exceed one
// pivot (O(n_tau * N_AO * |S|/N_atoms) doubles).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "gw_internal.hpp"
#include "tile_bf16x3.hpp"
#include "tile_gemm.hpp"

namespace gw {
namespace {

constexpr int A_WM = 4, AB_WN = 2, AB_NBW = 6;    // stage A tile 128 x 192, 8 waves
constexpr int AB_COLS = 16 * AB_NBW * AB_WN;      // stage B tile (32 WM) x 192
constexpr int C_WM = 4, C_WN = 2, C_NBW = 5;      // stage C tile 128 x 160, 8 waves
constexpr int C_COLS = 16 * C_NBW * C_WN;
constexpr int C_KC = 32;                          // K chunk staged per barrier pair

constexpr int kSegTab = 2048;     // max bricks per group (first atoms)
constexpr int kPanTab = 4096;     // max K functions per column panel (NA * |U_p|)

struct StageA {
  struct Tile : TileBase {
    int g, slot, tau, row0, col0, seg0, nseg;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kSegTab, kTabB = kSegTab;
  const double* dof;
  const double* t3c;
  double* mb;
  const int32_t* goff;
  const int32_t* seg_atom;
  const int64_t* seg_brick;
  int g0, n_rt, n_ct, rows_pt, cols_pt;
  int N, NA, NR, nRmax;
  int64_t bs;
  FastDiv fdNA, fdNR;

  __device__ bool tile(int bx, int by, int bz, Tile& t) const {
    const int per = n_rt * n_ct;
    t.slot = bx / per;
    const int rem = bx % per;
    t.row0 = (rem % n_rt) * rows_pt;
    t.col0 = (rem / n_rt) * cols_pt;
    t.g = g0 + t.slot;
    t.tau = by;
    t.seg0 = goff[t.g];
    t.nseg = goff[t.g + 1] - t.seg0;
    t.K = NA * t.nseg;
    t.rows = min(rows_pt, N - t.row0);
    t.cols = min(cols_pt, NA * NR - t.col0);
    return t.rows > 0 && t.cols > 0;
  }
  __device__ void fill(const Tile& t, int* ta, int* tb, int tid, int nt) const {
    for (int i = tid; i < t.nseg; i += nt) {
      ta[i] = seg_atom[t.seg0 + i];
      tb[i] = (int)seg_brick[t.seg0 + i];
    }
  }
  __device__ const double* abase(const Tile& t) const { return dof + (int64_t)t.tau * N * N + t.row0; }
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int64_t akoff(const Tile&, int k, const int* ta) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)(ta[sg] * NA + i) * N;
  }
  __device__ const double* bbase(const Tile& t) const { return t3c + t.col0; }
  __device__ int64_t bkoff(const Tile&, int k, const int* tb) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)tb[sg] * bs + (int64_t)i * NA * NR;
  }
  __device__ double ascale(const Tile&, int) const { return 1.0; }
  // M_b[tau][sigma][slot][mu][P]: row mu, column (sigma, P)
  __device__ double* obase(const Tile& t) const {
    return mb + ((int64_t)t.tau * NA * nRmax + t.slot) * N * NR;
  }
  __device__ int64_t rowoff(const Tile& t, int r) const { return (int64_t)(t.row0 + r) * NR; }
  __device__ int64_t coloff(const Tile& t, int c) const {
    const int col = t.col0 + c, sg = (int)fdNR.div((uint32_t)col), P = col - sg * NR;
    return (int64_t)sg * nRmax * N * NR + P;
  }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

struct StageB {
  struct Tile : TileBase {
    int g, row0, col0, seg0, nseg, p, cl, slot, KU;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kSegTab, kTabB = kSegTab;
  const double* dvg;        // [N][RS]
  const double* t3c;
  double* bp;
  const int32_t* goff;
  const int32_t* seg_atom;
  const int64_t* seg_brick;
  const int32_t* gc;
  const int32_t* gslot;
  const int32_t* ulen;
  const int64_t* bp_off;
  int n_rt, n_ct, rows_pt, cols_pt;
  int RS, NA, NR, PG, PC;
  int64_t bs, BPS;
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
    const int c = gc[t.g];
    t.p = c / PG;
    t.cl = c % PG;
    t.slot = gslot[t.g];
    t.KU = NA * ulen[t.p];
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
  __device__ const double* abase(const Tile& t) const { return dvg + t.row0; }
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
  // N_b panel: [tau][panel][sigma][u = slot*NA + mu][(cl, Q)]: row (tau, sigma), column (mu, Q)
  __device__ double* obase(const Tile& t) const { return bp + bp_off[t.p]; }
  __device__ int64_t rowoff(const Tile& t, int r) const {
    const int row = t.row0 + r, tau = (int)fdNA.div((uint32_t)row), sg = row - tau * NA;
    return (int64_t)tau * BPS + (int64_t)sg * t.KU * PC;
  }
  __device__ int64_t coloff(const Tile& t, int c) const {
    const int col = t.col0 + c, mul = (int)fdNR.div((uint32_t)col), Q = col - mul * NR;
    return (int64_t)(t.slot * NA + mul) * PC + t.cl * NR + Q;
  }
  static constexpr bool kAccum = false;
  static constexpr double kSign = 1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

// true if some upper (c <= c') block of the tile is kept by the screener
__device__ inline bool any_kept(const uint8_t* keep, const int32_t* slot_c, int s0, int s1,
                                int c0, int c1, int tau, int na) {
  const uint8_t* k = keep + (int64_t)tau * na * na;
  for (int sl = s0; sl <= s1; ++sl) {
    const int c = slot_c[sl];
    for (int c2 = c0; c2 <= c1; ++c2)
      if (c <= c2 && k[(int64_t)c * na + c2]) return true;
  }
  return false;
}

struct StageC {
  struct Tile : TileBase {
    int p, tau, row0, KU, km0;
    FastDiv fdKU;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kPanTab, kTabB = 0;
  const double* mb;
  const double* bp;
  double* chi;
  const int32_t* gc;
  const int32_t* kmap;
  const int32_t* km_off;
  const int32_t* ulen;
  const int64_t* bp_off;
  int g0, nR, n_rt, rows_pt;
  int N, NA, NR, NRI, PG, PC, nRmax, n_atoms;
  int64_t BPS;
  FastDiv fdNR;
  const uint8_t* keep;      // screener mask [tau][c][c'] (c <= c'), or null
  int* tiles_skipped;

  __device__ bool tile(int bx, int by, int bz, Tile& t) const {
    t.row0 = (bx % n_rt) * rows_pt;
    t.p = bx / n_rt;
    t.tau = bz;
    t.rows = min(rows_pt, nR * NR - t.row0);
    t.cols = min(PC, NRI - t.p * PC);
    if (t.rows <= 0 || t.cols <= 0) return false;
    const int c_min = gc[g0 + t.row0 / NR];
    const int cp_max = min(t.p * PG + PG - 1, n_atoms - 1);
    if (c_min > cp_max) return false;          // strictly below the block diagonal
    if (keep && !any_kept(keep, gc + g0, t.row0 / NR, (t.row0 + t.rows - 1) / NR, t.p * PG, cp_max,
                          t.tau, n_atoms)) {
      if (threadIdx.x == 0) atomicAdd(tiles_skipped, 1);
      return false;
    }
    t.KU = NA * ulen[t.p];
    t.km0 = km_off[t.p];
    t.K = NA * t.KU;
    t.fdKU.set((uint32_t)t.KU);
    return t.K > 0;
  }
  __device__ void fill(const Tile& t, int* ta, int*, int tid, int nt) const {
    for (int i = tid; i < t.KU; i += nt) ta[i] = kmap[t.km0 + i] * NR;
  }
  __device__ const double* abase(const Tile& t) const {
    return mb + (int64_t)t.tau * NA * nRmax * N * NR;
  }
  __device__ int64_t aroff(const Tile& t, int r) const {
    const int row = t.row0 + r, sl = (int)fdNR.div((uint32_t)row);
    return (int64_t)sl * N * NR + (row - sl * NR);
  }
  __device__ int64_t akoff(const Tile& t, int k, const int* ta) const {
    const int sg = (int)t.fdKU.div((uint32_t)k), u = k - sg * t.KU;
    return (int64_t)sg * nRmax * N * NR + ta[u];
  }
  __device__ const double* bbase(const Tile& t) const {
    return bp + (int64_t)t.tau * BPS + bp_off[t.p];
  }
  __device__ int64_t bkoff(const Tile&, int k, const int*) const { return (int64_t)k * PC; }
  __device__ double ascale(const Tile&, int) const { return 1.0; }
  // chi[tau][P][Q] -= tile, P = (RI atom of the row's slot, P), Q = panel column
  __device__ double* obase(const Tile& t) const { return chi + (int64_t)t.tau * NRI * NRI; }
  __device__ int64_t rowoff(const Tile& t, int r) const {
    const int row = t.row0 + r, sl = (int)fdNR.div((uint32_t)row), P = row - sl * NR;
    return ((int64_t)gc[g0 + sl] * NR + P) * NRI;
  }
  __device__ int64_t coloff(const Tile& t, int c) const { return (int64_t)t.p * PC + c; }
  static constexpr bool kAccum = true;
  static constexpr double kSign = -1.0;
  __device__ const double* dbase0(const Tile&) const { return nullptr; }
  __device__ const double* dbase1(const Tile&) const { return nullptr; }
  __device__ void dot_out(const Tile&, double, double) const {}
};

__global__ void gather_dvir_kernel(const double* __restrict__ dv, double* __restrict__ dvg, int N,
                                   int NA, int n_tau, int b) {
  const int RS = n_tau * NA;
  const int64_t total = (int64_t)N * RS;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int nu = (int)(e / RS), rc = (int)(e % RS);
    const int tau = rc / NA, sg = rc % NA;
    dvg[e] = dv[(int64_t)tau * N * N + (int64_t)nu * N + (int64_t)b * NA + sg];
  }
}

template <int WM>
hipError_t launch_stage_b(StageB sb, int n_groups, hipStream_t st) {
  sb.rows_pt = 32 * WM;
  sb.cols_pt = AB_COLS;
  sb.n_rt = (sb.RS + sb.rows_pt - 1) / sb.rows_pt;
  sb.n_ct = (sb.NA * sb.NR + sb.cols_pt - 1) / sb.cols_pt;
  return launch_tile_gemm<WM, AB_WN, AB_NBW, 16>(sb, dim3((unsigned)(n_groups * sb.n_rt * sb.n_ct)), st);
}

#include "chi_bf16x3.inc"

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" gw_status gw_contract_chi(const gw_system* s, const double* d_occ, const double* d_vir,
                                     int32_t n_tau, const gw_chi_opts* opts, double* chi,
                                     gw_chi_stats* stats, hipStream_t st) {
  clear_error();
  const auto t_start = std::chrono::steady_clock::now();
  gw_status rc = check_system(s);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(d_occ && d_vir && chi, "d_occ, d_vir and chi must be non-null");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
  const double eps_f = opts ? opts->filter_eps : 0.0;
  GW_CHECK_ARG(std::isfinite(eps_f) && eps_f >= 0.0, "filter_eps must be finite and >= 0");
  const int prec = opts ? opts->prec : GW_FP64;
  GW_CHECK_ARG(prec == GW_FP64 || prec == GW_BF16X3, "prec must be GW_FP64 or GW_BF16X3");
  const int na = s->n_atoms, NA = s->ao_per_atom, NR = s->ri_per_atom;
  GW_CHECK_ARG(NR <= C_COLS, "ri_per_atom must be <= 160");
  const int N = na * NA, NRI = na * NR;
  const int64_t bs = (int64_t)NA * NA * NR;
  GW_CHECK_ARG((int64_t)n_tau * NA <= (1 << 20), "n_tau * ao_per_atom too large");

  Scratch sc(st);
  if (stats) *stats = gw_chi_stats{};
  GW_HIP(hipMemsetAsync(chi, 0, sizeof(double) * (size_t)n_tau * NRI * NRI, st));
  if (s->n_trip == 0) return GW_OK;
  // ---- tensor filter and grouping (host)
  BrickGroups G;
  if ((rc = build_groups(s, eps_f, st, sc, G)) != GW_OK) return rc;
  const int n_groups = G.n_groups();
  const auto& gs = G.gs;
  const auto& gcv = G.gc;
  const auto& goff = G.goff;
  const auto& gb_start = G.gb_start;
  int nRmax = 0;
  for (int b = 0; b < na; ++b) nRmax = std::max(nRmax, gb_start[b + 1] - gb_start[b]);

  // ---- column panels of PG RI atoms; U_p = AO atoms coupling to the panel
  const int PG = std::max(1, C_COLS / NR), PC = PG * NR;
  const Panels pan = build_panels(na, PG, PC, gcv, gs, NA, NA);
  const int n_pan = pan.n_pan;
  const int64_t BPS = pan.off[n_pan];
  for (int g = 0; g < n_groups; ++g)
    GW_CHECK_ARG(goff[g + 1] - goff[g] <= kSegTab, "too many bricks in one (atom, RI atom) group");
  for (int p = 0; p < n_pan; ++p)
    GW_CHECK_ARG(NA * pan.ulen[p] <= kPanTab, "too many AO atoms coupled to one RI column panel");

  // ---- scratch
  double *dof = nullptr, *dvf = nullptr, *dvg = nullptr, *mb = nullptr, *bp = nullptr;
  uint8_t* dropped = nullptr;
  const int RS = n_tau * NA;
  const size_t dsz = (size_t)n_tau * N * N;
  if ((rc = sc.alloc(&dof, dsz)) != GW_OK) return rc;
  if ((rc = sc.alloc(&dvf, dsz)) != GW_OK) return rc;
  const bool fp64 = prec == GW_FP64;
  if (fp64) {
    if ((rc = sc.alloc(&dvg, (size_t)N * RS)) != GW_OK) return rc;
    if ((rc = sc.alloc(&mb, (size_t)n_tau * NA * std::max(nRmax, 1) * N * NR)) != GW_OK) return rc;
    if ((rc = sc.alloc(&bp, (size_t)n_tau * BPS)) != GW_OK) return rc;
  }
  const size_t nflag = (size_t)n_tau * na * na;
  if ((rc = sc.alloc(&dropped, 3 * nflag)) != GW_OK) return rc;
  int32_t *d_goff, *d_seg_atom, *d_gc, *d_gslot, *d_ulen, *d_kmap, *d_km_off;
  int64_t *d_seg_brick, *d_bp_off;
  if ((rc = sc.upload(&d_goff, goff)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_seg_atom, G.seg_atom)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_seg_brick, G.seg_brick)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_gc, gcv)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_gslot, pan.gslot)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_ulen, pan.ulen)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_kmap, pan.kmap)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_km_off, pan.km_off)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_bp_off, pan.off)) != GW_OK) return rc;
  if (fp64) GW_HIP(hipMemsetAsync(bp, 0, sizeof(double) * (size_t)n_tau * BPS, st));

  // ---- D filter (copies)
  GW_HIP(filter_square_blocks(d_occ, dof, n_tau, na, NA, eps_f, dropped, st));
  GW_HIP(filter_square_blocks(d_vir, dvf, n_tau, na, NA, eps_f, dropped + nflag, st));

  // ---- learned screener: keep mask of the output blocks
  uint8_t* d_keep = nullptr;
  int* d_tiles_skipped = nullptr;
  std::vector<uint8_t> keep_h;
  const bool screening = opts && opts->screener && eps_f > 0.0;
  if (screening) {
    GW_CHECK_ARG(opts->screen_tau != nullptr, "screen_tau is required with a screener");
    GW_CHECK_ARG(std::isfinite(opts->screen_margin) && opts->screen_margin >= 0.0,
                 "screen_margin must be finite and >= 0");
    const int64_t nb = (int64_t)n_tau * na * na;
    float *feat, *pred;
    if ((rc = sc.alloc(&feat, (size_t)nb * 6)) != GW_OK) return rc;
    if ((rc = sc.alloc(&pred, (size_t)nb)) != GW_OK) return rc;
    if ((rc = sc.alloc(&d_keep, (size_t)nb)) != GW_OK) return rc;
    if ((rc = sc.alloc(&d_tiles_skipped, 1)) != GW_OK) return rc;
    GW_HIP(hipMemsetAsync(d_tiles_skipped, 0, sizeof(int), st));
    if ((rc = gw_chi_block_features(s, d_occ, d_vir, n_tau, opts->screen_tau, eps_f, feat, st)) != GW_OK)
      return rc;
    if ((rc = gw_mlp_forward(opts->screener, nb, feat, pred, 1, st)) != GW_OK) return rc;
    std::vector<float> ph(nb);
    GW_HIP(hipMemcpyAsync(ph.data(), pred, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
    GW_HIP(hipStreamSynchronize(st));
    const float thr = (float)(std::log10(eps_f) - opts->screen_margin);
    keep_h.assign(nb, 0);
    for (int j = 0; j < n_tau; ++j)
      for (int c = 0; c < na; ++c)
        for (int c2 = c; c2 < na; ++c2) {
          const int64_t e = ((int64_t)j * na + c) * na + c2;
          keep_h[e] = (ph[e] >= thr) || !std::isfinite(ph[e]) ? 1 : 0;
        }
    GW_HIP(hipMemcpyAsync(d_keep, keep_h.data(), nb, hipMemcpyHostToDevice, st));
  }

  // ---- pivot loop
  StageA sa{};
  sa.dof = dof; sa.t3c = s->t3c; sa.mb = mb; sa.goff = d_goff; sa.seg_atom = d_seg_atom;
  sa.seg_brick = d_seg_brick; sa.rows_pt = 32 * A_WM; sa.cols_pt = AB_COLS;
  sa.n_rt = (N + sa.rows_pt - 1) / sa.rows_pt;
  sa.n_ct = (NA * NR + sa.cols_pt - 1) / sa.cols_pt;
  sa.N = N; sa.NA = NA; sa.NR = NR; sa.nRmax = std::max(nRmax, 1); sa.bs = bs;
  sa.fdNA.set((uint32_t)NA);
  sa.fdNR.set((uint32_t)NR);

  StageB sb{};
  sb.dvg = dvg; sb.t3c = s->t3c; sb.bp = bp; sb.goff = d_goff; sb.seg_atom = d_seg_atom;
  sb.seg_brick = d_seg_brick; sb.gc = d_gc; sb.gslot = d_gslot; sb.ulen = d_ulen;
  sb.bp_off = d_bp_off; sb.RS = RS; sb.NA = NA; sb.NR = NR; sb.PG = PG; sb.PC = PC; sb.bs = bs;
  sb.BPS = BPS;
  sb.fdNA.set((uint32_t)NA);
  sb.fdNR.set((uint32_t)NR);

  StageC scx{};
  scx.mb = mb; scx.bp = bp; scx.chi = chi; scx.gc = d_gc; scx.kmap = d_kmap; scx.km_off = d_km_off;
  scx.ulen = d_ulen; scx.bp_off = d_bp_off; scx.rows_pt = 32 * C_WM; scx.N = N; scx.NA = NA;
  scx.NR = NR; scx.NRI = NRI; scx.PG = PG; scx.PC = PC; scx.nRmax = std::max(nRmax, 1);
  scx.n_atoms = na; scx.BPS = BPS;
  scx.fdNR.set((uint32_t)NR);
  scx.keep = d_keep; scx.tiles_skipped = d_tiles_skipped;

  double flops_ab = 0.0, flops_c = 0.0, flops_a = 0.0, flops_b = 0.0;
  const bool timing = opts && opts->timing;
  std::vector<hipEvent_t> evs;
  auto mark = [&](void) -> hipError_t {
    if (!timing) return hipSuccess;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    evs.push_back(e);
    return hipEventRecord(e, st);
  };
  int64_t n_launch[3] = {0, 0, 0};
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() {
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
    }
  } ev_guard{evs};
  int64_t nnz_elems = G.n_kept * bs;
  // |A(c')| per RI atom: number of groups with that c
  std::vector<int32_t> acount(na, 0);
  for (int g = 0; g < n_groups; ++g) acount[gcv[g]]++;
  std::vector<double> asuffix(na + 1, 0.0);   // sum_{c' >= c} |A(c')|
  for (int c = na - 1; c >= 0; --c) asuffix[c] = asuffix[c + 1] + acount[c];

  // ---- split-precision form: operands as bf16 hi/lo pairs, FP32 accumulation
  // within a tile, FP64 accumulation across pivots
  uint16_t *th = nullptr, *tl = nullptr, *doh = nullptr, *dol = nullptr, *dvh = nullptr, *dvl = nullptr;
  uint16_t *mh = nullptr, *ml = nullptr, *nh = nullptr, *nl = nullptr;
  std::vector<int64_t> poffb(n_pan + 1, 0);
  for (int p = 0; p < n_pan; ++p) poffb[p + 1] = poffb[p] + (int64_t)NA * pan.ulen[p] * PC * 16;
  const int64_t BPS16 = poffb[n_pan];
  int64_t* d_poffb = nullptr;
  if (!fp64) {
    const size_t tsz = (size_t)s->n_trip * NR * NA * 16, dsz16 = (size_t)n_tau * N * na * 16;
    const size_t msz = (size_t)n_tau * std::max(nRmax, 1) * N * NR * 16, nsz = (size_t)n_tau * BPS16;
    if ((rc = sc.alloc(&th, tsz)) != GW_OK) return rc;
    if ((rc = sc.alloc(&tl, tsz)) != GW_OK) return rc;
    if ((rc = sc.alloc(&doh, dsz16)) != GW_OK) return rc;
    if ((rc = sc.alloc(&dol, dsz16)) != GW_OK) return rc;
    if ((rc = sc.alloc(&dvh, dsz16)) != GW_OK) return rc;
    if ((rc = sc.alloc(&dvl, dsz16)) != GW_OK) return rc;
    if ((rc = sc.alloc(&mh, msz)) != GW_OK) return rc;
    if ((rc = sc.alloc(&ml, msz)) != GW_OK) return rc;
    if ((rc = sc.alloc(&nh, nsz)) != GW_OK) return rc;
    if ((rc = sc.alloc(&nl, nsz)) != GW_OK) return rc;
    if ((rc = sc.upload(&d_poffb, poffb)) != GW_OK) return rc;
    GW_HIP(hipMemsetAsync(mh, 0, 2 * msz, st));
    GW_HIP(hipMemsetAsync(ml, 0, 2 * msz, st));
    GW_HIP(hipMemsetAsync(nh, 0, 2 * nsz, st));
    GW_HIP(hipMemsetAsync(nl, 0, 2 * nsz, st));
    auto blocks = [](int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20); };
    hipLaunchKernelGGL(split_t_kernel, dim3(blocks((int64_t)tsz)), dim3(256), 0, st, s->t3c, th, tl,
                       s->n_trip, NA, NR);
    GW_HIP(hipGetLastError());
    hipLaunchKernelGGL(split_d_kernel, dim3(blocks((int64_t)dsz16)), dim3(256), 0, st, dof, doh, dol,
                       n_tau, N, na, NA);
    GW_HIP(hipGetLastError());
    hipLaunchKernelGGL(split_d_kernel, dim3(blocks((int64_t)dsz16)), dim3(256), 0, st, dvf, dvh, dvl,
                       n_tau, N, na, NA);
    GW_HIP(hipGetLastError());
  }
  StageABf ba{};
  ba.dh = doh; ba.dl = dol; ba.th = th; ba.tl = tl; ba.mh = mh; ba.ml = ml; ba.goff = d_goff;
  ba.seg_atom = d_seg_atom; ba.seg_brick = d_seg_brick; ba.rows_pt = 16 * 4 * 4;
  ba.cols_pt = 16 * BF_NB_AB * BF_WN; ba.n_rt = (N + ba.rows_pt - 1) / ba.rows_pt;
  ba.n_ct = (NA * NR + ba.cols_pt - 1) / ba.cols_pt; ba.N = N; ba.NA = NA; ba.NR = NR; ba.na = na;
  ba.nRmax = std::max(nRmax, 1); ba.fdNA.set((uint32_t)NA);
  StageBBf bb{};
  bb.dh = dvh; bb.dl = dvl; bb.th = th; bb.tl = tl; bb.nh = nh; bb.nl = nl; bb.goff = d_goff;
  bb.seg_atom = d_seg_atom; bb.seg_brick = d_seg_brick; bb.gc = d_gc; bb.gslot = d_gslot;
  bb.poffb = d_poffb; bb.N = N; bb.NA = NA; bb.NR = NR; bb.na = na; bb.RS = RS; bb.PG = PG;
  bb.PC = PC; bb.BPS16 = BPS16; bb.fdNA.set((uint32_t)NA);
  StageCBf bc{};
  bc.mh = mh; bc.ml = ml; bc.nh = nh; bc.nl = nl; bc.chi = chi; bc.gc = d_gc; bc.kmap = d_kmap;
  bc.km_off = d_km_off; bc.ulen = d_ulen; bc.poffb = d_poffb; bc.rows_pt = 16 * 4 * 4; bc.N = N;
  bc.NA = NA; bc.NR = NR; bc.NRI = NRI; bc.PG = PG; bc.PC = PC; bc.nRmax = std::max(nRmax, 1);
  bc.n_atoms = na; bc.BPS16 = BPS16; bc.fdNR.set((uint32_t)NR);
  bc.keep = d_keep; bc.tiles_skipped = d_tiles_skipped;

  for (int b = 0; b < na; ++b) {
    const int g0 = gb_start[b], nR = gb_start[b + 1] - g0;
    if (nR == 0) continue;
    if (fp64) {
      {
        const int64_t total = (int64_t)N * RS;
        const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
        hipLaunchKernelGGL(gather_dvir_kernel, dim3(blocks), dim3(256), 0, st, dvf, dvg, N, NA,
                           n_tau, b);
        GW_HIP(hipGetLastError());
      }
      sa.g0 = g0;
      GW_HIP(mark());
      GW_HIP((launch_tile_gemm<A_WM, AB_WN, AB_NBW, 16>(sa, dim3((unsigned)(nR * sa.n_rt * sa.n_ct), n_tau), st)));
      GW_HIP(mark());
      hipError_t e;
      if (RS <= 64) e = launch_stage_b<2>(sb, n_groups, st);
      else if (RS <= 96) e = launch_stage_b<3>(sb, n_groups, st);
      else if (RS <= 128) e = launch_stage_b<4>(sb, n_groups, st);
      else if (RS <= 160) e = launch_stage_b<5>(sb, n_groups, st);
      else e = launch_stage_b<4>(sb, n_groups, st);
      GW_HIP(e);
      GW_HIP(mark());
      scx.g0 = g0;
      scx.nR = nR;
      scx.n_rt = (nR * NR + scx.rows_pt - 1) / scx.rows_pt;
      GW_HIP((launch_tile_gemm<C_WM, C_WN, C_NBW, C_KC>(scx, dim3((unsigned)(scx.n_rt * n_pan), 1, n_tau), st)));
      GW_HIP(mark());
    } else {
      ba.g0 = g0;
      GW_HIP(mark());
      GW_HIP((launch_tile_bf16x3<4, BF_WN, 4, BF_NB_AB, BF_KC>(ba, dim3((unsigned)(nR * ba.n_rt * ba.n_ct), n_tau), st)));
      GW_HIP(mark());
      bb.b = b;
      hipError_t e;
      if (RS <= 64) e = launch_stage_b_bf<2>(bb, n_groups, st);
      else if (RS <= 96) e = launch_stage_b_bf<3>(bb, n_groups, st);
      else if (RS <= 128) e = launch_stage_b_bf<4>(bb, n_groups, st);
      else e = launch_stage_b_bf<5>(bb, n_groups, st);
      GW_HIP(e);
      GW_HIP(mark());
      bc.g0 = g0;
      bc.nR = nR;
      bc.n_rt = (nR * NR + bc.rows_pt - 1) / bc.rows_pt;
      GW_HIP((launch_tile_bf16x3<4, BF_WN, 4, BF_NB_C, BF_KC>(bc, dim3((unsigned)(bc.n_rt * n_pan), 1, n_tau), st)));
      GW_HIP(mark());
    }
    n_launch[0]++; n_launch[1]++; n_launch[2]++;

    int64_t nnz_b = 0;
    for (int g = g0; g < g0 + nR; ++g) nnz_b += (int64_t)(goff[g + 1] - goff[g]) * bs;
    flops_a += 2.0 * N * (double)nnz_b;
    flops_b += 2.0 * NA * (double)nnz_elems;
    flops_ab += 2.0 * N * (double)nnz_b + 2.0 * NA * (double)nnz_elems;
    if (!screening) {
      for (int g = g0; g < g0 + nR; ++g)
        flops_c += 2.0 * NR * NR * NA * NA * asuffix[gcv[g]];
    } else {
      // per tau, kept blocks only (averaged into the per-tau figure below)
      for (int g = g0; g < g0 + nR; ++g) {
        const int c = gcv[g];
        for (int j = 0; j < n_tau; ++j)
          for (int c2 = c; c2 < na; ++c2)
            if (keep_h[((int64_t)j * na + c) * na + c2])
              flops_c += 2.0 * NR * NR * NA * NA * acount[c2] / n_tau;
      }
    }
  }

  // ---- symmetric completion and output filter
  GW_HIP(mirror_lower_blocks(chi, n_tau, NRI, NR, st));
  if (screening) GW_HIP(zero_unkept_blocks(chi, n_tau, na, NR, d_keep, st));
  if (eps_f > 0.0)
    GW_HIP(filter_square_blocks(chi, chi, n_tau, na, NR, eps_f, dropped + 2 * nflag, st));

  if (stats) {
    std::vector<uint8_t> fl(3 * nflag);
    GW_HIP(hipMemcpyAsync(fl.data(), dropped, fl.size(), hipMemcpyDeviceToHost, st));
    GW_HIP(hipStreamSynchronize(st));
    int64_t dd = 0, dc = 0;
    for (size_t i = 0; i < 2 * nflag; ++i) dd += fl[i];
    if (eps_f > 0.0)
      for (size_t i = 2 * nflag; i < 3 * nflag; ++i) dc += fl[i];
    stats->n_trip_kept = G.n_kept;
    if (screening) {
      int skipped = 0;
      GW_HIP(hipMemcpy(&skipped, d_tiles_skipped, sizeof(int), hipMemcpyDeviceToHost));
      stats->n_tiles_screened = skipped;
      int64_t nbs = 0;
      for (int j = 0; j < n_tau; ++j)
        for (int c = 0; c < na; ++c)
          for (int c2 = c; c2 < na; ++c2) nbs += keep_h[((int64_t)j * na + c) * na + c2] ? 0 : 1;
      stats->n_blocks_screened = nbs;
    }
    stats->n_dblk_dropped = dd;
    stats->n_chiblk_dropped = dc;
    stats->flops_ab = flops_ab * n_tau;
    stats->flops_c = flops_c * n_tau;
    for (int k = 0; k < 3; ++k) {
      stats->ms_stage[k] = 0.0;
      stats->n_launch[k] = n_launch[k];
    }
    stats->flops_stage[0] = flops_a * n_tau;
    stats->flops_stage[1] = flops_b * n_tau;
    stats->flops_stage[2] = flops_c * n_tau;
    for (size_t i = 0; timing && i + 3 < evs.size(); i += 4) {
      float ms;
      GW_HIP(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      stats->ms_stage[0] += ms;
      GW_HIP(hipEventElapsedTime(&ms, evs[i + 1], evs[i + 2]));
      stats->ms_stage[1] += ms;
      GW_HIP(hipEventElapsedTime(&ms, evs[i + 2], evs[i + 3]));
      stats->ms_stage[2] += ms;
    }
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return GW_OK;
}
