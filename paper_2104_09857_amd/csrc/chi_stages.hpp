// Problem types of the three chi stages (FP64 and split-precision forms)
// for the tile engines.  Included once, by chi.hip.
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
// the end (chi is symmetric).
#pragma once
#include "gw_internal.hpp"
#include "tile_bf16x3.hpp"
#include "tile_bf16x3_dma.hpp"
#include "tile_dma.hpp"

namespace gw {
namespace {

constexpr int A_WM = 4, AB_WN = 2, AB_NBW = 6;    // stage A tile 128 x 192, 8 waves
constexpr int AB_NBN = 2;                         // narrow stage-A/B tiles: 64 columns
constexpr int C_WM = 4, C_WN = 2, C_NBW = 5;      // stage C tile 128 x 160, 8 waves
constexpr int C_COLS = 16 * C_NBW * C_WN;
constexpr int C_KC = 32;                          // K chunk staged per barrier pair

constexpr int kSegTab = 2048;     // max bricks per group (first atoms)
// max union atoms per RI column panel (|U_p|: one table entry per atom); the
// FP64 direct-to-LDS outer contraction with 32-deep K chunks (144 KB of
// operand stages) and this table fit in the 160 KB of LDS
constexpr int kPanTab = 3968;

// screening masks of the half contractions: any AO atom a0 .. a1 needed
__device__ inline bool any_row_needed(const uint8_t* need, int a0, int a1) {
  for (int a = a0; a <= a1; ++a)
    if (need[a]) return true;
  return false;
}

// T: operand type (double: FP64 form, float: FP32 form)
template <class T>
struct StageA {
  using In = T;
  using Out = T;
  struct Tile : TileBase {
    int g, slot, tau, row0, col0, seg0, nseg;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kSegTab, kTabB = kSegTab;
  const T* dof;
  const T* t3c;
  T* mb;
  const int32_t* goff;
  const int32_t* seg_atom;
  const int64_t* seg_brick;
  int g0, n_rt, n_ct, rows_pt, cols_pt;
  int N, NA, NR, nRmax;
  int lda;                  // row stride of the D^occ stack (N, or N padded to 4 in FP32)
  int64_t bs;
  int bs32;                 // brick size (elements) as int for the offset products
  FastDiv fdNA, fdNR;
  // screened calls: needa[c * nat + a] = 0 when the M_b rows of AO atom a for
  // slot atom c feed no kept chi block (the rows are then not computed)
  const uint8_t* needa;
  const int32_t* gc;        // RI atom of each brick group
  int nat;

  __device__ bool tile(int bx, int by, int bz, Tile& t) const {
    const int per = n_rt * n_ct;
    t.slot = bx / per;
    const int rem = bx % per;
    t.row0 = (rem % n_rt) * rows_pt;
    t.col0 = (rem / n_rt) * cols_pt;
    t.g = g0 + t.slot;
    t.tau = by;
    t.rows = min(rows_pt, N - t.row0);
    if (needa && t.rows > 0 &&
        !any_row_needed(needa + (int64_t)gc[t.g] * nat, t.row0 / NA, (t.row0 + t.rows - 1) / NA))
      return false;
    t.seg0 = goff[t.g];
    t.nseg = goff[t.g + 1] - t.seg0;
    t.K = NA * t.nseg;
    t.cols = min(cols_pt, NA * NR - t.col0);
    return t.rows > 0 && t.cols > 0;
  }
  __device__ void fill(const Tile& t, int* ta, int* tb, int tid, int nt) const {
    for (int i = tid; i < t.nseg; i += nt) {
      ta[i] = seg_atom[t.seg0 + i];
      tb[i] = (int)seg_brick[t.seg0 + i];
    }
  }
  __device__ const T* abase(const Tile& t) const { return dof + (int64_t)t.tau * N * lda + t.row0; }
  // A(r = mu, k = (segment sg, lambda = ta[sg] * NA + u)) = D^occ_{lambda mu}
  static constexpr bool kAStep = true;
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int adiv(const Tile&) const { return NA; }
  __device__ uint32_t akoff2(const Tile&, int sg, int u, const int* ta) const {
    return (uint32_t)(ta[sg] * NA + u) * (uint32_t)lda;
  }
  __device__ const T* bbase(const Tile& t) const { return t3c + t.col0; }
  __device__ int64_t bkoff(const Tile&, int k, const int* tb) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)tb[sg] * bs32 + i * NA * NR;
  }
  __device__ T ascale(const Tile&, int) const { return T(1); }
  // M_b[tau][sigma][slot][mu][P]: row mu, column (sigma, P)
  __device__ T* obase(const Tile& t) const {
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

// any pivot b0 .. b0 + ng - 1 whose stage-B column block c is needed
__device__ inline bool any_needed(const uint8_t* needb, int b0, int ng, int nat, int c) {
  for (int i = 0; i < ng; ++i)
    if (needb[(int64_t)(b0 + i) * nat + c]) return true;
  return false;
}

template <class T>
struct StageB {
  using In = T;
  using Out = T;
  struct Tile : TileBase {
    int g, row0, col0, seg0, nseg, p, cl, slot, KU;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kSegTab, kTabB = kSegTab;
  const T* dvg;             // [N][ld]: rows (pivot of the group, tau, sigma)
  const T* t3c;
  T* bp;
  const int32_t* goff;
  const int32_t* seg_atom;
  const int64_t* seg_brick;
  const int32_t* gc;
  const int32_t* gslot;
  const int32_t* ulen;
  const int64_t* bp_off;
  int n_rt, n_ct, rows_pt, cols_pt;
  int RS, NA, NR, PG, PC;   // RS: rows of this group (its pivots x n_tau x NA)
  int ld;                   // row stride of dvg (the plan's group rows)
  int64_t bs, BPS;
  int bs32;
  FastDiv fdNA, fdNR;
  // screened calls: needb[b * nat + c] = 0 when no chi block that N_b column
  // block c of pivot b feeds is kept (the block is then not computed)
  const uint8_t* needb;
  int b0, ng, nat;          // pivots b0 .. b0 + ng - 1 of this launch

  __device__ bool tile(int bx, int, int, Tile& t) const {
    const int per = n_rt * n_ct;
    t.g = bx / per;
    const int c = gc[t.g];
    if (needb && !any_needed(needb, b0, ng, nat, c)) return false;
    const int rem = bx % per;
    t.row0 = (rem % n_rt) * rows_pt;
    t.col0 = (rem / n_rt) * cols_pt;
    t.seg0 = goff[t.g];
    t.nseg = goff[t.g + 1] - t.seg0;
    t.K = NA * t.nseg;
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
  __device__ const T* abase(const Tile& t) const { return dvg + t.row0; }
  // A(r = (pivot, tau, sigma), k = (segment sg, nu = ta[sg] * NA + u)) = dvg[nu][r]
  static constexpr bool kAStep = true;
  __device__ int64_t aroff(const Tile&, int r) const { return r; }
  __device__ int adiv(const Tile&) const { return NA; }
  __device__ uint32_t akoff2(const Tile&, int sg, int u, const int* ta) const {
    return (uint32_t)(ta[sg] * NA + u) * (uint32_t)ld;
  }
  __device__ const T* bbase(const Tile& t) const { return t3c + t.col0; }
  __device__ int64_t bkoff(const Tile&, int k, const int* tb) const {
    const int sg = (int)fdNA.div((uint32_t)k), i = k - sg * NA;
    return (int64_t)tb[sg] * bs32 + i * NA * NR;
  }
  __device__ T ascale(const Tile&, int) const { return T(1); }
  // N_b panel: [pivot][tau][panel][sigma][u = slot*NA + mu][(cl, Q)]: row (pivot, tau,
  // sigma), column (mu, Q); (pivot, tau) is one merged index of BPS-sized slabs
  __device__ T* obase(const Tile& t) const { return bp + bp_off[t.p]; }
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

template <class T>
struct StageC {
  using In = T;
  using Out = double;
  struct Tile : TileBase {
    int p, tau, row0, KU, km0;
  };
  static constexpr bool kAScale = false, kDot = false;
  static constexpr int kTabA = kPanTab, kTabB = 0;
  const T* mb;
  const T* bp;
  double* chi;
  const int32_t* gc;
  const int32_t* kmap;
  const int32_t* km_off;
  const int32_t* ulen;
  const int64_t* bp_off;
  int g0, nR, n_rt, rows_pt;
  int N, NA, NR, NRI, PG, PC, nRmax, n_atoms;
  int sgs;                  // nRmax * N * NR: stride of sigma in M_b
  int64_t BPS;
  FastDiv fdNR, fdNA;
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
    return t.K > 0;
  }
  // one table entry per union atom j: the M_b offset of its first AO
  // function (the panel's functions are whole atoms, NA each)
  __device__ void fill(const Tile& t, int* ta, int*, int tid, int nt) const {
    const int nu = t.KU / NA;
    for (int j = tid; j < nu; j += nt) ta[j] = kmap[t.km0 + j * NA] * NR;
  }
  __device__ const T* abase(const Tile& t) const {
    return mb + (int64_t)t.tau * NA * nRmax * N * NR;
  }
  __device__ int64_t aroff(const Tile& t, int r) const {
    const int row = t.row0 + r, sl = (int)fdNR.div((uint32_t)row);
    return (int64_t)sl * N * NR + (row - sl * NR);
  }
  // k = (sigma = sg, u over the panel's AO functions); offsets within one tau
  // of M_b, below 2^31 (checked on the host)
  static constexpr bool kAStep = true, kBLin = true;
  __device__ int adiv(const Tile& t) const { return t.KU; }
  __device__ uint32_t akoff2(const Tile&, int sg, int u, const int* ta) const {
    const int j = (int)fdNA.div((uint32_t)u), i = u - j * NA;    // union atom j, function i
    return (uint32_t)sg * (uint32_t)sgs + (uint32_t)ta[j] + (uint32_t)(i * NR);
  }
  __device__ int bstride(const Tile&) const { return PC; }
  __device__ const T* bbase(const Tile& t) const {
    return bp + (int64_t)t.tau * BPS + bp_off[t.p];
  }
  __device__ T ascale(const Tile&, int) const { return T(1); }
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

// D^vir columns of the pivot atoms b .. b + ng - 1 of one stage-B group,
// gathered as dvg[nu][(g, tau, sigma)] (row stride ld; rows of pivots beyond
// ng are zero) for the systems of one batch (blockIdx.y = entry)
template <class T>
struct GatherEnt {
  const T* dv;
  T* dvg;
  int N, b, ng;
};

template <class T>
__global__ void gather_dvir_kernel(const GatherEnt<T>* __restrict__ ents, int NA, int n_tau, int ld) {
  const GatherEnt<T> en = ents[blockIdx.y];
  const int RS1 = n_tau * NA, N = en.N;
  const int64_t total = (int64_t)N * ld;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int nu = (int)(e / ld), rc = (int)(e % ld);
    const int g = rc / RS1, r2 = rc - g * RS1;
    const int tau = r2 / NA, sg = r2 - tau * NA;
    en.dvg[e] = g < en.ng ? en.dv[(int64_t)tau * N * N + (int64_t)nu * N + (int64_t)(en.b + g) * NA + sg]
                          : T(0);
  }
}

// FP64 -> FP32 copy of n elements (operands of the FP32 form)
__global__ void to_f32_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

hipError_t to_f32(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

// rows of n_rows x n_cols FP64 matrices to FP32 rows of stride ld >= n_cols,
// the padding set to zero
__global__ void to_f32_rows_kernel(const double* __restrict__ x, float* __restrict__ y, int64_t rows,
                                   int n_cols, int ld) {
  const int64_t total = rows * ld;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ld;
    const int c = (int)(i - r * ld);
    y[i] = c < n_cols ? (float)x[r * n_cols + c] : 0.f;
  }
}

hipError_t to_f32_rows(const double* x, float* y, int64_t rows, int n_cols, int ld, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((rows * ld + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(to_f32_rows_kernel, dim3(blocks), dim3(256), 0, st, x, y, rows, n_cols, ld);
  return hipGetLastError();
}

#include "chi_bf16x3.inc"

}  // namespace
}  // namespace gw
