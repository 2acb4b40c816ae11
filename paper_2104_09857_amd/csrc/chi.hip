// Block-sparse polarizability chi_PQ(tau) (Eq. 3): plans and launches.
//
// A plan holds, for every system of a batch, the brick grouping (kept
// bricks after the norm filter), the RI column panels of stage C, scratch for
// one pivot's half-contracted tensors and the problem descriptions of the
// three stages (chi_stages.hpp).  Execution walks the pivot index
// i = 0 .. max(n_atoms) - 1 and issues per stage ONE launch over the tiles
// of every system that has a pivot atom i, for all tau at once, so a batch of
// uneven molecules fills the chip with a few launches per pivot index instead
// of a few per (molecule, pivot).  Launches are plain grids or persistent
// grids that take tiles from a device queue (largest systems first).  The
// whole sequence can be captured once into a hipGraph and replayed.  The
// stage-C tile shape and the launch mode are chosen per shape class by an
// autotuner that times the candidates on the plan and caches the winner in a
// text file.  gw_contract_chi is the one-system, eager case of the same code.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <memory>
#include <new>
#include <numeric>
#include <sstream>
#include <type_traits>

#include "chi_stages.hpp"

namespace gw {
namespace {

// stage-C tile variants: rows of a tile (columns are one 160-wide panel)
//   FP64 and FP32  0: <WM 4, KC 32> 128 rows  1: <WM 2, KC 32> 64 rows  2: <WM 4, KC 16> 128 rows
//                  3: direct-to-LDS copies (tile_dma.hpp), 128 rows:
//                     FP64 <WM 4, WN 2, NB 5, KC 32> two chunks deep, one workgroup per CU,
//                     FP32 <WM 4, WN 2, NB 5, KC 16> three chunks deep, two per CU;
//                     needs NR a multiple of 2 (FP64) / 4 (FP32)
//   BF16x3  0: <WM 4, RB 4> 256 rows    1: <WM 4, RB 2> 128 rows   2: <WM 2, RB 4> 128 rows
//           3: direct-to-LDS copies three chunks deep (tile_bf16x3_dma.hpp),
//              <WM 4, RB 4> 256 rows
constexpr int kNVar = 4;
int c_rows(int prec, int v) {
  static const int f64[kNVar] = {128, 64, 128, 128}, f32[kNVar] = {128, 64, 128, 128},
                   bf[kNVar] = {256, 128, 128, 256};
  return prec == GW_BF16X3 ? bf[v] : prec == GW_FP32 ? f32[v] : f64[v];
}
// stage-C variant usable for this precision and RI block size
bool variant_ok(int prec, int NR, int v) {
  if (v < 0 || v >= kNVar) return false;
  if (v == 3 && prec != GW_BF16X3) return NR % (prec == GW_FP64 ? 2 : 4) == 0;
  return true;
}
// stage-B waves (FP64) / row blocks (BF16x3) by the row count n_tau * NA
int b_wm(int RS) { return RS <= 64 ? 2 : RS <= 96 ? 3 : RS <= 128 ? 4 : RS <= 160 ? 5 : 4; }
// stage-A/B column blocks per wave by the column count NA * NR of one RI
// atom block: 64-wide tiles for small bases, 192-wide otherwise
int ab_nb(int cols) { return cols <= 16 * AB_NBN * AB_WN ? AB_NBN : AB_NBW; }
int b_rb(int RS) { return RS <= 64 ? 2 : RS <= 96 ? 3 : RS <= 128 ? 4 : 5; }
// BF16x3 entries per atom of D and the bricks (the half contractions' index)
int bf_width(int NA) { return NA <= 8 ? 8 : 16; }

// Work of one stage at every pivot index, for a batched launch.
template <class P>
struct Table {
  std::vector<BatchEntry<P>> ent;
  std::vector<int32_t> toff;
  std::vector<int> ent0, toff0, n, work;
  BatchEntry<P>* d_ent = nullptr;
  int32_t* d_toff = nullptr;
  size_t cap_ent = 0, cap_toff = 0;

  void begin(int n_piv) {
    ent.clear();
    toff.clear();
    ent0.assign(n_piv, 0);
    toff0.assign(n_piv, 0);
    n.assign(n_piv, 0);
    work.assign(n_piv, 0);
  }
  void open(int piv) {
    ent0[piv] = (int)ent.size();
    toff0[piv] = (int)toff.size();
    toff.push_back(0);
  }
  void add(int piv, const P& p, int gx, int gy, int gz) {
    ent.push_back(BatchEntry<P>{p, gx, gy});
    work[piv] += gx * gy * gz;
    toff.push_back(work[piv]);
    n[piv]++;
  }
  gw_status upload(Scratch& mem, hipStream_t st) {
    if (ent.size() > cap_ent) {
      gw_status rc = mem.alloc(&d_ent, ent.size());
      if (rc != GW_OK) return rc;
      cap_ent = ent.size();
    }
    if (toff.size() > cap_toff) {
      gw_status rc = mem.alloc(&d_toff, toff.size());
      if (rc != GW_OK) return rc;
      cap_toff = toff.size();
    }
    if (!ent.empty())
      GW_HIP(hipMemcpyAsync(d_ent, ent.data(), ent.size() * sizeof(ent[0]), hipMemcpyHostToDevice, st));
    if (!toff.empty())
      GW_HIP(hipMemcpyAsync(d_toff, toff.data(), toff.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    return GW_OK;
  }
  Batched<P> at(int piv) const {
    Batched<P> b{};
    b.ent = d_ent + ent0[piv];
    b.tile_off = d_toff + toff0[piv];
    b.n_sys = n[piv];
    return b;
  }
};

// Buffers and problem descriptions of the FP64 (T = double) or FP32
// (T = float) form of one system.
template <class T>
struct FBufs {
  const T* dof = nullptr;      // filtered D^occ, D^vir in the operand type
  const T* dvf = nullptr;
  const T* t3c = nullptr;      // bricks in the operand type
  T* dvg = nullptr;            // gathered D^vir columns of the pivot
  T* mb = nullptr;             // M_b
  T* bp = nullptr;             // N_b panels
  // the same for the second pivot of a pair (SysPlan::pair_h)
  T* dvg1 = nullptr;
  T* mb1 = nullptr;
  T* bp1 = nullptr;
  StageA<T> sa{};
  StageB<T> sb{};
  StageC<T> sc{};
};

// One system of a plan.
struct SysPlan {
  gw_system s{};
  int na = 0, N = 0, NRI = 0, n_groups = 0, nRmax = 1, PG = 1, PC = 0, n_pan = 0;
  // pivot pairs: loop index i runs pivot i and pivot i + pair_h together (their
  // chi rows are disjoint); 0: one pivot per loop index
  int pair_h = 0;
  int64_t bs = 0, BPS = 0, BPS16 = 0;   // BPS16: BF16x3 N_b entries per tau
  BrickGroups G;
  Panels pan;
  std::vector<int32_t> acount;
  std::vector<double> asuffix;
  double fl_a = 0.0, fl_b = 0.0, fl_c = 0.0;   // FLOPs per tau (all blocks)
  double *dof = nullptr, *dvf = nullptr;       // filtered D stacks (FP64)
  float *dof32 = nullptr, *dvf32 = nullptr;    // their FP32 copies (FP32 form)
  int ld32 = 0;                                // row stride of dof32 (N rounded up to 4)
  uint8_t* dropped = nullptr;
  uint16_t *th = nullptr, *tl = nullptr, *doh = nullptr, *dol = nullptr, *dvh = nullptr, *dvl = nullptr;
  uint16_t *mh = nullptr, *ml = nullptr, *nh = nullptr, *nl = nullptr;
  uint16_t *mh1 = nullptr, *ml1 = nullptr, *nh1 = nullptr, *nl1 = nullptr;   // second pivot of a pair
  uint8_t* keep = nullptr;          // screener mask (one-system calls only)
  uint8_t* needb = nullptr;         // stage-B column blocks needed per pivot [na][na] (same)
  uint8_t* needa = nullptr;         // stage-A rows (AO atoms) needed per slot atom [na][na] (same)
  FBufs<double> f64;
  FBufs<float> f32;
  StageABf ba{};
  StageBBf bb{};
  StageCBf bc{};
};

template <class T>
FBufs<T>& bufs(SysPlan& P);
template <>
FBufs<double>& bufs<double>(SysPlan& P) { return P.f64; }
template <>
FBufs<float>& bufs<float>(SysPlan& P) { return P.f32; }

// per-pivot-index launch tables of the FP64 / FP32 form
template <class T>
struct FTables {
  Table<StageA<T>> tA;
  Table<StageB<T>> tB;
  Table<StageC<T>> tC;
  std::vector<GatherEnt<T>> gath;
  std::vector<int> gath0, gathn;
  GatherEnt<T>* d_gath = nullptr;
};

}  // namespace
}  // namespace gw

using namespace gw;

struct gw_chi_batch {
  int n_sys = 0, n_tau = 0, NA = 0, NR = 0, prec = GW_FP64, max_na = 0;
  int n_loop = 0;                    // pivot loop length (pairs count once)
  double eps_f = 0.0;
  bool timing = false;
  bool out_filter = true;            // zero chi blocks below eps_f at the end
  Scratch mem;
  std::vector<SysPlan> sys;
  std::vector<int> order;            // systems by decreasing size
  int variant = 0, persistent = 0;
  int RS = 0;              // rows of one pivot's half contraction (n_tau * NA)
  int GB = 1;              // pivots per stage-B launch (a group)
  int RSB = 0;             // rows of a full group (GB * RS)
  int LDB = 0;             // row stride of dvg: RSB rounded up to whole 16-byte groups
  int ab_nb = AB_NBW;      // 16-column blocks per wave of the stage-A/B tiles
  bool b_dma = false;      // stage B on the direct-to-LDS engine (FP64, FP32)
  bool a_dma = false;      // stage A on the direct-to-LDS engine (FP64, FP32)
  bool bf_dma_ab = false;  // BF16x3 stages A and B on the direct-to-LDS engine
  // where the plan's rows allow the direct-to-LDS half contractions (the
  // flags above follow these unless gw_chi_batch_set_engine chose engine 1)
  bool a_dma_ok = false, b_dma_ok = false, bf_dma_ok = false;
  int ab_engine = 0;
  FTables<double> t64;
  FTables<float> t32;
  Table<StageABf> tAb;
  Table<StageBBf> tBb;
  Table<StageCBf> tCb;
  int* queues = nullptr;
  int n_queues = 0;
  int* tiles_skipped = nullptr;
  // pointers the stage-C tables and the captured graph were built for
  std::vector<double*> bound_chi;
  std::vector<const double*> g_occ, g_vir;
  int c_built_variant = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_variant = -1, g_persistent = -1;
  hipStream_t g_stream = nullptr;
  std::vector<hipEvent_t> ev;        // per-stage timing events (eager runs)

  explicit gw_chi_batch(hipStream_t st) : mem(st, false) {}
  ~gw_chi_batch() {
    drop_graph();
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
};

namespace gw {
namespace {

// BF16x3 stage-A/B column blocks per wave (same rule as the FP64 / FP32 form)
int bf_ab_nb(const gw_chi_batch& B) {
  return B.NA * B.NR <= 16 * BF_NB_ABN * BF_WN ? BF_NB_ABN : BF_NB_AB;
}

// device copies of a system's grouping and panel index arrays
struct Index {
  int32_t *goff, *seg_atom, *gc, *gslot, *ulen, *kmap, *km_off;
  int64_t *seg_brick, *bp_off;
};

// scratch and problem descriptions of the FP64 / FP32 form of one system
template <class T>
gw_status prepare_f(gw_chi_batch& B, SysPlan& P, const gw_system* s, const Index& ix, hipStream_t st) {
  const int n_tau = B.n_tau, NA = B.NA, NR = B.NR, N = P.N, RS = B.RSB, LD = B.LDB;
  Scratch& M = B.mem;
  FBufs<T>& F = bufs<T>(P);
  gw_status rc;
  if constexpr (std::is_same<T, double>::value) {
    F.dof = P.dof;
    F.dvf = P.dvf;
    F.t3c = s->t3c;
  } else {
    // operands rounded to FP32 once: the bricks here, D(tau) at every execution
    const size_t dsz = (size_t)n_tau * N * N, tsz = (size_t)s->n_trip * P.bs;
    float* t32;
    // D^occ rows padded to a multiple of 4 floats (16-byte copies of stage A)
    if ((rc = M.alloc(&P.dof32, (size_t)n_tau * N * P.ld32)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.dvf32, dsz)) != GW_OK) return rc;
    if ((rc = M.alloc(&t32, tsz)) != GW_OK) return rc;
    GW_HIP(to_f32(s->t3c, t32, (int64_t)tsz, st));
    F.dof = P.dof32;
    F.dvf = P.dvf32;
    F.t3c = t32;
  }
  // per-tile offsets of the stage maps are 32-bit
  GW_CHECK_ARG((int64_t)N * P.ld32 < (1ll << 31) && (int64_t)N * LD < (1ll << 31) &&
                   (int64_t)NA * P.nRmax * N * NR < (1ll << 31) && P.bs < (1ll << 31),
               "system too large for 32-bit tile offsets");
  for (int p = 0; p < P.n_pan; ++p)
    GW_CHECK_ARG((int64_t)NA * NA * P.pan.ulen[p] * P.PC < (1ll << 31),
                 "column panel too large for 32-bit tile offsets");
  const size_t n_mb = (size_t)n_tau * NA * P.nRmax * N * NR, n_bp = (size_t)B.GB * n_tau * P.BPS;
  if ((rc = M.alloc(&F.dvg, (size_t)N * LD)) != GW_OK) return rc;
  if ((rc = M.alloc(&F.mb, n_mb)) != GW_OK) return rc;
  // N_b of every pivot of a stage-B group: [pivot][tau] slabs of BPS
  if ((rc = M.alloc(&F.bp, n_bp)) != GW_OK) return rc;
  // entries of N_b that no group writes stay zero for the life of the plan
  GW_HIP(hipMemsetAsync(F.bp, 0, sizeof(T) * n_bp, st));
  // buffers of the second pivot of a pair, within 32 GiB (else no pairs)
  if (P.pair_h > 0 && sizeof(T) * (n_mb + n_bp + (size_t)N * LD) > (32ull << 30)) P.pair_h = 0;
  if (P.pair_h > 0) {
    if ((rc = M.alloc(&F.dvg1, (size_t)N * LD)) != GW_OK) return rc;
    if ((rc = M.alloc(&F.mb1, n_mb)) != GW_OK) return rc;
    if ((rc = M.alloc(&F.bp1, n_bp)) != GW_OK) return rc;
    GW_HIP(hipMemsetAsync(F.bp1, 0, sizeof(T) * n_bp, st));
  }

  StageA<T>& sa = F.sa;
  sa.dof = F.dof; sa.t3c = F.t3c; sa.mb = F.mb; sa.goff = ix.goff; sa.seg_atom = ix.seg_atom;
  sa.gc = ix.gc; sa.nat = P.na;
  sa.seg_brick = ix.seg_brick; sa.rows_pt = 32 * A_WM; sa.cols_pt = 16 * B.ab_nb * AB_WN;
  sa.n_rt = (N + sa.rows_pt - 1) / sa.rows_pt;
  sa.n_ct = (NA * NR + sa.cols_pt - 1) / sa.cols_pt;
  sa.N = N; sa.NA = NA; sa.NR = NR; sa.nRmax = P.nRmax; sa.bs = P.bs; sa.bs32 = (int)P.bs;
  sa.lda = std::is_same<T, float>::value ? P.ld32 : N;
  sa.fdNA.set((uint32_t)NA);
  sa.fdNR.set((uint32_t)NR);

  StageB<T>& sb = F.sb;
  sb.dvg = F.dvg; sb.t3c = F.t3c; sb.bp = F.bp; sb.goff = ix.goff; sb.seg_atom = ix.seg_atom;
  sb.seg_brick = ix.seg_brick; sb.gc = ix.gc; sb.gslot = ix.gslot; sb.ulen = ix.ulen;
  sb.bp_off = ix.bp_off; sb.RS = RS; sb.ld = LD; sb.NA = NA; sb.NR = NR; sb.PG = P.PG; sb.PC = P.PC;
  sb.bs = P.bs; sb.bs32 = (int)P.bs; sb.BPS = P.BPS;
  sb.rows_pt = 32 * b_wm(RS);
  sb.cols_pt = 16 * B.ab_nb * AB_WN;
  sb.n_rt = (RS + sb.rows_pt - 1) / sb.rows_pt;
  sb.n_ct = (NA * NR + sb.cols_pt - 1) / sb.cols_pt;
  sb.fdNA.set((uint32_t)NA);
  sb.fdNR.set((uint32_t)NR);

  StageC<T>& sc = F.sc;
  sc.mb = F.mb; sc.bp = F.bp; sc.gc = ix.gc; sc.kmap = ix.kmap; sc.km_off = ix.km_off;
  sc.ulen = ix.ulen; sc.bp_off = ix.bp_off; sc.N = N; sc.NA = NA; sc.NR = NR; sc.NRI = P.NRI;
  sc.PG = P.PG; sc.PC = P.PC; sc.nRmax = P.nRmax; sc.n_atoms = P.na; sc.BPS = P.BPS;
  sc.sgs = P.nRmax * N * NR;
  sc.fdNR.set((uint32_t)NR);
  sc.fdNA.set((uint32_t)NA);
  return GW_OK;
}

gw_status prepare_sys(gw_chi_batch& B, SysPlan& P, const gw_system* s, hipStream_t st) {
  const int n_tau = B.n_tau, NA = B.NA, NR = B.NR;
  P.s = *s;
  P.na = s->n_atoms;
  P.N = P.na * NA;
  P.ld32 = (P.N + 3) / 4 * 4;
  P.NRI = P.na * NR;
  P.bs = (int64_t)NA * NA * NR;
  const int na = P.na, N = P.N;
  gw_status rc;
  if (s->n_trip > 0) {
    Scratch tmp(st);
    if ((rc = build_groups(s, B.eps_f, st, tmp, P.G)) != GW_OK) return rc;
  } else {
    P.G.goff.assign(1, 0);
    P.G.gb_start.assign(na + 1, 0);
  }
  const BrickGroups& G = P.G;
  P.n_groups = G.n_groups();
  P.nRmax = 1;
  for (int b = 0; b < na; ++b) P.nRmax = std::max(P.nRmax, G.gb_start[b + 1] - G.gb_start[b]);
  P.PG = std::max(1, C_COLS / NR);
  P.PC = P.PG * NR;
  P.pan = build_panels(na, P.PG, P.PC, G.gc, G.gs, NA, NA);
  P.n_pan = P.pan.n_pan;
  P.BPS = P.pan.off[P.n_pan];
  for (int g = 0; g < P.n_groups; ++g)
    GW_CHECK_ARG(G.goff[g + 1] - G.goff[g] <= kSegTab, "too many bricks in one (atom, RI atom) group");
  for (int p = 0; p < P.n_pan; ++p)
    GW_CHECK_ARG(P.pan.ulen[p] <= kPanTab, "too many AO atoms coupled to one RI column panel");

  // FLOPs of the three stages per tau (every output block computed)
  P.acount.assign(na, 0);
  for (int g = 0; g < P.n_groups; ++g) P.acount[G.gc[g]]++;
  P.asuffix.assign(na + 1, 0.0);
  for (int c = na - 1; c >= 0; --c) P.asuffix[c] = P.asuffix[c + 1] + P.acount[c];
  const double nnz = (double)G.n_kept * P.bs;
  for (int b = 0; b < na; ++b) {
    const int g0 = G.gb_start[b], nR = G.gb_start[b + 1] - g0;
    if (nR == 0) continue;
    int64_t nnz_b = 0;
    for (int g = g0; g < g0 + nR; ++g) nnz_b += (int64_t)(G.goff[g + 1] - G.goff[g]) * P.bs;
    P.fl_a += 2.0 * N * (double)nnz_b;
    P.fl_b += 2.0 * NA * nnz;
    for (int g = g0; g < g0 + nR; ++g) P.fl_c += 2.0 * NR * NR * NA * NA * P.asuffix[G.gc[g]];
  }

  // scratch of the plan (one pivot's half-contracted tensors)
  Scratch& M = B.mem;
  const int RS = n_tau * NA;
  const size_t dsz = (size_t)n_tau * N * N, nflag = (size_t)n_tau * na * na;
  if ((rc = M.alloc(&P.dof, dsz)) != GW_OK) return rc;
  if ((rc = M.alloc(&P.dvf, dsz)) != GW_OK) return rc;
  if ((rc = M.alloc(&P.dropped, 3 * nflag)) != GW_OK) return rc;
  int32_t *d_goff, *d_seg_atom, *d_gc, *d_gslot, *d_ulen, *d_kmap, *d_km_off;
  int64_t *d_seg_brick, *d_bp_off;
  if ((rc = M.upload(&d_goff, G.goff)) != GW_OK) return rc;
  if ((rc = M.upload(&d_seg_atom, G.seg_atom)) != GW_OK) return rc;
  if ((rc = M.upload(&d_seg_brick, G.seg_brick)) != GW_OK) return rc;
  if ((rc = M.upload(&d_gc, G.gc)) != GW_OK) return rc;
  if ((rc = M.upload(&d_gslot, P.pan.gslot)) != GW_OK) return rc;
  if ((rc = M.upload(&d_ulen, P.pan.ulen)) != GW_OK) return rc;
  if ((rc = M.upload(&d_kmap, P.pan.kmap)) != GW_OK) return rc;
  if ((rc = M.upload(&d_km_off, P.pan.km_off)) != GW_OK) return rc;
  if ((rc = M.upload(&d_bp_off, P.pan.off)) != GW_OK) return rc;

  const Index ix{d_goff, d_seg_atom, d_gc, d_gslot, d_ulen, d_kmap, d_km_off, d_seg_brick, d_bp_off};
  // pivot pairs (FP64 / FP32): pivots i and i + h, h = ceil(na / 2), share the
  // stage-C launch when no RI atom couples to both (their chi rows are then
  // disjoint); the launches of the strip's last pivots, whose upper-triangle
  // blocks are few, then carry the first pivots' tiles as well
  P.pair_h = 0;
  if (na >= 4) {
    const int h = (na + 1) / 2;
    std::vector<int> mark(na, -1);
    bool disjoint = true;
    for (int i = 0; i + h < na && disjoint; ++i) {
      for (int g = G.gb_start[i]; g < G.gb_start[i + 1]; ++g) mark[G.gc[g]] = i;
      for (int g = G.gb_start[i + h]; g < G.gb_start[i + h + 1]; ++g)
        if (mark[G.gc[g]] == i) disjoint = false;
    }
    if (disjoint) P.pair_h = h;
  }
  if (B.GB == 0) {
    // pivots per stage-B launch, fixed by the first system of the plan: up to
    // 128 (FP64) / 160 (FP32) rows (pivot, tau, sigma) per tile, the group's N_b
    // within 16 GiB (FP64: a 160-row tile needs ten waves, whose register
    // budget of 168 spills; 128 rows run on eight waves without spills)
    // (BF16x3: N_b hi + lo, its index packed per atom to E entries)
    int64_t slab = P.BPS * (B.prec == GW_FP64 ? 8 : 4);
    if (B.prec == GW_BF16X3) {
      const int64_t E = (NA * NA + 15) / 16 * 16;
      slab = 0;
      for (int p = 0; p < P.n_pan; ++p) slab += (int64_t)P.pan.ulen[p] * P.PC * E * 4;
    }
    int gb = std::max(1, (B.prec == GW_FP64 ? 128 : 160) / B.RS);
    while (gb > 1 && (int64_t)gb * n_tau * slab > (16ll << 30)) --gb;
    B.GB = gb;
    B.RSB = gb * B.RS;
    // the direct-to-LDS copies take D^vir rows in 16-byte groups (2 FP64 /
    // 4 FP32 elements); the padding rows of dvg are zeros (gather kernel)
    const int q = B.prec == GW_FP32 ? 4 : 2;
    B.LDB = (B.RSB + q - 1) / q * q;
  }
  if (B.prec == GW_FP64) {
    if ((rc = prepare_f<double>(B, P, s, ix, st)) != GW_OK) return rc;
  } else if (B.prec == GW_FP32) {
    if ((rc = prepare_f<float>(B, P, s, ix, st)) != GW_OK) return rc;
  } else {
    // split-precision form: operands as bf16 hi/lo pairs; T is split once per plan.
    // M_b and N_b hold the outer contraction's index (AO function i of an atom,
    // sigma) packed per atom: E = NA^2 rounded up to 16 entries, G = E / 16 k
    // pairs of 16 per atom, each pair stored [pair][row or column][16]
    const int E = (NA * NA + 15) / 16 * 16, Gp = E / 16;
    std::vector<int64_t> poffb(P.n_pan + 1, 0);
    std::vector<int32_t> ptab, pt_off(P.n_pan + 1, 0);
    for (int p = 0; p < P.n_pan; ++p) {
      poffb[p + 1] = poffb[p] + (int64_t)P.pan.ulen[p] * P.PC * E;
      GW_CHECK_ARG(P.pan.ulen[p] <= kPanTab, "too many AO atoms coupled to one RI column panel");
      for (int j = 0; j < P.pan.ulen[p]; ++j) {
        const int a = P.pan.kmap[P.pan.km_off[p] + j * NA] / NA;   // union atom j
        for (int e = 0; e < Gp; ++e) ptab.push_back(a * Gp + e);
      }
      pt_off[p + 1] = (int32_t)ptab.size();
    }
    P.BPS16 = poffb[P.n_pan];
    int64_t* d_poffb;
    int32_t *d_ptab, *d_pt_off;
    if ((rc = M.upload(&d_poffb, poffb)) != GW_OK) return rc;
    if ((rc = M.upload(&d_ptab, ptab)) != GW_OK) return rc;
    if ((rc = M.upload(&d_pt_off, pt_off)) != GW_OK) return rc;
    // D and the bricks carry W entries per atom (8 for bases of at most 8 functions)
    const int W = bf_width(NA);
    const size_t tsz = (size_t)s->n_trip * NR * NA * W, dsz16 = (size_t)n_tau * N * na * W;
    // N_b of every pivot of a stage-B group: [pivot][tau] slabs of BPS16
    const size_t msz = (size_t)n_tau * P.nRmax * NR * na * E, nsz = (size_t)B.GB * n_tau * P.BPS16;
    // the direct-to-LDS outer contraction takes its M_b offsets within one tau in 32 bits
    GW_CHECK_ARG((int64_t)(P.nRmax + 1) * NR * na * E < (1ll << 31),
                 "system too large for 32-bit tile offsets");
    (void)d_kmap; (void)d_km_off; (void)d_ulen;
    if ((rc = M.alloc(&P.th, tsz)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.tl, tsz)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.doh, dsz16)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.dol, dsz16)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.dvh, dsz16)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.dvl, dsz16)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.mh, msz)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.ml, msz)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.nh, nsz)) != GW_OK) return rc;
    if ((rc = M.alloc(&P.nl, nsz)) != GW_OK) return rc;
    // padding entries (past NA^2 of an atom block) and uncoupled panel entries stay zero
    GW_HIP(hipMemsetAsync(P.mh, 0, 2 * msz, st));
    GW_HIP(hipMemsetAsync(P.ml, 0, 2 * msz, st));
    GW_HIP(hipMemsetAsync(P.nh, 0, 2 * nsz, st));
    GW_HIP(hipMemsetAsync(P.nl, 0, 2 * nsz, st));
    // buffers of the second pivot of a pair, within 32 GiB (else no pairs)
    if (P.pair_h > 0 && 2 * 2 * (msz + nsz) > (32ull << 30)) P.pair_h = 0;
    if (P.pair_h > 0) {
      if ((rc = M.alloc(&P.mh1, msz)) != GW_OK) return rc;
      if ((rc = M.alloc(&P.ml1, msz)) != GW_OK) return rc;
      if ((rc = M.alloc(&P.nh1, nsz)) != GW_OK) return rc;
      if ((rc = M.alloc(&P.nl1, nsz)) != GW_OK) return rc;
      GW_HIP(hipMemsetAsync(P.mh1, 0, 2 * msz, st));
      GW_HIP(hipMemsetAsync(P.ml1, 0, 2 * msz, st));
      GW_HIP(hipMemsetAsync(P.nh1, 0, 2 * nsz, st));
      GW_HIP(hipMemsetAsync(P.nl1, 0, 2 * nsz, st));
    }
    if (s->n_trip > 0) {
      const unsigned blocks = (unsigned)std::min<int64_t>(((int64_t)tsz + 255) / 256, 1 << 20);
      hipLaunchKernelGGL(split_t_kernel, dim3(blocks), dim3(256), 0, st, s->t3c, P.th, P.tl,
                         s->n_trip, NA, NR, W);
      GW_HIP(hipGetLastError());
    }

    StageABf& ba = P.ba;
    ba.dh = P.doh; ba.dl = P.dol; ba.th = P.th; ba.tl = P.tl; ba.mh = P.mh; ba.ml = P.ml;
    ba.goff = d_goff; ba.seg_atom = d_seg_atom; ba.seg_brick = d_seg_brick; ba.gc = d_gc;
    ba.rows_pt = 16 * 4 * 4; ba.cols_pt = 16 * bf_ab_nb(B) * BF_WN;
    ba.n_rt = (N + ba.rows_pt - 1) / ba.rows_pt;
    ba.n_ct = (NA * NR + ba.cols_pt - 1) / ba.cols_pt;
    ba.N = N; ba.NA = NA; ba.NR = NR; ba.na = na; ba.nRmax = P.nRmax; ba.G = Gp; ba.W = W;
    ba.fdNA.set((uint32_t)NA);

    StageBBf& bb = P.bb;
    bb.dh = P.dvh; bb.dl = P.dvl; bb.th = P.th; bb.tl = P.tl; bb.nh = P.nh; bb.nl = P.nl;
    bb.goff = d_goff; bb.seg_atom = d_seg_atom; bb.seg_brick = d_seg_brick; bb.gc = d_gc;
    bb.gslot = d_gslot; bb.poffb = d_poffb; bb.N = N; bb.NA = NA; bb.NR = NR; bb.na = na;
    bb.RS = RS; bb.PG = P.PG; bb.PC = P.PC; bb.G = Gp; bb.W = W; bb.BPSE = P.BPS16;
    bb.n_tau = n_tau; bb.ng = 1;
    bb.fdGN.set((uint32_t)NA);
    bb.rows_pt = 16 * b_rb(B.RSB) * 2;
    bb.cols_pt = 16 * bf_ab_nb(B) * BF_WN;
    bb.n_rt = (RS + bb.rows_pt - 1) / bb.rows_pt;
    bb.n_ct = (NA * NR + bb.cols_pt - 1) / bb.cols_pt;
    bb.fdNA.set((uint32_t)NA);

    StageCBf& bc = P.bc;
    bc.mh = P.mh; bc.ml = P.ml; bc.nh = P.nh; bc.nl = P.nl; bc.gc = d_gc; bc.ptab = d_ptab;
    bc.pt_off = d_pt_off; bc.poffb = d_poffb; bc.NA = NA; bc.NR = NR; bc.NRI = P.NRI;
    bc.PG = P.PG; bc.PC = P.PC; bc.nRmax = P.nRmax; bc.n_atoms = na; bc.na = na;
    bc.G = Gp; bc.BPSE = P.BPS16;
    bc.fdNR.set((uint32_t)NR);
    bc.fdG.set((uint32_t)Gp);
  }
  return GW_OK;
}

template <class T>
FTables<T>& tabs(gw_chi_batch& B);
template <>
FTables<double>& tabs<double>(gw_chi_batch& B) { return B.t64; }
template <>
FTables<float>& tabs<float>(gw_chi_batch& B) { return B.t32; }
template <class T>
const FTables<T>& tabs(const gw_chi_batch& B) { return tabs<T>(const_cast<gw_chi_batch&>(B)); }

// pivot atom index piv of system P: first group and group count (0: no work)
inline int pivot_groups(const SysPlan& P, int piv, int& g0) {
  if (piv >= P.na) return 0;
  g0 = P.G.gb_start[piv];
  return P.G.gb_start[piv + 1] - g0;
}

// the pivots of system P at loop index i: pivot, buffer slot and the range
// [lo, hi) of pivots of that slot (stage-B groups do not cross it)
struct PivSlot {
  int piv, slot, lo, hi;
};
inline int loop_pivots(const SysPlan& P, int i, PivSlot out[2]) {
  if (P.pair_h == 0) {
    if (i >= P.na) return 0;
    out[0] = PivSlot{i, 0, 0, P.na};
    return 1;
  }
  int n = 0;
  if (i < P.pair_h) out[n++] = PivSlot{i, 0, 0, P.pair_h};
  if (i + P.pair_h < P.na) out[n++] = PivSlot{i + P.pair_h, 1, P.pair_h, P.na};
  return n;
}

// tables of stages A and B (and the D^vir gathers) for every loop index
template <class T>
gw_status ab_tables_f(gw_chi_batch& B, hipStream_t st) {
  FTables<T>& F = tabs<T>(B);
  const int n_idx = B.n_loop, n_tau = B.n_tau;
  F.tA.begin(n_idx);
  F.tB.begin(n_idx);
  F.gath.clear();
  F.gath0.assign(n_idx, 0);
  F.gathn.assign(n_idx, 0);
  for (int i = 0; i < n_idx; ++i) {
    F.tA.open(i);
    F.tB.open(i);
    F.gath0[i] = (int)F.gath.size();
    for (int m : B.order) {
      SysPlan& P = B.sys[m];
      FBufs<T>& pb = bufs<T>(P);
      PivSlot ps[2];
      const int np = loop_pivots(P, i, ps);
      for (int k = 0; k < np; ++k) {
        const int piv = ps[k].piv;
        const bool s1 = ps[k].slot == 1;
        int g0 = 0;
        const int nR = pivot_groups(P, piv, g0);
        if (nR > 0) {
          StageA<T> a = pb.sa;
          a.needa = P.needa;
          a.g0 = g0;
          a.mb = s1 ? pb.mb1 : pb.mb;
          F.tA.add(i, a, nR * a.n_rt * a.n_ct, n_tau, 1);
        }
        // stage B once per group of GB pivots of the slot, at its first
        // pivot: rows (pivot, tau, sigma) of the group's pivots
        if ((piv - ps[k].lo) % B.GB != 0) continue;
        const int ng = std::min(B.GB, ps[k].hi - piv);
        StageB<T> b = pb.sb;
        b.RS = ng * B.RS;
        b.needb = P.needb;
        b.b0 = piv;
        b.ng = ng;
        b.nat = P.na;
        b.n_rt = (b.RS + b.rows_pt - 1) / b.rows_pt;
        b.dvg = s1 ? pb.dvg1 : pb.dvg;
        b.bp = s1 ? pb.bp1 : pb.bp;
        F.tB.add(i, b, P.n_groups * b.n_rt * b.n_ct, 1, 1);
        F.gath.push_back(GatherEnt<T>{pb.dvf, s1 ? pb.dvg1 : pb.dvg, P.N, piv, ng});
        F.gathn[i]++;
      }
    }
  }
  gw_status rc;
  if ((rc = F.tA.upload(B.mem, st)) != GW_OK) return rc;
  if ((rc = F.tB.upload(B.mem, st)) != GW_OK) return rc;
  return B.mem.upload(&F.d_gath, F.gath);
}

gw_status ab_tables_bf(gw_chi_batch& B, hipStream_t st) {
  const int n_idx = B.n_loop, n_tau = B.n_tau;
  B.tAb.begin(n_idx);
  B.tBb.begin(n_idx);
  for (int i = 0; i < n_idx; ++i) {
    B.tAb.open(i);
    B.tBb.open(i);
    for (int m : B.order) {
      SysPlan& P = B.sys[m];
      PivSlot ps[2];
      const int np = loop_pivots(P, i, ps);
      for (int k = 0; k < np; ++k) {
        const int piv = ps[k].piv;
        const bool s1 = ps[k].slot == 1;
        int g0 = 0;
        const int nR = pivot_groups(P, piv, g0);
        if (nR > 0) {
          StageABf a = P.ba;
          a.needa = P.needa;
          a.g0 = g0;
          a.mh = s1 ? P.mh1 : P.mh;
          a.ml = s1 ? P.ml1 : P.ml;
          B.tAb.add(i, a, nR * a.n_rt * a.n_ct, n_tau, 1);
        }
        // stage B once per group of GB pivots of the slot, at its first
        // pivot: rows (tau, pivot, sigma) of the group's pivots
        if ((piv - ps[k].lo) % B.GB != 0) continue;
        StageBBf b = P.bb;
        b.needb = P.needb;
        b.b = piv;
        b.ng = std::min(B.GB, ps[k].hi - piv);
        b.RS = n_tau * b.ng * B.NA;
        b.fdGN.set((uint32_t)(b.ng * B.NA));
        b.n_rt = (b.RS + b.rows_pt - 1) / b.rows_pt;
        b.nh = s1 ? P.nh1 : P.nh;
        b.nl = s1 ? P.nl1 : P.nl;
        B.tBb.add(i, b, P.n_groups * b.n_rt * b.n_ct, 1, 1);
      }
    }
  }
  gw_status rc;
  if ((rc = B.tAb.upload(B.mem, st)) != GW_OK) return rc;
  return B.tBb.upload(B.mem, st);
}

gw_status build_ab_tables(gw_chi_batch& B, hipStream_t st) {
  if (B.prec == GW_FP64) return ab_tables_f<double>(B, st);
  if (B.prec == GW_FP32) return ab_tables_f<float>(B, st);
  return ab_tables_bf(B, st);
}

// stage-C tables for the current variant and output pointers
template <class C, class Get>
void c_tables(gw_chi_batch& B, Table<C>& tab, Get get, double* const* chi) {
  // get(P, ps): the system's stage-C problem for pivot ps.piv of buffer slot ps.slot
  const int n_idx = B.n_loop, n_tau = B.n_tau, rows = c_rows(B.prec, B.variant);
  tab.begin(n_idx);
  for (int i = 0; i < n_idx; ++i) {
    tab.open(i);
    for (int m : B.order) {
      SysPlan& P = B.sys[m];
      PivSlot ps[2];
      const int np = loop_pivots(P, i, ps);
      for (int k = 0; k < np; ++k) {
        int g0 = 0;
        const int nR = pivot_groups(P, ps[k].piv, g0);
        if (nR == 0) continue;
        const int n_rt = (nR * B.NR + rows - 1) / rows;
        C c = get(P, ps[k]);
        c.chi = chi[m];
        c.g0 = g0;
        c.nR = nR;
        c.rows_pt = rows;
        c.n_rt = n_rt;
        c.keep = P.keep;
        c.tiles_skipped = B.tiles_skipped;
        tab.add(i, c, n_rt * P.n_pan, 1, n_tau);
      }
    }
  }
}

gw_status build_c_tables(gw_chi_batch& B, double* const* chi, hipStream_t st) {
  gw_status rc;
  // FP64 / FP32: pivot piv reads M_b of its slot and its slab of the slot's
  // stage-B group N_b
  const int64_t slab = (int64_t)B.n_tau;
  auto slot_c = [&](auto& F, const SysPlan& P, const PivSlot& ps) {
    auto c = F.sc;
    const bool s1 = ps.slot == 1;
    c.mb = s1 ? F.mb1 : F.mb;
    c.bp = (s1 ? F.bp1 : F.bp) + ((ps.piv - ps.lo) % B.GB) * slab * P.BPS;
    return c;
  };
  if (B.prec == GW_FP64) {
    c_tables(B, B.t64.tC, [&](SysPlan& P, const PivSlot& ps) { return slot_c(P.f64, P, ps); }, chi);
    rc = B.t64.tC.upload(B.mem, st);
  } else if (B.prec == GW_FP32) {
    c_tables(B, B.t32.tC, [&](SysPlan& P, const PivSlot& ps) { return slot_c(P.f32, P, ps); }, chi);
    rc = B.t32.tC.upload(B.mem, st);
  } else {
    // BF16x3: pivot piv reads M_b of its slot and its slab of the slot's
    // stage-B group N_b
    c_tables(B, B.tCb, [&](SysPlan& P, const PivSlot& ps) {
      StageCBf c = P.bc;
      const bool s1 = ps.slot == 1;
      const int64_t off = (int64_t)((ps.piv - ps.lo) % B.GB) * B.n_tau * P.BPS16;
      c.mh = s1 ? P.mh1 : P.mh;
      c.ml = s1 ? P.ml1 : P.ml;
      c.nh = (s1 ? P.nh1 : P.nh) + off;
      c.nl = (s1 ? P.nl1 : P.nl) + off;
      return c;
    }, chi);
    rc = B.tCb.upload(B.mem, st);
  }
  if (rc != GW_OK) return rc;
  B.bound_chi.assign(chi, chi + B.n_sys);
  B.c_built_variant = B.variant;
  return GW_OK;
}

// With queue == nullptr the call only computes the persistent grid size of
// the kernel (done at plan creation, outside any graph capture).
template <int WM, int WN, int NB, int KC, class P>
hipError_t run_mfma(const Table<P>& T, int piv, bool pers, int* queue, hipStream_t st) {
  if (!queue) {
    (void)persistent_cap_gemm<WM, WN, NB, KC, Batched<P>>();
    return hipSuccess;
  }
  const int work = T.work[piv];
  if (T.n[piv] == 0 || work == 0) return hipSuccess;
  if (!pers && T.n[piv] == 1) {         // one system: its own 3D grid, problem in kernel arguments
    const BatchEntry<P>& e = T.ent[T.ent0[piv]];
    return launch_tile_gemm<WM, WN, NB, KC>(e.p, dim3(e.gx, e.gy, work / (e.gx * e.gy)), st);
  }
  const Batched<P> b = T.at(piv);
  return pers ? launch_tile_gemm_persistent<WM, WN, NB, KC>(b, work, queue, st)
              : launch_tile_gemm<WM, WN, NB, KC>(b, dim3((unsigned)work), st);
}

// the same for the direct-to-LDS form of the outer contraction
template <int WM, int WN, int NB, int KC, int S, class P>
hipError_t run_dma(const Table<P>& T, int piv, bool pers, int* queue, hipStream_t st) {
  if (!queue) {
    (void)persistent_cap_dma<WM, WN, NB, KC, S, Batched<P>>();
    return hipSuccess;
  }
  const int work = T.work[piv];
  if (T.n[piv] == 0 || work == 0) return hipSuccess;
  // a one-system grid launch of a narrow tile takes the problem in its
  // arguments (many small tiles: no table search per tile); wide tiles go
  // through the batched form, whose kernel needs fewer registers (two
  // workgroups per CU)
  if (NB <= AB_NBN && !pers && T.n[piv] == 1) {
    const BatchEntry<P>& e = T.ent[T.ent0[piv]];
    return launch_tile_dma<WM, WN, NB, KC, S>(e.p, dim3(e.gx, e.gy, work / (e.gx * e.gy)), st);
  }
  const Batched<P> b = T.at(piv);
  return pers ? launch_tile_dma_persistent<WM, WN, NB, KC, S>(b, work, queue, st)
              : launch_tile_dma<WM, WN, NB, KC, S>(b, dim3((unsigned)work), st);
}

template <int WM, int WN, int RB, int NB, int KC, class P>
hipError_t run_bf(const Table<P>& T, int piv, bool pers, int* queue, hipStream_t st) {
  if (!queue) {
    (void)persistent_cap_bf16x3<WM, WN, RB, NB, KC, Batched<P>>();
    return hipSuccess;
  }
  const int work = T.work[piv];
  if (T.n[piv] == 0 || work == 0) return hipSuccess;
  if (!pers && T.n[piv] == 1) {
    const BatchEntry<P>& e = T.ent[T.ent0[piv]];
    return launch_tile_bf16x3<WM, WN, RB, NB, KC>(e.p, dim3(e.gx, e.gy, work / (e.gx * e.gy)), st);
  }
  const Batched<P> b = T.at(piv);
  return pers ? launch_tile_bf16x3_persistent<WM, WN, RB, NB, KC>(b, work, queue, st)
              : launch_tile_bf16x3<WM, WN, RB, NB, KC>(b, dim3((unsigned)work), st);
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
hipError_t run_bf_dma(const Table<P>& T, int piv, bool pers, int* queue, hipStream_t st) {
  if (!queue) {
    (void)persistent_cap_bf3_dma<WM, WN, RB, NB, S, HS, Batched<P>>();
    return hipSuccess;
  }
  const int work = T.work[piv];
  if (T.n[piv] == 0 || work == 0) return hipSuccess;
  if (!pers && T.n[piv] == 1) {
    const BatchEntry<P>& e = T.ent[T.ent0[piv]];
    return launch_tile_bf3_dma<WM, WN, RB, NB, S, HS>(e.p, dim3(e.gx, e.gy, work / (e.gx * e.gy)), st);
  }
  const Batched<P> b = T.at(piv);
  return pers ? launch_tile_bf3_dma_persistent<WM, WN, RB, NB, S, HS>(b, work, queue, st)
              : launch_tile_bf3_dma<WM, WN, RB, NB, S, HS>(b, dim3((unsigned)work), st);
}

template <class T>
hipError_t stage_a_f(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (B.a_dma) {
    if (B.ab_nb == AB_NBN) return run_dma<A_WM, AB_WN, AB_NBN, 16, 2>(tabs<T>(B).tA, piv, pers, q, st);
    return run_dma<A_WM, AB_WN, AB_NBW, 16, 2>(tabs<T>(B).tA, piv, pers, q, st);
  }
  if (B.ab_nb == AB_NBN) return run_mfma<A_WM, AB_WN, AB_NBN, 16>(tabs<T>(B).tA, piv, pers, q, st);
  return run_mfma<A_WM, AB_WN, AB_NBW, 16>(tabs<T>(B).tA, piv, pers, q, st);
}
template <int NB, class Tab>
hipError_t stage_b_rows(const gw_chi_batch& B, const Tab& t, int piv, bool pers, int* q, hipStream_t st) {
  switch (b_wm(B.RSB)) {
    case 2: return run_mfma<2, AB_WN, NB, 16>(t, piv, pers, q, st);
    case 3: return run_mfma<3, AB_WN, NB, 16>(t, piv, pers, q, st);
    case 5: return run_mfma<5, AB_WN, NB, 16>(t, piv, pers, q, st);
    default: return run_mfma<4, AB_WN, NB, 16>(t, piv, pers, q, st);
  }
}
template <int NB, class Tab>
hipError_t stage_b_dma_rows(const gw_chi_batch& B, const Tab& t, int piv, bool pers, int* q, hipStream_t st) {
  switch (b_wm(B.RSB)) {
    case 2: return run_dma<2, AB_WN, NB, 16, 2>(t, piv, pers, q, st);
    case 3: return run_dma<3, AB_WN, NB, 16, 2>(t, piv, pers, q, st);
    case 5: return run_dma<5, AB_WN, NB, 16, 2>(t, piv, pers, q, st);
    default: return run_dma<4, AB_WN, NB, 16, 2>(t, piv, pers, q, st);
  }
}
template <class T>
hipError_t stage_b_f(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (B.b_dma) {
    if (B.ab_nb == AB_NBN) return stage_b_dma_rows<AB_NBN>(B, tabs<T>(B).tB, piv, pers, q, st);
    return stage_b_dma_rows<AB_NBW>(B, tabs<T>(B).tB, piv, pers, q, st);
  }
  if (B.ab_nb == AB_NBN) return stage_b_rows<AB_NBN>(B, tabs<T>(B).tB, piv, pers, q, st);
  return stage_b_rows<AB_NBW>(B, tabs<T>(B).tB, piv, pers, q, st);
}
template <class T>
hipError_t stage_c_f(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  const auto& t = tabs<T>(B).tC;
  switch (B.variant) {
    case 1: return run_mfma<2, C_WN, C_NBW, C_KC>(t, piv, pers, q, st);
    case 2: return run_mfma<4, C_WN, C_NBW, 16>(t, piv, pers, q, st);
    case 3:
      if constexpr (std::is_same<T, double>::value) return run_dma<4, 2, 5, 32, 2>(t, piv, pers, q, st);
      else return run_dma<4, C_WN, C_NBW, 16, 3>(t, piv, pers, q, st);
    default: return run_mfma<4, C_WN, C_NBW, C_KC>(t, piv, pers, q, st);
  }
}
// the direct-to-LDS stage A / B instance for the plan's table width: with
// 8 entries per atom a k pair spans two segments (half select)
template <int HS>
hipError_t stage_a_bf_dma(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (bf_ab_nb(B) == BF_NB_ABN) return run_bf_dma<4, BF_WN, 4, BF_NB_ABN, 3, HS>(B.tAb, piv, pers, q, st);
  return run_bf_dma<4, BF_WN, 4, BF_NB_AB, 2, HS>(B.tAb, piv, pers, q, st);
}
template <int NB, int HS>
hipError_t stage_b_bf_dma(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if constexpr (NB == BF_NB_AB) {
    switch (b_rb(B.RSB)) {
      case 2: return run_bf_dma<2, BF_WN_B, 2, BF_NB_B, 3, HS>(B.tBb, piv, pers, q, st);
      case 3: return run_bf_dma<2, BF_WN_B, 3, BF_NB_B, 3, HS>(B.tBb, piv, pers, q, st);
      case 4: return run_bf_dma<2, BF_WN_B, 4, BF_NB_B, 3, HS>(B.tBb, piv, pers, q, st);
      default: return run_bf_dma<2, BF_WN_B, 5, BF_NB_B, 3, HS>(B.tBb, piv, pers, q, st);
    }
  } else {
    switch (b_rb(B.RSB)) {
      case 2: return run_bf_dma<2, BF_WN, 2, NB, 3, HS>(B.tBb, piv, pers, q, st);
      case 3: return run_bf_dma<2, BF_WN, 3, NB, 3, HS>(B.tBb, piv, pers, q, st);
      case 4: return run_bf_dma<2, BF_WN, 4, NB, 3, HS>(B.tBb, piv, pers, q, st);
      default: return run_bf_dma<2, BF_WN, 5, NB, 3, HS>(B.tBb, piv, pers, q, st);
    }
  }
}
hipError_t stage_a_bf(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (B.bf_dma_ab) {
    return bf_width(B.NA) == 8 ? stage_a_bf_dma<1>(B, piv, pers, q, st) : stage_a_bf_dma<0>(B, piv, pers, q, st);
  }
  if (bf_ab_nb(B) == BF_NB_ABN) return run_bf<4, BF_WN, 4, BF_NB_ABN, BF_KC>(B.tAb, piv, pers, q, st);
  return run_bf<4, BF_WN, 4, BF_NB_AB, BF_KC>(B.tAb, piv, pers, q, st);
}
template <int NB>
hipError_t stage_b_bf_rows(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (B.bf_dma_ab) {
    return bf_width(B.NA) == 8 ? stage_b_bf_dma<NB, 1>(B, piv, pers, q, st) : stage_b_bf_dma<NB, 0>(B, piv, pers, q, st);
  }
  switch (b_rb(B.RSB)) {
    case 2: return run_bf<2, BF_WN, 2, NB, BF_KC>(B.tBb, piv, pers, q, st);
    case 3: return run_bf<2, BF_WN, 3, NB, BF_KC>(B.tBb, piv, pers, q, st);
    case 4: return run_bf<2, BF_WN, 4, NB, BF_KC>(B.tBb, piv, pers, q, st);
    default: return run_bf<2, BF_WN, 5, NB, BF_KC>(B.tBb, piv, pers, q, st);
  }
}
hipError_t stage_b_bf(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  if (bf_ab_nb(B) == BF_NB_ABN) return stage_b_bf_rows<BF_NB_ABN>(B, piv, pers, q, st);
  return stage_b_bf_rows<BF_NB_AB>(B, piv, pers, q, st);
}
hipError_t stage_c_bf(const gw_chi_batch& B, int piv, bool pers, int* q, hipStream_t st) {
  switch (B.variant) {
    case 1: return run_bf<4, BF_WN, 2, BF_NB_C, BF_KC>(B.tCb, piv, pers, q, st);
    case 2: return run_bf<2, BF_WN, 4, BF_NB_C, BF_KC>(B.tCb, piv, pers, q, st);
    case 3: return run_bf_dma<4, BF_WN, 4, BF_NB_C, 3, 0>(B.tCb, piv, pers, q, st);
    default: return run_bf<4, BF_WN, 4, BF_NB_C, BF_KC>(B.tCb, piv, pers, q, st);
  }
}

// persistent grid sizes of every kernel a plan may launch
void prime(gw_chi_batch& B) {
  const int v0 = B.variant;
  for (int v = 0; v < kNVar; ++v) {
    B.variant = v;
    if (B.prec == GW_FP64) {
      (void)stage_a_f<double>(B, 0, true, nullptr, nullptr);
      (void)stage_b_f<double>(B, 0, true, nullptr, nullptr);
      (void)stage_c_f<double>(B, 0, true, nullptr, nullptr);
    } else if (B.prec == GW_FP32) {
      (void)stage_a_f<float>(B, 0, true, nullptr, nullptr);
      (void)stage_b_f<float>(B, 0, true, nullptr, nullptr);
      (void)stage_c_f<float>(B, 0, true, nullptr, nullptr);
    } else {
      (void)stage_a_bf(B, 0, true, nullptr, nullptr);
      (void)stage_b_bf(B, 0, true, nullptr, nullptr);
      (void)stage_c_bf(B, 0, true, nullptr, nullptr);
    }
  }
  B.variant = v0;
}

// the three stages of pivot index piv, FP64 / FP32 form
template <class T>
gw_status pivot_f(gw_chi_batch& B, int piv, int pers, int* q, std::vector<hipEvent_t>* ev,
                  hipStream_t st) {
  const FTables<T>& F = tabs<T>(B);
  auto mark = [&](int k) -> hipError_t { return ev ? hipEventRecord((*ev)[4 * piv + k], st) : hipSuccess; };
  if (F.gathn[piv] > 0) {
    int64_t most = 0;
    for (int e = 0; e < F.gathn[piv]; ++e)
      most = std::max<int64_t>(most, (int64_t)F.gath[F.gath0[piv] + e].N * B.LDB);
    const unsigned bx = (unsigned)std::min<int64_t>((most + 255) / 256, 4096);
    hipLaunchKernelGGL(gather_dvir_kernel<T>, dim3(bx, (unsigned)F.gathn[piv]), dim3(256), 0, st,
                       F.d_gath + F.gath0[piv], B.NA, B.n_tau, B.LDB);
    GW_HIP(hipGetLastError());
  }
  GW_HIP(mark(0));
  GW_HIP(stage_a_f<T>(B, piv, pers & 1, q, st));
  GW_HIP(mark(1));
  GW_HIP(stage_b_f<T>(B, piv, pers & 2, q + kXcds, st));
  GW_HIP(mark(2));
  GW_HIP(stage_c_f<T>(B, piv, pers & 4, q + 2 * kXcds, st));
  GW_HIP(mark(3));
  return GW_OK;
}

// Every launch of one execution, in stream order (no allocation, copy,
// memset or synchronization: the sequence may be captured into a graph).
// With `ev` (eager runs only) events bracket each stage of each pivot.
gw_status enqueue(gw_chi_batch& B, const double* const* occ, const double* const* vir,
                  double* const* chi, std::vector<hipEvent_t>* ev, hipStream_t st) {
  const int n_tau = B.n_tau, NA = B.NA, NR = B.NR;
  const int pers = B.persistent;     // bit k: stage k in the persistent form
  GW_HIP(fill_zero(B.queues, B.n_queues, st));
  for (int m = 0; m < B.n_sys; ++m) {
    SysPlan& P = B.sys[m];
    const size_t nflag = (size_t)n_tau * P.na * P.na;
    GW_HIP(fill_zero(chi[m], 2 * (int64_t)n_tau * P.NRI * P.NRI, st));
    if (P.s.n_trip == 0) continue;
    GW_HIP(filter_square_blocks(occ[m], P.dof, n_tau, P.na, NA, B.eps_f, P.dropped, st));
    GW_HIP(filter_square_blocks(vir[m], P.dvf, n_tau, P.na, NA, B.eps_f, P.dropped + nflag, st));
    if (B.prec == GW_FP32) {
      GW_HIP(to_f32_rows(P.dof, P.dof32, (int64_t)n_tau * P.N, P.N, P.ld32, st));
      GW_HIP(to_f32(P.dvf, P.dvf32, (int64_t)n_tau * P.N * P.N, st));
    } else if (B.prec == GW_BF16X3) {
      const int W = bf_width(NA);
      const int64_t dsz = (int64_t)n_tau * P.N * P.na * W;
      const unsigned blocks = (unsigned)std::min<int64_t>((dsz + 255) / 256, 1 << 20);
      hipLaunchKernelGGL(split_d_kernel, dim3(blocks), dim3(256), 0, st, P.dof, P.doh, P.dol, n_tau,
                         P.N, P.na, NA, W);
      GW_HIP(hipGetLastError());
      hipLaunchKernelGGL(split_d_kernel, dim3(blocks), dim3(256), 0, st, P.dvf, P.dvh, P.dvl, n_tau,
                         P.N, P.na, NA, W);
      GW_HIP(hipGetLastError());
    }
  }
  auto mark = [&](int piv, int k) -> hipError_t {
    return ev ? hipEventRecord((*ev)[4 * piv + k], st) : hipSuccess;
  };
  for (int piv = 0; piv < B.n_loop; ++piv) {
    int* q = B.queues + 3 * kXcds * piv;
    gw_status rc = GW_OK;
    if (B.prec == GW_FP64) {
      rc = pivot_f<double>(B, piv, pers, q, ev, st);
    } else if (B.prec == GW_FP32) {
      rc = pivot_f<float>(B, piv, pers, q, ev, st);
    } else {
      GW_HIP(mark(piv, 0));
      GW_HIP(stage_a_bf(B, piv, pers & 1, q, st));
      GW_HIP(mark(piv, 1));
      GW_HIP(stage_b_bf(B, piv, pers & 2, q + kXcds, st));
      GW_HIP(mark(piv, 2));
      GW_HIP(stage_c_bf(B, piv, pers & 4, q + 2 * kXcds, st));
      GW_HIP(mark(piv, 3));
    }
    if (rc != GW_OK) return rc;
  }
  // symmetric completion and output filter
  for (int m = 0; m < B.n_sys; ++m) {
    SysPlan& P = B.sys[m];
    if (P.s.n_trip == 0) continue;
    const size_t nflag = (size_t)n_tau * P.na * P.na;
    GW_HIP(mirror_lower_blocks(chi[m], n_tau, P.NRI, NR, st));
    if (P.keep) GW_HIP(zero_unkept_blocks(chi[m], n_tau, P.na, NR, P.keep, st));
    if (B.eps_f > 0.0 && B.out_filter)
      GW_HIP(filter_square_blocks(chi[m], chi[m], n_tau, P.na, NR, B.eps_f, P.dropped + 2 * nflag, st));
  }
  return GW_OK;
}

gw_status check_ptrs(const gw_chi_batch* B, const double* const* occ, const double* const* vir,
                     double* const* chi) {
  GW_CHECK_ARG(occ && vir && chi, "d_occ, d_vir and chi arrays must be non-null");
  for (int m = 0; m < B->n_sys; ++m)
    GW_CHECK_ARG(occ[m] && vir[m] && chi[m], "every d_occ, d_vir and chi pointer must be non-null");
  return GW_OK;
}

// One execution: eager launches, or replay of the captured graph (captured
// on first use and again whenever the pointers or the configuration change).
gw_status execute(gw_chi_batch& B, const double* const* occ, const double* const* vir,
                  double* const* chi, bool use_graph, gw_chi_stats* stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  gw_status rc;
  const bool rebind = B.c_built_variant != B.variant ||
                      !std::equal(B.bound_chi.begin(), B.bound_chi.end(), chi) ||
                      (int)B.bound_chi.size() != B.n_sys;
  if (rebind) {
    B.drop_graph();
    if ((rc = build_c_tables(B, chi, st)) != GW_OK) return rc;
  }
  const bool timing = B.timing && !use_graph;
  if (use_graph) {
    const bool same = B.gexec && B.g_variant == B.variant && B.g_persistent == B.persistent &&
                      B.g_stream == st && std::equal(B.g_occ.begin(), B.g_occ.end(), occ) &&
                      std::equal(B.g_vir.begin(), B.g_vir.end(), vir);
    if (!same) {
      B.drop_graph();
      GW_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      rc = enqueue(B, occ, vir, chi, nullptr, st);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(st, &g);
      if (rc != GW_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      GW_HIP(e);
      B.graph = g;
      GW_HIP(hipGraphInstantiate(&B.gexec, B.graph, nullptr, nullptr, 0));
      B.g_variant = B.variant;
      B.g_persistent = B.persistent;
      B.g_stream = st;
      B.g_occ.assign(occ, occ + B.n_sys);
      B.g_vir.assign(vir, vir + B.n_sys);
    }
    GW_HIP(hipGraphLaunch(B.gexec, st));
  } else {
    if (timing && B.ev.size() < 4 * (size_t)B.n_loop) {
      while (B.ev.size() < 4 * (size_t)B.n_loop) {
        hipEvent_t e;
        GW_HIP(hipEventCreate(&e));
        B.ev.push_back(e);
      }
    }
    if ((rc = enqueue(B, occ, vir, chi, timing ? &B.ev : nullptr, st)) != GW_OK) return rc;
  }

  if (stats) {
    *stats = gw_chi_stats{};
    int64_t dd = 0, dc = 0, kept = 0;
    double fa = 0.0, fb = 0.0, fc = 0.0;
    for (const SysPlan& P : B.sys) {
      const size_t nflag = (size_t)B.n_tau * P.na * P.na;
      std::vector<uint8_t> fl(3 * nflag);
      GW_HIP(hipMemcpyAsync(fl.data(), P.dropped, fl.size(), hipMemcpyDeviceToHost, st));
      GW_HIP(hipStreamSynchronize(st));
      if (P.s.n_trip > 0) {
        for (size_t i = 0; i < 2 * nflag; ++i) dd += fl[i];
        if (B.eps_f > 0.0 && B.out_filter)
          for (size_t i = 2 * nflag; i < 3 * nflag; ++i) dc += fl[i];
      }
      kept += P.G.n_kept;
      fa += P.fl_a;
      fb += P.fl_b;
      fc += P.fl_c;
    }
    GW_HIP(hipStreamSynchronize(st));
    stats->n_trip_kept = kept;
    stats->n_dblk_dropped = dd;
    stats->n_chiblk_dropped = dc;
    stats->flops_stage[0] = fa * B.n_tau;
    stats->flops_stage[1] = fb * B.n_tau;
    stats->flops_stage[2] = fc * B.n_tau;
    stats->flops_ab = (fa + fb) * B.n_tau;
    stats->flops_c = fc * B.n_tau;
    for (int k = 0; k < 3; ++k) {
      int64_t nl = 0;
      for (int piv = 0; piv < B.n_loop; ++piv)
        nl += (B.prec == GW_FP64   ? (k == 0 ? B.t64.tA.n[piv] : k == 1 ? B.t64.tB.n[piv] : B.t64.tC.n[piv])
               : B.prec == GW_FP32 ? (k == 0 ? B.t32.tA.n[piv] : k == 1 ? B.t32.tB.n[piv] : B.t32.tC.n[piv])
                                   : (k == 0 ? B.tAb.n[piv] : k == 1 ? B.tBb.n[piv] : B.tCb.n[piv])) > 0;
      stats->n_launch[k] = nl;
    }
    for (int piv = 0; timing && piv < B.n_loop; ++piv)
      for (int k = 0; k < 3; ++k) {
        float ms;
        GW_HIP(hipEventElapsedTime(&ms, B.ev[4 * piv + k], B.ev[4 * piv + k + 1]));
        stats->ms_stage[k] += ms;
      }
    stats->c_variant = B.variant;
    stats->launch_mask = B.persistent;
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return GW_OK;
}

gw_status create(int n_sys, const gw_system* systems, int n_tau, const gw_chi_opts* opts,
                 gw_chi_batch** out, hipStream_t st) {
  GW_CHECK_ARG(out != nullptr, "plan must be non-null");
  *out = nullptr;
  GW_CHECK_ARG(n_sys >= 1 && n_sys <= 65536, "n_sys must be in [1, 65536]");
  GW_CHECK_ARG(systems != nullptr, "systems must be non-null");
  GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
  const double eps_f = opts ? opts->filter_eps : 0.0;
  GW_CHECK_ARG(std::isfinite(eps_f) && eps_f >= 0.0, "filter_eps must be finite and >= 0");
  const int prec = opts ? opts->prec : GW_FP64;
  GW_CHECK_ARG(prec == GW_FP64 || prec == GW_FP32 || prec == GW_BF16X3,
               "prec must be GW_FP64, GW_FP32 or GW_BF16X3");
  gw_status rc;
  for (int m = 0; m < n_sys; ++m) {
    if ((rc = check_system(&systems[m])) != GW_OK) return rc;
    GW_CHECK_ARG(systems[m].ao_per_atom == systems[0].ao_per_atom &&
                     systems[m].ri_per_atom == systems[0].ri_per_atom,
                 "all systems of a batch must share ao_per_atom and ri_per_atom");
  }
  const int NA = systems[0].ao_per_atom, NR = systems[0].ri_per_atom;
  GW_CHECK_ARG(NR <= C_COLS, "ri_per_atom must be <= 160");
  GW_CHECK_ARG((int64_t)n_tau * NA <= (1 << 20), "n_tau * ao_per_atom too large");
  // the BF16x3 half contractions hold an atom's AO functions in one k pair
  GW_CHECK_ARG(prec != GW_BF16X3 || NA <= 16, "GW_BF16X3 needs ao_per_atom <= 16");

  std::unique_ptr<gw_chi_batch> B(new (std::nothrow) gw_chi_batch(st));
  if (!B) {
    set_error("host allocation of the plan failed");
    return GW_ERR_NOMEM;
  }
  B->n_sys = n_sys;
  B->n_tau = n_tau;
  B->NA = NA;
  B->NR = NR;
  B->RS = n_tau * NA;
  B->GB = 0;               // set by the first system (prepare_sys)
  B->ab_nb = ab_nb(NA * NR);
  B->prec = prec;
  B->eps_f = eps_f;
  B->timing = opts && opts->timing;
  B->out_filter = !(opts && opts->keep_small_blocks);
  // default tile configuration per precision (fastest measured for 13 AO / 40 RI per atom)
  // direct-to-LDS outer contraction (variant 3) when the RI block size allows
  // its 16-byte copies (always in BF16x3); else the register-staged tiles
  B->variant = variant_ok(prec, NR, 3) ? 3 : prec == GW_FP64 ? 2 : 0;
  // FP32: stage A as a grid; stage B persistent on the wide tiles, a grid on
  // the narrow ones (measured on 13/40 and 5/12 bases)
  B->persistent = prec == GW_FP32 ? (B->ab_nb == AB_NBN ? 4 : 6) : 7;
  B->sys.resize(n_sys);
  // FP32 stage A copies D^occ rows 16 bytes at a time (rows padded to four
  // floats in the plan's FP32 copy) and brick rows of NA * NR floats
  B->a_dma = prec == GW_FP32 && NR % 4 == 0;
  for (int m = 0; m < n_sys; ++m) {
    if ((rc = prepare_sys(*B, B->sys[m], &systems[m], st)) != GW_OK) return rc;
    B->max_na = std::max(B->max_na, systems[m].n_atoms);
  }
  // 16-byte copies need the brick rows (NA * NR elements) in whole groups of
  // 16 bytes (the gathered D^vir rows are padded to them, LDB), and in FP64
  // stage A the D^occ rows (N doubles; the FP32 copy is padded)
  B->b_dma = prec == GW_FP32 ? NR % 4 == 0 : prec == GW_FP64 && NR % 2 == 0;
  if (prec == GW_FP64) {
    B->a_dma = NR % 2 == 0;
    for (const SysPlan& P : B->sys) B->a_dma = B->a_dma && P.N % 2 == 0;
  }
  // BF16x3 stages A and B on the direct-to-LDS engine, whose per-lane parts
  // of the D offsets (rows tau * N + mu of na 16-entry groups) are 32-bit
  if (prec == GW_BF16X3) {
    B->bf_dma_ab = true;
    for (const SysPlan& P : B->sys)
      B->bf_dma_ab = B->bf_dma_ab && (int64_t)(n_tau + 1) * P.N * P.na * bf_width(NA) < (1ll << 32);
  }
  // largest systems first: their tiles lead every batched launch
  B->order.resize(n_sys);
  std::iota(B->order.begin(), B->order.end(), 0);
  std::stable_sort(B->order.begin(), B->order.end(), [&](int x, int y) {
    return B->sys[x].fl_c + B->sys[x].fl_a > B->sys[y].fl_c + B->sys[y].fl_a;
  });
  for (const SysPlan& P : B->sys) B->n_loop = std::max(B->n_loop, P.pair_h > 0 ? P.pair_h : P.na);
  B->n_queues = 3 * kXcds * std::max(B->n_loop, 1);
  if ((rc = B->mem.alloc(&B->queues, B->n_queues)) != GW_OK) return rc;
  if ((rc = B->mem.alloc(&B->tiles_skipped, 1)) != GW_OK) return rc;
  GW_HIP(hipMemsetAsync(B->tiles_skipped, 0, sizeof(int), st));
  // screened one-system calls: stages A and B may skip tiles that feed only
  // unkept chi blocks (the masks are set per call from the screener's keep
  // mask; everything is needed until then)
  if (n_sys == 1 && opts && opts->screener && opts->filter_eps > 0.0) {
    SysPlan& P = B->sys[0];
    if ((rc = B->mem.alloc(&P.needb, (size_t)P.na * P.na)) != GW_OK) return rc;
    if ((rc = B->mem.alloc(&P.needa, (size_t)P.na * P.na)) != GW_OK) return rc;
    GW_HIP(hipMemsetAsync(P.needb, 1, (size_t)P.na * P.na, st));
    GW_HIP(hipMemsetAsync(P.needa, 1, (size_t)P.na * P.na, st));
  }
  if ((rc = build_ab_tables(*B, st)) != GW_OK) return rc;
  B->a_dma_ok = B->a_dma;
  B->b_dma_ok = B->b_dma;
  B->bf_dma_ok = B->bf_dma_ab;
  prime(*B);
  GW_HIP(hipStreamSynchronize(st));
  *out = B.release();
  return GW_OK;
}

// shape class of a plan for the autotune cache
std::string shape_key(const gw_chi_batch& B) {
  double atoms = 0.0;
  for (const SysPlan& P : B.sys) atoms += P.na;
  atoms /= B.n_sys;
  std::ostringstream k;
  k << (B.prec == GW_FP64 ? "fp64" : B.prec == GW_FP32 ? "fp32" : "bf16x3") << "_ao" << B.NA << "_ri" << B.NR << "_tau" << B.n_tau
    << "_sys" << (int)std::lround(std::log2((double)B.n_sys)) << "_atoms"
    << (int)std::lround(2.0 * std::log2(std::max(1.0, atoms)));
  return k.str();
}

}  // namespace
}  // namespace gw

extern "C" gw_status gw_chi_batch_create(int32_t n_sys, const gw_system* systems, int32_t n_tau,
                                         const gw_chi_opts* opts, gw_chi_batch** plan,
                                         hipStream_t st) {
  clear_error();
  if (systems && n_sys >= 1 && n_sys <= 65536)
    for (int32_t m = 0; m < n_sys; ++m)
      GW_CHECK_ARG(!systems[m].ao_off && !systems[m].ri_off,
                   "batched plans take systems without per-atom offsets (use gw_contract_chi)");
  GW_CHECK_ARG(!(opts && opts->screener), "the batched form takes no screener");
  return create(n_sys, systems, n_tau, opts, plan, st);
}

extern "C" gw_status gw_chi_batch_execute(gw_chi_batch* plan, const double* const* d_occ,
                                          const double* const* d_vir, double* const* chi,
                                          int32_t use_graph, gw_chi_stats* stats, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(plan != nullptr, "plan must be non-null");
  gw_status rc = check_ptrs(plan, d_occ, d_vir, chi);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(!use_graph || st != nullptr, "graph capture needs a created (non-null) stream");
  return execute(*plan, d_occ, d_vir, chi, use_graph != 0, stats, st);
}

extern "C" gw_status gw_chi_batch_set_config(gw_chi_batch* plan, int32_t variant, int32_t persistent) {
  clear_error();
  GW_CHECK_ARG(plan != nullptr, "plan must be non-null");
  GW_CHECK_ARG(variant >= 0 && variant < kNVar, "variant out of range");
  GW_CHECK_ARG(variant_ok(plan->prec, plan->NR, variant),
               "stage-C variant 3 needs ri_per_atom a multiple of 2 (FP64) or 4 (FP32)");
  GW_CHECK_ARG(persistent >= 0 && persistent <= 7, "persistent must be a mask of bits 0..2");
  plan->variant = variant;
  plan->persistent = persistent;
  return GW_OK;
}

extern "C" gw_status gw_chi_batch_set_engine(gw_chi_batch* plan, int32_t engine) {
  clear_error();
  GW_CHECK_ARG(plan != nullptr, "plan must be non-null");
  GW_CHECK_ARG(engine == 0 || engine == 1, "engine must be 0 or 1");
  if (engine == plan->ab_engine) return GW_OK;
  plan->ab_engine = engine;
  plan->a_dma = engine == 0 && plan->a_dma_ok;
  plan->b_dma = engine == 0 && plan->b_dma_ok;
  plan->bf_dma_ab = engine == 0 && plan->bf_dma_ok;
  plan->drop_graph();
  prime(*plan);          // persistent grid sizes of the kernels now in use
  return GW_OK;
}

extern "C" gw_status gw_chi_batch_get_config(const gw_chi_batch* plan, int32_t* variant,
                                             int32_t* persistent, int32_t* n_variants) {
  clear_error();
  GW_CHECK_ARG(plan != nullptr, "plan must be non-null");
  if (variant) *variant = plan->variant;
  if (persistent) *persistent = plan->persistent;
  if (n_variants) *n_variants = kNVar;
  return GW_OK;
}

extern "C" gw_status gw_chi_batch_tune(gw_chi_batch* plan, const double* const* d_occ,
                                       const double* const* d_vir, double* const* chi, int32_t reps,
                                       const char* cache_path, double* ms_out, hipStream_t st) {
  clear_error();
  GW_CHECK_ARG(plan != nullptr, "plan must be non-null");
  gw_status rc = check_ptrs(plan, d_occ, d_vir, chi);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(reps >= 1 && reps <= 100, "reps must be in [1, 100]");
  const std::string key = shape_key(*plan);
  // cached winner of this shape class
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int v = -1, pers = -1;
      double ms = 0.0;
      if ((ls >> k >> v >> pers >> ms) && k == key && variant_ok(plan->prec, plan->NR, v) && pers >= 0 &&
          pers <= 7) {
        plan->variant = v;
        plan->persistent = pers;
        if (ms_out) *ms_out = ms;
        return GW_OK;
      }
    }
  }
  // every stage-C variant in both launch modes, stage times from HIP events;
  // each stage takes its fastest mode (A, B: over all runs; C: with its variant)
  const bool timing = plan->timing;
  plan->timing = true;
  double best_a[2] = {1e300, 1e300}, best_b[2] = {1e300, 1e300}, best_c = 1e300;
  int best_v = 0, best_pc = 0;
  for (int v = 0; v < kNVar && rc == GW_OK; ++v)
    for (int pers = 0; pers < 2 && rc == GW_OK; ++pers) {
      if (!variant_ok(plan->prec, plan->NR, v)) continue;
      plan->variant = v;
      plan->persistent = pers ? 7 : 0;
      if ((rc = execute(*plan, d_occ, d_vir, chi, false, nullptr, st)) != GW_OK) break;  // warm-up
      double ms[3] = {0.0, 0.0, 0.0};
      for (int r = 0; r < reps && rc == GW_OK; ++r) {
        gw_chi_stats sx{};
        rc = execute(*plan, d_occ, d_vir, chi, false, &sx, st);
        for (int k = 0; k < 3; ++k) ms[k] += sx.ms_stage[k] / reps;
      }
      best_a[pers] = std::min(best_a[pers], ms[0]);
      best_b[pers] = std::min(best_b[pers], ms[1]);
      if (ms[2] < best_c) {
        best_c = ms[2];
        best_v = v;
        best_pc = pers;
      }
    }
  plan->timing = timing;
  if (rc != GW_OK) return rc;
  plan->variant = best_v;
  plan->persistent = (best_a[1] < best_a[0] ? 1 : 0) | (best_b[1] < best_b[0] ? 2 : 0) | (best_pc ? 4 : 0);
  // time of the chosen configuration (whole executions, eager)
  hipEvent_t e0, e1;
  GW_HIP(hipEventCreate(&e0));
  GW_HIP(hipEventCreate(&e1));
  float total = 0.0f;
  hipError_t he = hipEventRecord(e0, st);
  for (int r = 0; r < reps && rc == GW_OK && he == hipSuccess; ++r)
    rc = execute(*plan, d_occ, d_vir, chi, false, nullptr, st);
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  if (he == hipSuccess) he = hipEventSynchronize(e1);
  if (he == hipSuccess) he = hipEventElapsedTime(&total, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != GW_OK) return rc;
  GW_HIP(he);
  const double best = total / reps;
  if (ms_out) *ms_out = best;
  if (cache_path && *cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    if (outf) {
      outf.precision(10);
      outf << key << " " << plan->variant << " " << plan->persistent << " " << best << "\n";
    }
  }
  return GW_OK;
}

extern "C" gw_status gw_chi_batch_destroy(gw_chi_batch* plan) {
  clear_error();
  delete plan;
  return GW_OK;
}

extern "C" gw_status gw_contract_chi(const gw_system* s, const double* d_occ, const double* d_vir,
                                     int32_t n_tau, const gw_chi_opts* opts, double* chi,
                                     gw_chi_stats* stats, hipStream_t st) {
  clear_error();
  const auto t_start = std::chrono::steady_clock::now();
  gw_status rc = check_system(s);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(d_occ && d_vir && chi, "d_occ, d_vir and chi must be non-null");
  if (s->ao_off || s->ri_off) {
    // per-atom sizes: the padded system (missing functions as zero functions)
    GW_CHECK_ARG(!(opts && opts->screener), "the block screener takes systems without per-atom offsets");
    GW_CHECK_ARG(n_tau >= 1 && n_tau <= 4096, "n_tau must be in [1, 4096]");
    Scratch sc(st);
    PadMaps pm;
    if ((rc = pad_maps(s, sc, pm)) != GW_OK) return rc;
    double *po, *pv, *pc;
    if ((rc = sc.alloc(&po, (size_t)n_tau * pm.N * pm.N)) != GW_OK) return rc;
    if ((rc = sc.alloc(&pv, (size_t)n_tau * pm.N * pm.N)) != GW_OK) return rc;
    if ((rc = sc.alloc(&pc, (size_t)n_tau * pm.NRI * pm.NRI)) != GW_OK) return rc;
    GW_HIP(scatter_square(d_occ, pm.n_ao, po, pm.N, pm.ao, n_tau, st));
    GW_HIP(scatter_square(d_vir, pm.n_ao, pv, pm.N, pm.ao, n_tau, st));
    const gw_system ps = padded_view(s);
    if ((rc = gw_contract_chi(&ps, po, pv, n_tau, opts, pc, stats, st)) != GW_OK) return rc;
    GW_HIP(gather_square(pc, pm.NRI, chi, pm.n_ri, pm.ri, n_tau, st));
    GW_HIP(hipStreamSynchronize(st));
    if (stats)
      stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return GW_OK;
  }
  const bool screening = opts && opts->screener && opts->filter_eps > 0.0;
  if (screening) {
    GW_CHECK_ARG(opts->screen_tau != nullptr, "screen_tau is required with a screener");
    GW_CHECK_ARG(std::isfinite(opts->screen_margin) && opts->screen_margin >= 0.0,
                 "screen_margin must be finite and >= 0");
  }
  gw_chi_batch* raw = nullptr;
  if ((rc = create(1, s, n_tau, opts, &raw, st)) != GW_OK) return rc;
  std::unique_ptr<gw_chi_batch> B(raw);
  SysPlan& P = B->sys[0];
  const int na = P.na;

  // learned screener: keep mask of the output blocks (c <= c')
  std::vector<uint8_t> keep_h;
  if (screening && s->n_trip > 0) {
    const int64_t nb = (int64_t)n_tau * na * na;
    Scratch sc(st);
    float *feat, *pred;
    if ((rc = sc.alloc(&feat, (size_t)nb * 6)) != GW_OK) return rc;
    if ((rc = sc.alloc(&pred, (size_t)nb)) != GW_OK) return rc;
    if ((rc = B->mem.alloc(&P.keep, (size_t)nb)) != GW_OK) return rc;
    if ((rc = gw_chi_block_features(s, d_occ, d_vir, n_tau, opts->screen_tau, opts->filter_eps, feat,
                                    st)) != GW_OK)
      return rc;
    if ((rc = gw_mlp_forward(opts->screener, nb, feat, pred, 1, st)) != GW_OK) return rc;
    std::vector<float> ph(nb);
    GW_HIP(hipMemcpyAsync(ph.data(), pred, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
    GW_HIP(hipStreamSynchronize(st));
    const float thr = (float)(std::log10(opts->filter_eps) - opts->screen_margin);
    keep_h.assign(nb, 0);
    for (int j = 0; j < n_tau; ++j)
      for (int c = 0; c < na; ++c)
        for (int c2 = c; c2 < na; ++c2) {
          const int64_t e = ((int64_t)j * na + c) * na + c2;
          keep_h[e] = (ph[e] >= thr) || !std::isfinite(ph[e]) ? 1 : 0;
        }
    GW_HIP(hipMemcpyAsync(P.keep, keep_h.data(), nb, hipMemcpyHostToDevice, st));
    // stage B: N_b column block c of pivot b feeds the chi blocks (c_r, c),
    // c_r an RI atom of the pivot's groups, c_r <= c (the lower ones are
    // mirrored); it is needed when one of them is kept at some tau
    if (P.needb) {
      const int nw = (na + 63) / 64;
      std::vector<uint64_t> any((size_t)na * nw, 0);       // kept at some tau, bit c2 of row c
      for (int j = 0; j < n_tau; ++j)
        for (int c = 0; c < na; ++c) {
          const uint8_t* k = &keep_h[((int64_t)j * na + c) * na];
          for (int c2 = c; c2 < na; ++c2)
            if (k[c2]) any[(size_t)c * nw + c2 / 64] |= 1ull << (c2 % 64);
        }
      std::vector<uint8_t> need_h((size_t)na * na, 0);
      std::vector<uint64_t> acc(nw);
      for (int b = 0; b < na; ++b) {
        int g0 = 0;
        const int nR = pivot_groups(P, b, g0);
        std::fill(acc.begin(), acc.end(), 0ull);
        for (int sl = 0; sl < nR; ++sl) {
          const int cr = P.G.gc[g0 + sl];
          for (int w = 0; w < nw; ++w) acc[w] |= any[(size_t)cr * nw + w];
        }
        for (int c2 = 0; c2 < na; ++c2) need_h[(size_t)b * na + c2] = (acc[c2 / 64] >> (c2 % 64)) & 1;
      }
      GW_HIP(hipMemcpyAsync(P.needb, need_h.data(), need_h.size(), hipMemcpyHostToDevice, st));
      // stage A: the M_b rows of slot atom c enter stage C as the K rows of the
      // panels that hold a kept block (c, c'), c' >= c: the AO atoms of their unions
      std::vector<uint8_t> needa_h((size_t)na * na, 0);      // [c][a]
      for (int c = 0; c < na; ++c)
        for (int p = 0; p < P.n_pan; ++p) {
          bool kept = false;
          for (int c2 = p * P.PG; c2 < std::min(na, p * P.PG + P.PG) && !kept; ++c2)
            kept = (any[(size_t)c * nw + c2 / 64] >> (c2 % 64)) & 1;
          if (!kept) continue;
          for (int j = 0; j < P.pan.ulen[p]; ++j)
            needa_h[(size_t)c * na + P.pan.kmap[P.pan.km_off[p] + j * B->NA] / B->NA] = 1;
        }
      GW_HIP(hipMemcpyAsync(P.needa, needa_h.data(), needa_h.size(), hipMemcpyHostToDevice, st));
      GW_HIP(hipStreamSynchronize(st));          // the host vectors outlive the copies
    }
    GW_HIP(hipStreamSynchronize(st));
  }
  if ((rc = execute(*B, &d_occ, &d_vir, &chi, false, stats, st)) != GW_OK) return rc;
  // audit: the exact contraction (same plan, no screener, no output filter)
  // judges every skipped block by the output filter's own FP64 decision
  gw_chi_stats audit{};
  bool audit_failed = false;
  if (screening && opts->screen_audit && !keep_h.empty()) {
    const auto t_a = std::chrono::steady_clock::now();
    const int64_t nb = (int64_t)n_tau * na * na;
    const int64_t nsq = (int64_t)P.NRI * P.NRI;
    Scratch sc(st);
    double* ex;
    float* nrm;
    uint8_t* small;
    if ((rc = sc.alloc(&ex, (size_t)n_tau * nsq)) != GW_OK) return rc;
    if ((rc = sc.alloc(&nrm, (size_t)nb)) != GW_OK) return rc;
    if ((rc = sc.alloc(&small, (size_t)nb)) != GW_OK) return rc;
    uint8_t* keep_dev = P.keep;
    const bool out_filter = B->out_filter;
    P.keep = nullptr;
    B->out_filter = false;
    // every stage-A and stage-B tile in the exact run (and a fallback after it)
    if (P.needb) GW_HIP(hipMemsetAsync(P.needb, 1, (size_t)na * na, st));
    if (P.needa) GW_HIP(hipMemsetAsync(P.needa, 1, (size_t)na * na, st));
    B->c_built_variant = -1;            // rebuild the stage-C tables without the mask
    rc = execute(*B, &d_occ, &d_vir, &ex, false, nullptr, st);
    P.keep = keep_dev;
    B->out_filter = out_filter;
    if (rc != GW_OK) return rc;
    GW_HIP(block_norms_f32(ex, n_tau, na, B->NR, 0, nrm, st));
    // small[e] = 1 for blocks the output filter zeroes (norm < filter_eps, FP64)
    GW_HIP(filter_square_blocks(ex, ex, n_tau, na, B->NR, opts->filter_eps, small, st));
    std::vector<float> nh(nb);
    std::vector<uint8_t> sh(nb);
    GW_HIP(hipMemcpyAsync(nh.data(), nrm, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
    GW_HIP(hipMemcpyAsync(sh.data(), small, nb, hipMemcpyDeviceToHost, st));
    GW_HIP(hipStreamSynchronize(st));
    double mass = 0.0, total = 0.0, mx = 0.0;
    int64_t viol = 0;
    for (int j = 0; j < n_tau; ++j)
      for (int c = 0; c < na; ++c)
        for (int c2 = 0; c2 < na; ++c2) {
          const int64_t e = ((int64_t)j * na + c) * na + c2;
          const double v = nh[e];
          total += v * v;
          const int64_t u = ((int64_t)j * na + std::min(c, c2)) * na + std::max(c, c2);
          if (keep_h[u]) continue;
          mass += v * v;
          mx = std::max(mx, v);
          if (!sh[e] && c <= c2) ++viol;
        }
    audit.audit_done = 1;
    audit.n_audit_violations = viol;
    audit.audit_max_skipped = mx;
    audit.audit_skipped_mass = total > 0.0 ? std::sqrt(mass / total) : 0.0;
    audit_failed = viol > 0;
    if (audit_failed && opts->screen_fallback) {
      // ex now holds the exact chi after the output filter: the plain result
      // (unless the caller asked to keep the small blocks)
      if (out_filter) {
        GW_HIP(hipMemcpyAsync(chi, ex, sizeof(double) * n_tau * nsq, hipMemcpyDeviceToDevice, st));
      } else {
        B->c_built_variant = -1;
        P.keep = nullptr;
        rc = execute(*B, &d_occ, &d_vir, &chi, false, nullptr, st);
        P.keep = keep_dev;
        if (rc != GW_OK) return rc;
      }
      GW_HIP(hipStreamSynchronize(st));
      audit.audit_fallback = 1;
    }
    audit.audit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
  }
  if (stats) {
    stats->audit_done = audit.audit_done;
    stats->audit_fallback = audit.audit_fallback;
    stats->n_audit_violations = audit.n_audit_violations;
    stats->audit_max_skipped = audit.audit_max_skipped;
    stats->audit_skipped_mass = audit.audit_skipped_mass;
    stats->audit_ms = audit.audit_ms;
    if (!keep_h.empty() && !audit.audit_fallback) {
      int skipped = 0;
      GW_HIP(hipMemcpyAsync(&skipped, B->tiles_skipped, sizeof(int), hipMemcpyDeviceToHost, st));
      GW_HIP(hipStreamSynchronize(st));
      stats->n_tiles_screened = skipped;
      int64_t nbs = 0;
      const int NA = B->NA, NR = B->NR;
      for (int64_t e = 0; e < (int64_t)n_tau * na * na; ++e) {
        const int c = (int)((e / na) % na), c2 = (int)(e % na);
        if (c <= c2 && !keep_h[e]) ++nbs;
      }
      stats->n_blocks_screened = nbs;
      // stage-C FLOPs of the kept blocks only: every group with RI atom c pairs
      // with the kept partners c2 >= c, each of |A(c2)| groups
      std::vector<double> kept_a((size_t)n_tau * na, 0.0);   // [j][c]: sum of |A(c2)| over kept c2
      for (int j = 0; j < n_tau; ++j)
        for (int c = 0; c < na; ++c) {
          double a = 0.0;
          const uint8_t* k = &keep_h[((int64_t)j * na + c) * na];
          for (int c2 = c; c2 < na; ++c2) a += k[c2] ? P.acount[c2] : 0;
          kept_a[(size_t)j * na + c] = a;
        }
      double fl = 0.0;
      for (int g = 0; g < P.n_groups; ++g)
        for (int j = 0; j < n_tau; ++j) fl += 2.0 * NR * NR * NA * NA * kept_a[(size_t)j * na + P.G.gc[g]];
      stats->flops_c = fl;
      stats->flops_stage[2] = fl;
    }
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (audit_failed && !audit.audit_fallback) {
    set_error("screener audit failed: " + std::to_string(audit.n_audit_violations) +
              " skipped output blocks are kept by the exact contraction's filter (largest skipped "
              "norm " + std::to_string(audit.audit_max_skipped) + ")");
    return GW_ERR_AUDIT;
  }
  return GW_OK;
}
