// FP64 / FP32 MFMA tile engine for gfx950 (CDNA4), shared by every contraction.
//
// A workgroup of WM x WN waves computes a (32*WM) x (16*NB*WN) output tile
//   C[r][c] = sum_k A(r, k) * B(k, c)
// with v_mfma_f64_16x16x4f64, or v_mfma_f32_16x16x4f32 when the problem's
// operand type P::In is float (FP32 products, FP32 accumulation; P::Out is
// the type of the output array, FP64 for an accumulated result).  Wave w owns rows [32w, 32w + 32) (two 16-row
// MFMA blocks) and all NB 16-column blocks, i.e. 2*NB accumulators of four
// doubles per lane.  K is staged through LDS in chunks of KC = 16: A as
// As[k][r], B as Bs[k][c] (both with a pad that puts consecutive k rows in
// opposite LDS bank halves).  The next chunk is prefetched into registers
// while the current one feeds the matrix cores.
//
// Index maps come from the problem type P (offsets in doubles):
//   bool tile(bx, by, bz, Tile&)        rows/cols/K of the tile; false = skip
//   void fill(const Tile&, int* ta, int* tb, tid, nthreads)
//                                       per-tile int tables in LDS (P::kTabA /
//                                       P::kTabB entries) read by the maps below
//   const double* abase(t), int64 aroff(t, r), int64 akoff(t, k, ta)
//   const double* bbase(t), int64 bkoff(t, k, tb)
//   double ascale(t, k)                 (only if P::kAScale)
// so A(r, k) = abase[aroff(r) + akoff(k)] (* ascale(k)) and
// B(k, c) = bbase[bkoff(k) + c]; entries outside rows/cols/K read as zero
// (branch-free: out-of-range lanes load element 0 and discard it).
// Operand and output types default to double (P::In, P::Out).
// Output offsets are separable, out(r, c) at rowoff(t, r) + coloff(t, c):
//   kDot == false: double* obase(t); the tile is stored (kAccum == false) or
//                  added with factor kSign to what is there (kAccum == true)
//   kDot == true:  const double* dbase0(t), dbase1(t); the tile is reduced to
//                  s0 = sum C * D0, s1 = sum C * D1, passed to dot_out(t, s0, s1)
// The LDS tables replace dependent global loads of the index arrays, and
// divisions by per-tile extents use FastDiv (multiply-high).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace gw {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// LDS row stride: consecutive k rows start 16 elements apart modulo the bank
// width (32 doubles or 64 floats), so the four k rows read by one MFMA step
// fall in different banks
template <class T>
__host__ __device__ constexpr int lds_stride(int n) {
  constexpr int w = sizeof(T) == 8 ? 32 : 64;
  return n + (16 - n % w + w) % w;
}

// operand / output element types of a problem (double unless it says otherwise)
template <class P, class = void>
struct in_type { using type = double; };
template <class P>
struct in_type<P, std::void_t<typename P::In>> { using type = typename P::In; };
template <class P, class = void>
struct out_type { using type = double; };
template <class P>
struct out_type<P, std::void_t<typename P::Out>> { using type = typename P::Out; };

// one 16x16x4 MFMA step and the accumulator / output layout of each type
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc = dbl4;
  __device__ static acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // lane l, element i -> row 4*i + l/16 (measured on gfx950), col l%16
  __device__ static int row(int i, int lk) { return 4 * i + lk; }
};
template <>
struct Mfma<float> {
  using acc = flt4;
  __device__ static acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // lane l, element i -> row 4*(l/16) + i, col l%16
  __device__ static int row(int i, int lk) { return 4 * lk + i; }
};

// q = k / d for k * d < 2^32 (the hosts that size K check this)
struct FastDiv {
  uint64_t m;   // ceil(2^32 / d), 2^32 for d = 1
  __host__ __device__ void set(uint32_t d) { m = (0x100000000ull + d - 1) / d; }
  __device__ __forceinline__ uint32_t div(uint32_t k) const { return (uint32_t)(((uint64_t)k * m) >> 32); }
};

struct TileBase {
  int rows, cols, K;
};

// Global-memory view of a pointer.  Problem descriptions reach the kernels
// through memory (batched tables), so the compiler cannot infer that their
// pointers are global and would emit flat accesses, which also count against
// the LDS wait counter; the kernels access operands through this view.
template <class T>
using gmem = T __attribute__((address_space(1)));
template <class T>
__device__ __forceinline__ gmem<T>* to_global(T* p) {
  return (gmem<T>*)p;
}

// A batched problem (one launch over the tiles of many systems) defines
// kBatched and local(t), which returns the problem of the tile's system;
// a plain problem is its own local problem.
template <class P, class = void>
struct is_batched : std::false_type {};
template <class P>
struct is_batched<P, std::void_t<decltype(P::kBatched)>> : std::true_type {};

// Optional cheaper index maps (detected):
//   P::kAStep: A(r, k) at abase[aroff(r) + akoff2(t, sg, u, ta)] with
//              k = sg * adiv(t) + u; the engine steps (sg, u) along a thread's
//              k sequence instead of dividing (when adiv(t) > NT / ROWS), and
//              all A offsets of a tile fit in 32 bits
//   P::kBLin:  B(k, c) at bbase[k * bstride(t) + c], offsets below 2^31
template <class P, class = void>
struct has_astep : std::false_type {};
template <class P>
struct has_astep<P, std::void_t<decltype(P::kAStep)>> : std::bool_constant<P::kAStep> {};
template <class P, class = void>
struct has_blin : std::false_type {};
template <class P>
struct has_blin<P, std::void_t<decltype(P::kBLin)>> : std::bool_constant<P::kBLin> {};

template <class P, class T>
__device__ __forceinline__ auto resolve(const P& p, const T& t) {
  if constexpr (is_batched<P>::value) return p.local(t);
  else return p;
}

// One system of a batched launch: its problem and the extents (gx, gy) of
// the 3D grid it would be launched with on its own.
template <class P>
struct BatchEntry {
  P p;
  int gx, gy;
};

// Concatenated work of several systems in one 1D launch: work item w belongs
// to entry s with tile_off[s] <= w < tile_off[s + 1] (binary search) and is
// block (bx, by, bz) of that entry's own grid, l = w - tile_off[s] =
// bx + gx * (by + gy * bz).
template <class P>
struct Batched : P {
  static constexpr bool kBatched = true;
  struct Tile : P::Tile {
    int sys;
  };
  const BatchEntry<P>* ent;
  const int32_t* tile_off;
  int n_sys;
  __device__ bool tile(int w, int, int, Tile& t) const {
    int lo = 0, hi = n_sys;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tile_off[mid] <= w) lo = mid;
      else hi = mid;
    }
    t.sys = lo;
    const int gx = ent[lo].gx, gy = ent[lo].gy;
    const int l = w - tile_off[lo], r = l / gx;
    return ent[lo].p.tile(l - r * gx, r % gy, r / gy, t);
  }
  __device__ P local(const Tile& t) const { return ent[t.sys].p; }
};

template <int WM, int WN, int NB, int KC, class P>
__device__ __forceinline__ void tile_gemm_body(const P& p, int bx, int by, int bz) {
  using TI = typename in_type<P>::type;
  using TO = typename out_type<P>::type;
  using MF = Mfma<TI>;
  constexpr int ROWS = 32 * WM, COLS = 16 * NB * WN, NT = 64 * WM * WN;
  constexpr int AST = lds_stride<TI>(ROWS), BST = lds_stride<TI>(COLS);
  constexpr int KSTEP = NT / ROWS;                    // k rows of A per pass of the threads
  constexpr int APT = KC / KSTEP;
  constexpr int BPT = (KC * COLS + NT - 1) / NT;
  static_assert(NT % ROWS == 0 && KC % KSTEP == 0, "A staging layout");
  __shared__ TI As[KC * AST];
  __shared__ TI Bs[KC * BST];
  __shared__ int tabA[P::kTabA > 0 ? P::kTabA : 1];
  __shared__ int tabB[P::kTabB > 0 ? P::kTabB : 1];

  typename P::Tile t;
  if (!p.tile(bx, by, bz, t)) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const auto lp = resolve(p, t);
  lp.fill(t, tabA, tabB, tid, NT);
  __syncthreads();
  const gmem<const TI>* __restrict__ abase = to_global(lp.abase(t));
  const gmem<const TI>* __restrict__ bbase = to_global(lp.bbase(t));

  // this thread's A row is fixed: r = tid % ROWS, k = tid / ROWS + KSTEP i
  constexpr bool ASTEP = has_astep<P>::value, BLIN = has_blin<P>::value;
  const int ar = tid % ROWS;
  const bool arow_ok = ar < t.rows;
  const int64_t aro = arow_ok ? lp.aroff(t, ar) : 0;
  const int ak0 = tid / ROWS;

  // Wave-uniform index maps.  When ROWS is a multiple of 64 a wave loads 64
  // consecutive rows of one k, so the k sequence (and the k part of every A
  // offset) is the same for all its lanes; lane j computes the offset of
  // element j and every lane reads them back (readlane).  Likewise, when
  // COLS is a multiple of 64 (and B is not linear), B is loaded in slots of
  // 64 consecutive columns of one k row.
  constexpr bool AUNI = ASTEP && ROWS % 64 == 0;
  constexpr int NW = NT / 64, CSL = COLS / 64;
  constexpr bool BUNI = !BLIN && COLS % 64 == 0;
  constexpr int BPTU = BUNI ? (KC * CSL + NW - 1) / NW : 1;
  constexpr int NB_ = BUNI ? BPTU : BPT;    // B elements per thread
  // this thread's B elements (k row, column) are the same in every chunk
  int bkl[NB_], bcc[NB_];
  uint32_t bstat = 0u;       // element i inside the chunk and the tile's columns
  uint32_t bin = 0u;         // element i inside the chunk (it has an LDS slot)
#pragma unroll
  for (int i = 0; i < NB_; ++i) {
    int kl, c;
    if constexpr (BUNI) {
      const int sl = wave + NW * i;
      kl = sl / CSL;
      c = (sl % CSL) * 64 + lane;
    } else {
      const int e = tid + i * NT;
      kl = e / COLS;
      c = e % COLS;
    }
    bkl[i] = kl < KC ? kl : KC - 1;
    bcc[i] = c;
    bstat |= (kl < KC && c < t.cols) ? (1u << i) : 0u;
    bin |= kl < KC ? (1u << i) : 0u;
  }
  int adiv = 1, sgmax = 0;
  FastDiv afd{};
  if constexpr (ASTEP) {
    adiv = lp.adiv(t);
    afd.set((uint32_t)adiv);
    sgmax = (t.K - 1) / adiv;
  }
  int bstr = 0;
  if constexpr (BLIN) bstr = lp.bstride(t);

  TI ra[APT], rbv[NB_];
  TI ascl[P::kAScale ? APT : 1];
  uint32_t amask = 0u, bmask = 0u;
  const int kmax = t.K - 1;
  auto load = [&](int k0) {
    // offsets for a clamped k first (no branches, table reads batched), then the loads
    int64_t aoff[APT], boff[NB_];
    if constexpr (AUNI) {
      const int kw = __builtin_amdgcn_readfirstlane(k0 + ak0);
      int kj = kw + KSTEP * (lane < APT ? lane : 0);
      kj = kj < kmax ? kj : kmax;
      const int sgj = (int)afd.div((uint32_t)kj);
      const int offj = (int)lp.akoff2(t, sgj < sgmax ? sgj : sgmax, kj - sgj * adiv, tabA);
#pragma unroll
      for (int i = 0; i < APT; ++i) aoff[i] = (uint32_t)__builtin_amdgcn_readlane(offj, i);
    } else if constexpr (ASTEP) {
      const int ks = k0 + ak0 < kmax ? k0 + ak0 : kmax;
      int sg = (int)afd.div((uint32_t)ks), u = ks - sg * adiv;
#pragma unroll
      for (int i = 0; i < APT; ++i) {
        aoff[i] = (uint32_t)lp.akoff2(t, sg < sgmax ? sg : sgmax, u, tabA);
        if (adiv > KSTEP) {       // uniform: at most one wrap per step
          u += KSTEP;
          const bool w = u >= adiv;
          u -= w ? adiv : 0;
          sg += w ? 1 : 0;
        } else {
          const int k = k0 + ak0 + KSTEP * (i + 1);
          const int kc = k < kmax ? k : kmax;
          sg = (int)afd.div((uint32_t)kc);
          u = kc - sg * adiv;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < APT; ++i) {
        const int k = k0 + ak0 + KSTEP * i;
        aoff[i] = lp.akoff(t, k < kmax ? k : kmax, tabA);
      }
    }
    if constexpr (BUNI) {
      // lane j: offset of the k row of slot j (uniform over the slot's 64 lanes)
      const int slj = wave + NW * (lane < NB_ ? lane : 0);
      const int klj = slj / CSL;
      int kj = k0 + (klj < KC ? klj : KC - 1);
      kj = kj < kmax ? kj : kmax;
      const int64_t offj = lp.bkoff(t, kj, tabB);
      const int lo = (int)(uint32_t)offj, hi = (int)(offj >> 32);
#pragma unroll
      for (int i = 0; i < NB_; ++i) {
        const uint32_t l32 = (uint32_t)__builtin_amdgcn_readlane(lo, i);
        const uint32_t h32 = (uint32_t)__builtin_amdgcn_readlane(hi, i);
        boff[i] = (int64_t)(((uint64_t)h32 << 32) | l32) + bcc[i];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NB_; ++i) {
        if constexpr (BLIN) {
          boff[i] = (uint32_t)((k0 + bkl[i]) * bstr + bcc[i]);
        } else {
          const int k = k0 + bkl[i];
          boff[i] = lp.bkoff(t, k < kmax ? k : kmax, tabB) + bcc[i];
        }
      }
    }
    // raw values now; out-of-range entries are zeroed at stash time so that
    // nothing waits on these loads before the matrix-core work of this chunk
    amask = 0u;
    bmask = 0u;
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int k = k0 + ak0 + KSTEP * i;
      const bool ok = arow_ok && k < t.K;
      amask |= ok ? (1u << i) : 0u;
      if constexpr (ASTEP) ra[i] = abase[ok ? (uint32_t)(aro + aoff[i]) : 0u];
      else ra[i] = abase[ok ? aro + aoff[i] : 0];
      if constexpr (P::kAScale) ascl[i] = lp.ascale(t, k < kmax ? k : kmax);
    }
#pragma unroll
    for (int i = 0; i < NB_; ++i) {
      const bool ok = ((bstat >> i) & 1u) && k0 + bkl[i] < t.K;
      bmask |= ok ? (1u << i) : 0u;
      if constexpr (BLIN) rbv[i] = bbase[ok ? (uint32_t)boff[i] : 0u];
      else rbv[i] = bbase[ok ? boff[i] : 0];
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      TI v = ra[i];
      if constexpr (P::kAScale) v *= ascl[i];
      As[(ak0 + KSTEP * i) * AST + ar] = ((amask >> i) & 1u) ? v : TI(0);
    }
#pragma unroll
    for (int i = 0; i < NB_; ++i)
      if ((bin >> i) & 1u) Bs[bkl[i] * BST + bcc[i]] = ((bmask >> i) & 1u) ? rbv[i] : TI(0);
  };

  typename MF::acc acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = typename MF::acc{0, 0, 0, 0};

  const int nch = (t.K + KC - 1) / KC;
  load(0);
  stash();
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) load((ch + 1) * KC);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int krow = 4 * kk + lk;
      const TI a0 = As[krow * AST + wm * 32 + lr];
      const TI a1 = As[krow * AST + wm * 32 + 16 + lr];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const TI b = Bs[krow * BST + (wn * NB + cb) * 16 + lr];
        acc[0][cb] = MF::step(a0, b, acc[0][cb]);
        acc[1][cb] = MF::step(a1, b, acc[1][cb]);
      }
    }
    __syncthreads();
    if (ch + 1 < nch) {
      stash();
      __syncthreads();
    }
  }

  int64_t ro[2][4];
  bool rv[2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 32 + rb * 16 + MF::row(i, lk);
      rv[rb][i] = r < t.rows;
      ro[rb][i] = rv[rb][i] ? lp.rowoff(t, r) : 0;
    }
  if constexpr (!P::kDot) {
    gmem<TO>* __restrict__ ob = to_global(lp.obase(t));
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = (wn * NB + cb) * 16 + lr;
      const bool cv = c < t.cols;
      const int64_t co = cv ? lp.coloff(t, c) : 0;
      if constexpr (P::kAccum) {
        TO old[2][4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) old[rb][i] = ob[(rv[rb][i] && cv) ? ro[rb][i] + co : 0];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rv[rb][i] && cv) ob[ro[rb][i] + co] = old[rb][i] + (TO)P::kSign * (TO)acc[rb][cb][i];
      } else {
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (rv[rb][i] && cv) ob[ro[rb][i] + co] = (TO)acc[rb][cb][i];
      }
    }
  } else {
    const gmem<const double>* __restrict__ d0 = to_global(lp.dbase0(t));
    const gmem<const double>* __restrict__ d1 = to_global(lp.dbase1(t));
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = (wn * NB + cb) * 16 + lr;
      const bool cv = c < t.cols;
      const int64_t co = cv ? lp.coloff(t, c) : 0;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool ok = rv[rb][i] && cv;
          const int64_t e = ok ? ro[rb][i] + co : 0;
          const double x0 = d0[e], x1 = d1[e];
          s0 += ok ? (double)acc[rb][cb][i] * x0 : 0.0;
          s1 += ok ? (double)acc[rb][cb][i] * x1 : 0.0;
        }
    }
    // fixed-order block reduction (deterministic)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
    }
    constexpr int NW = WM * WN;
    __shared__ double red[2 * NW];
    if (lane == 0) {
      red[wave] = s0;
      red[NW + wave] = s1;
    }
    __syncthreads();
    if (tid == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < NW; ++w) {
        t0 += red[w];
        t1 += red[NW + w];
      }
      lp.dot_out(t, t0, t1);
    }
  }
}

// XCD-aware block order.  The dispatcher hands workgroup b (linear id over
// x, then y, then z) to XCD b mod 8, and each XCD has its own L2.  Block b is
// given tile number xcd_tile(b): XCD x works through the x-th contiguous
// eighth of the tiles in order, so neighbouring tiles, which share operand
// rows or panels, meet in the same L2.  A bijection on [0, n) for any n.
constexpr int kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t q = n / kXcds, r = n % kXcds, x = b % kXcds, l = b / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}
__device__ __forceinline__ void grid_tile(int& bx, int& by, int& bz) {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t t = xcd_tile(b, gx * gy * gridDim.z);
  bx = (int)(t % gx);
  by = (int)((t / gx) % gy);
  bz = (int)(t / (gx * gy));
}

template <int WM, int WN, int NB, int KC, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_gemm_kernel(P p) {
  int bx, by, bz;
  grid_tile(bx, by, bz);
  tile_gemm_body<WM, WN, NB, KC>(p, bx, by, bz);
}

// Persistent form: a grid sized to the resident capacity takes work items
// 0 .. n_work-1 from kXcds queues (atomic counters queue[0..7], zero at
// launch), one per contiguous eighth of the items.  A workgroup starts on the
// queue of its own XCD (blockIdx.x mod 8, the dispatcher's round-robin), so
// neighbouring items share an L2, and then helps the other queues in turn;
// it leaves once every counter has passed its range, so every item is taken
// exactly once and every workgroup exits.
template <int WM, int WN, int NB, int KC, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_gemm_persistent(P p, int n_work, int* queue) {
  __shared__ int next;
  const uint32_t q = (uint32_t)n_work / kXcds, r = (uint32_t)n_work % kXcds;
  const uint32_t home = blockIdx.x % kXcds;
  for (uint32_t j = 0; j < kXcds; ++j) {
    const uint32_t x = (home + j) % kXcds;
    const int start = (int)(x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q);
    const int len = (int)(x < r ? q + 1 : q);
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) next = atomicAdd(queue + x, 1);
      __syncthreads();
      const int l = next;
      if (l >= len) break;
      tile_gemm_body<WM, WN, NB, KC>(p, start + l, 0, 0);
    }
  }
}

template <int WM, int WN, int NB, int KC, class P>
inline hipError_t launch_tile_gemm(const P& p, dim3 grid, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_gemm_kernel<WM, WN, NB, KC, P>), grid, dim3(64 * WM * WN), 0, st, p);
  return hipGetLastError();
}

// resident workgroups of a kernel on the whole device (persistent grid size)
template <class K>
inline int resident_groups(K kernel, int threads) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) return 0;
  return ncu * (per > 0 ? per : 1);
}

// grid of the persistent form: the resident capacity (computed once per
// kernel; call it outside graph capture before the first launch)
template <int WM, int WN, int NB, int KC, class P>
inline int persistent_cap_gemm() {
  static int cap = 0;
  if (cap == 0) cap = resident_groups(tile_gemm_persistent<WM, WN, NB, KC, P>, 64 * WM * WN);
  return cap;
}

template <int WM, int WN, int NB, int KC, class P>
inline hipError_t launch_tile_gemm_persistent(const P& p, int n_work, int* queue, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  const int cap = persistent_cap_gemm<WM, WN, NB, KC, P>();
  const int grid = cap > 0 ? (n_work < cap ? n_work : cap) : n_work;
  hipLaunchKernelGGL((tile_gemm_persistent<WM, WN, NB, KC, P>), dim3(grid), dim3(64 * WM * WN), 0, st,
                     p, n_work, queue);
  return hipGetLastError();
}

}  // namespace gw
