// Direct-to-LDS form of the tile engine for problems whose A offsets step in k
// (kAStep): the outer contraction of chi (B a linear panel, kBLin) and the
// D^vir half contraction (B rows gathered from the bricks through a table).
//
// The register-staged engine (tile_gemm.hpp) loads each K chunk into
// registers, waits, and writes it to LDS; its prefetch registers, their
// addresses and the unrolled operand reads put an FP64 128 x 160 tile at ~200
// VGPRs, one workgroup per CU.  Here the load units copy global memory
// straight into LDS (global_load_lds, 16 bytes per lane), S chunks deep, so no
// operand passes through registers and two workgroups fit on a CU.
//
// Layout of one stage: A chunk [KC][ROWS], B chunk [KC][COLS], both without
// padding; k row k of width W is stored rotated (element e at position
// (e + rot(k)) mod W) with rot(k) = (16 (k mod G) - k W) mod BW, BW the bank
// width in elements (32 doubles, 64 floats) and G = BW / 16: the k rows read
// by one matrix-core step then start 16 elements apart modulo the bank
// width, in different LDS banks, as the padded rows of the register-staged
// engine do.  A copy instruction fills 64 * EPL
// consecutive LDS elements (EPL = 16 bytes / element size); each lane fetches
// the EPL global elements that the rotation places at its position, which
// are consecutive in global memory as long as ROWS / COLS and the problem's
// row blocks are multiples of EPL (the host checks NR % EPL == 0).
//
// Rows and columns outside the tile are copied from a clamped valid address
// (they only reach outputs that are not stored); K rows past t.K are copied
// from row K - 1 and zeroed in the A operand of the last chunk.
#pragma once

#include "tile_gemm.hpp"

namespace gw {

// s_waitcnt with vmcnt(n) (n < 16) and no wait on the other counters
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// Workgroup barrier without the memory fence of __syncthreads (whose release
// waits for every outstanding load, here the copies of the chunks ahead).
// The waits the pipeline needs are explicit (wait_vm); LDS needs no cache
// maintenance; the empty asm statements keep the compiler from moving LDS
// accesses across the barrier.
__device__ __forceinline__ void stage_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int WM, int WN, int NB, int KC, int S, class P>
__device__ __forceinline__ void tile_dma_body(const P& p, int bx, int by, int bz) {
  using TI = typename in_type<P>::type;
  using TO = typename out_type<P>::type;
  using MF = Mfma<TI>;
  static_assert(has_astep<P>::value, "direct-to-LDS form needs kAStep");
  constexpr bool BLIN = has_blin<P>::value;
  constexpr int ROWS = 32 * WM, COLS = 16 * NB * WN, NT = 64 * WM * WN, NW = NT / 64;
  constexpr int EPL = 16 / (int)sizeof(TI), PER = 64 * EPL;
  constexpr int ACH = KC * ROWS, BCH = KC * COLS;
  constexpr int NCA = ACH / PER, NCB = BCH / PER;                   // copies per chunk
  // copies per wave: JA of A then JB of B, the same count on every wave (a
  // wave with fewer repeats its operand's last copy: same cells, same data)
  constexpr int JA = (NCA + NW - 1) / NW, JB = (NCB + NW - 1) / NW, CPW = JA + JB;
  constexpr int BW = sizeof(TI) == 8 ? 32 : 64, G = BW / 16;
  auto rot = [](int k, int w) { return ((16 * (k % G) - (k * w) % BW) % BW + BW) % BW; };
  static_assert(ACH % PER == 0 && BCH % PER == 0 && ROWS % 16 == 0 && COLS % 16 == 0, "copy layout");
  static_assert(KC % 4 == 0 && (S == 2 || S == 3) && CPW * (S - 2) < 16, "pipeline shape");
  // one LDS array per stage and operand (see the main loop)
  __shared__ __attribute__((aligned(16))) TI As0[ACH];
  __shared__ __attribute__((aligned(16))) TI As1[ACH];
  __shared__ __attribute__((aligned(16))) TI As2[S > 2 ? ACH : EPL];
  __shared__ __attribute__((aligned(16))) TI Bs0[BCH];
  __shared__ __attribute__((aligned(16))) TI Bs1[BCH];
  __shared__ __attribute__((aligned(16))) TI Bs2[S > 2 ? BCH : EPL];
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
  const int adiv = lp.adiv(t);
  int bstr = 0;
  if constexpr (BLIN) bstr = lp.bstride(t);
  const int kmax = t.K - 1;
  FastDiv afd{};
  afd.set((uint32_t)adiv);
  const int sgmax = kmax / adiv;

  // copies of this wave: A copy c = wave + NW * j (j < JA), B copy
  // c = wave + NW * (j - JA) (j >= JA), each clamped to its operand's last;
  // for each, the k row inside the chunk, the LDS offset inside the stage and
  // the lane's fixed part of the global offset (A: row offset; B: k row *
  // stride + column for a linear panel, the column for a gathered one)
  int ck[CPW], cl[CPW];
  uint32_t cg[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const bool isb = j >= JA;
    const int n = isb ? NCB : NCA, cj = wave + NW * (isb ? j - JA : j);
    const int c = cj < n ? cj : n - 1;
    const int e = c * PER + lane * EPL;                       // element of the chunk
    const int width = isb ? COLS : ROWS;
    const int k = e / width, pos = e % width;
    int x = pos - rot(k, width);
    x += x < 0 ? width : 0;                                   // row / column in the tile
    ck[j] = k;
    cl[j] = c * PER;
    if (isb) {
      cg[j] = (uint32_t)((BLIN ? k * bstr : 0) + (x < t.cols ? x : 0));
    } else {
      cg[j] = x < t.rows ? (uint32_t)lp.aroff(t, x) : (uint32_t)lp.aroff(t, 0);
    }
  }
  // the copies of chunk ch (k clamped: chunks past the end copy the last k row)
  auto issue = [&](int ch, TI* adst, TI* bdst) {
    const int k0 = ch * KC;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      int k = k0 + ck[j];
      k = k < kmax ? k : kmax;
      if (j >= JA) {
        const gmem<const TI>* g;
        if constexpr (BLIN) g = bbase + (cg[j] + (uint32_t)((k - ck[j]) * bstr));
        else g = bbase + (lp.bkoff(t, k, tabB) + cg[j]);
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                         (void __attribute__((address_space(3)))*)(bdst + cl[j]),
                                         16, 0, 0);
      } else {
        const int sg = (int)afd.div((uint32_t)k), u = k - sg * adiv;
        const uint32_t ko = lp.akoff2(t, sg < sgmax ? sg : sgmax, u, tabA);
        const gmem<const TI>* g = abase + (cg[j] + ko);
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                         (void __attribute__((address_space(3)))*)(adst + cl[j]),
                                         16, 0, 0);
      }
    }
  };

  typename MF::acc acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = typename MF::acc{0, 0, 0, 0};

  // LDS offsets of this lane's operands inside a stage (k row 4 kk + lk has
  // the rotation of row lk: 4 kk W is a multiple of the bank width)
  const int lr = lane & 15, lk = lane >> 4, ra = rot(lk, ROWS), rbo = rot(lk, COLS);
  const int a0o = lk * ROWS + ((wm * 32 + lr + ra) % ROWS);
  const int a1o = lk * ROWS + ((wm * 32 + 16 + lr + ra) % ROWS);
  int bo[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) bo[cb] = lk * COLS + (((wn * NB + cb) * 16 + lr + rbo) % COLS);

  const int nch = (t.K + KC - 1) / KC;
  // One chunk: this wave's copies of chunk ch have landed (those of the
  // chunks after it may still be in flight), then every wave's have and the
  // stage of chunk ch - 1 is free: the copies of chunk ch + S - 1 go there,
  // and the matrix cores take chunk ch.
  auto chunk = [&](int ch, TI* adst, TI* bdst, const TI* as, const TI* bs) {
    wait_vm<CPW * (S - 2)>();
    stage_barrier();
    issue(ch + S - 1, adst, bdst);
    const int kv = t.K - ch * KC;            // valid k rows of this chunk
    if (kv >= KC) {
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        const TI a0 = as[kk * 4 * ROWS + a0o];
        const TI a1 = as[kk * 4 * ROWS + a1o];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const TI b = bs[kk * 4 * COLS + bo[cb]];
          acc[0][cb] = MF::step(a0, b, acc[0][cb]);
          acc[1][cb] = MF::step(a1, b, acc[1][cb]);
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KC / 4; ++kk) {
        const bool ok = 4 * kk + lk < kv;
        const TI a0 = ok ? as[kk * 4 * ROWS + a0o] : TI(0);
        const TI a1 = ok ? as[kk * 4 * ROWS + a1o] : TI(0);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const TI b = bs[kk * 4 * COLS + bo[cb]];
          acc[0][cb] = MF::step(a0, b, acc[0][cb]);
          acc[1][cb] = MF::step(a1, b, acc[1][cb]);
        }
      }
    }
  };
  // Every access names its stage array (the loop is unrolled by S), and the
  // copies are issued without branches, the same number on every wave: the
  // compiler then sees that the copies in flight write other stages than
  // the one read, and does not wait for all of them before each LDS read
  // (which would serialize the copies with the matrix cores).  The waits
  // the pipeline needs are the explicit ones at the top of each chunk.
  issue(0, As0, Bs0);
  int c0 = 0;
  if constexpr (S == 2) {
    for (; c0 + 2 <= nch; c0 += 2) {
      chunk(c0, As1, Bs1, As0, Bs0);
      chunk(c0 + 1, As0, Bs0, As1, Bs1);
    }
    if (c0 < nch) chunk(c0, As1, Bs1, As0, Bs0);
  } else {
    issue(1, As1, Bs1);
    for (; c0 + 3 <= nch; c0 += 3) {
      chunk(c0, As2, Bs2, As0, Bs0);
      chunk(c0 + 1, As0, Bs0, As1, Bs1);
      chunk(c0 + 2, As1, Bs1, As2, Bs2);
    }
    if (c0 < nch) chunk(c0, As2, Bs2, As0, Bs0);
    if (c0 + 1 < nch) chunk(c0 + 1, As0, Bs0, As1, Bs1);
  }
  wait_vm<0>();                              // no copy of a past-the-end chunk outlives the tile

  // epilogue one 16-row block at a time (keeps the live registers of the
  // accumulators, row offsets and old values within the occupancy budget)
  gmem<TO>* __restrict__ ob = to_global(lp.obase(t));
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    int64_t ro[4];
    bool rv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 32 + rb * 16 + MF::row(i, lk);
      rv[i] = r < t.rows;
      ro[i] = rv[i] ? lp.rowoff(t, r) : 0;
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int c = (wn * NB + cb) * 16 + lr;
      const bool cv = c < t.cols;
      const int64_t co = cv ? lp.coloff(t, c) : 0;
      if constexpr (P::kAccum) {
        TO old[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) old[i] = ob[(rv[i] && cv) ? ro[i] + co : 0];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rv[i] && cv) ob[ro[i] + co] = old[i] + (TO)P::kSign * (TO)acc[rb][cb][i];
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rv[i] && cv) ob[ro[i] + co] = (TO)acc[rb][cb][i];
      }
    }
  }
}

template <int WM, int WN, int NB, int KC, int S, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_dma_kernel(P p) {
  int bx, by, bz;
  grid_tile(bx, by, bz);
  tile_dma_body<WM, WN, NB, KC, S>(p, bx, by, bz);
}

// persistent form: the work queues of tile_gemm_persistent
template <int WM, int WN, int NB, int KC, int S, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_dma_persistent(P p, int n_work, int* queue) {
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
      tile_dma_body<WM, WN, NB, KC, S>(p, start + l, 0, 0);
    }
  }
}

template <int WM, int WN, int NB, int KC, int S, class P>
inline hipError_t launch_tile_dma(const P& p, dim3 grid, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_dma_kernel<WM, WN, NB, KC, S, P>), grid, dim3(64 * WM * WN), 0, st, p);
  return hipGetLastError();
}

template <int WM, int WN, int NB, int KC, int S, class P>
inline int persistent_cap_dma() {
  static int cap = 0;
  if (cap == 0) cap = resident_groups(tile_dma_persistent<WM, WN, NB, KC, S, P>, 64 * WM * WN);
  return cap;
}

template <int WM, int WN, int NB, int KC, int S, class P>
inline hipError_t launch_tile_dma_persistent(const P& p, int n_work, int* queue, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  const int cap = persistent_cap_dma<WM, WN, NB, KC, S, P>();
  const int grid = cap > 0 ? (n_work < cap ? n_work : cap) : n_work;
  hipLaunchKernelGGL((tile_dma_persistent<WM, WN, NB, KC, S, P>), dim3(grid), dim3(64 * WM * WN), 0, st,
                     p, n_work, queue);
  return hipGetLastError();
}

}  // namespace gw
