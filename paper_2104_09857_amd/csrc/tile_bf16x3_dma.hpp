// Direct-to-LDS form of the split-precision (BF16 x 3) engine, for the three
// stages of chi.
//
// The register-staged engine (tile_bf16x3.hpp) keeps one K chunk in flight:
// it loads the next chunk into registers while the current one feeds the
// matrix cores, so each 32-deep chunk (about 1900 matrix-core cycles per SIMD
// on a 256 x 160 tile) must hide a whole global-memory round trip, and it
// waits at two barriers per chunk.  Here the load units copy the operands
// straight into LDS (global_load_lds, 16 bytes per lane), S chunks deep,
// with one barrier per chunk; the per-tile LDS table of panel offsets is
// replaced by wave-uniform (scalar) reads of the index array, which leaves
// room for three stages of a 256 x 160 tile.
//
// Operands (bf16 hi and lo arrays, same offsets) are addressed by k pairs:
// pair u holds 16 consecutive k values (two 16-byte groups) of a row:
//   A(r, 16 u + j) at abase + arow(r) + a_tab[u] * a_mul + j
//   B(16 u + j, c) at bbase + bcs c + b_tab[u] * b_mul + j      (bf16 units)
// with 16 u < t.K, and b_tab[u] * b_mul replaced by b_pairoff(u) unless the
// problem has a B table (P::kBTab, 64-bit entries).  In the half-select
// instance (HS = 1, tables of 8-wide segments) half h of pair u comes from
// entry 2 u + h instead: A(r, 16 u + 8 h + j) at abase + arow(r) +
// a_tab[2 u + h] * a_mul + j (j < 8), and B alike.  The tables are read with
// scalar loads (their addresses and u are wave-uniform), which do not count
// against the vector-memory counter that tracks the copies in flight.  The
// output is added to an FP64 array (P::kOut == 0) or stored split into bf16
// hi / lo arrays (P::kOut == 1), at rowoff(r) + coloff(c) (or outoff(r, c)).
// One LDS stage holds, per array, [KC / 16][ROWS][2] (A) and
// [KC / 16][COLS][2] (B) cells of 16 bytes; the two cells of a row
// and pair are swapped when bit 2 of the row is set, so the 16 rows read by
// one quarter of a wave fall on distinct banks.  A copy instruction fills 64
// consecutive cells (32 rows of one pair); each lane fetches the cell the
// swap places at its position, so a copy reads 32 whole 32-byte row pieces.
//
// The matrix-core steps, the k values of each lane and the order of every
// sum are those of the register-staged engine: results are bit-identical.
// Rows and columns outside the tile are copied from clamped valid addresses
// (their outputs are not stored); pairs past the end are copied from the
// last pair and their A values are zeroed when read.
#pragma once

#include "tile_bf16x3.hpp"
#include "tile_dma.hpp"

namespace gw {

template <class P, class = void>
struct has_btab : std::false_type {};
template <class P>
struct has_btab<P, std::void_t<decltype(P::kBTab)>> : std::bool_constant<P::kBTab> {};

// wave-uniform pointer in the constant address space (scalar loads)
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* scalar_view(const T* p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const __attribute__((address_space(4))) T*)(((uint64_t)hi << 32) | lo);
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
__device__ __forceinline__ void tile_bf3_dma_body(const P& p, int bx, int by, int bz) {
  constexpr int ROWS = 16 * RB * WM, COLS = 16 * NB * WN, NT = 64 * WM * WN, NW = NT / 64;
  constexpr int KC = 32, NP = KC / 16;                       // k pairs per chunk
  constexpr int AC = NP * ROWS * 2, BC = NP * COLS * 2;      // cells per array per stage
  constexpr int SC = 2 * AC + 2 * BC;                        // cells per stage
  constexpr int NCA = AC / 64, NCB = BC / 64;                // copies per array
  constexpr int NC = 2 * NCA + 2 * NCB, CPW = (NC + NW - 1) / NW;
  constexpr bool BTAB = has_btab<P>::value;
  static_assert(ROWS % 32 == 0 && COLS % 32 == 0 && NC >= NW, "copy layout");
  static_assert((S == 2 || S == 3) && CPW * (S - 2) < 16, "two or three stages; vmcnt immediate");
  __shared__ __attribute__((aligned(16))) u32x4_t L0[SC];
  __shared__ __attribute__((aligned(16))) u32x4_t L1[SC];
  __shared__ __attribute__((aligned(16))) u32x4_t L2[S > 2 ? SC : 1];

  typename P::Tile t;
  if (!p.tile(bx, by, bz, t)) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const auto lp = resolve(p, t);
  // K is a multiple of 8; a pair's two halves are table entry u, 8 apart
  // (HS == 0), or entries 2u and 2u + 1, each 8 wide (HS == 1)
  const int npairs = (t.K + 15) / 16, pmax = npairs - 1;
  const int emax = (HS ? t.K / 8 : t.K / 16) - 1;        // last table entry
  // the pair tables through the scalar (constant) path
  const auto atab = scalar_view(lp.a_tab(t));
  const __attribute__((address_space(4))) int64_t* btab = nullptr;
  if constexpr (BTAB) btab = scalar_view(lp.b_tab(t));
  const uint32_t amul = __builtin_amdgcn_readfirstlane(lp.a_mul());
  int64_t bmul = 0;
  if constexpr (BTAB) bmul = (int64_t)__builtin_amdgcn_readfirstlane(lp.b_mul());
  const int bcs = lp.bcs();

  // copies of this wave: copy c = wave + NW * j over [A hi | A lo | B hi | B lo];
  // for each, its array, its pair inside the chunk, the cell offset inside
  // the stage and the lane's fixed part of the global offset
  const gmem<const uint16_t>* cbase[CPW];
  bool cisb[CPW];
  int cpair[CPW], ccell[CPW];
  bool chalf[CPW];    // the lane's half (HS == 1 only)
  uint32_t clane[CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + NW * j < NC ? wave + NW * j : NC - 1;
    const int arr = c < NCA ? 0 : c < 2 * NCA ? 1 : c < 2 * NCA + NCB ? 2 : 3;
    const int cc = arr == 0 ? c : arr == 1 ? c - NCA : arr == 2 ? c - 2 * NCA : c - 2 * NCA - NCB;
    const bool isb = arr >= 2;
    const int width = isb ? COLS : ROWS;
    const int e = cc * 64 + lane;                            // cell inside the array
    const int pair = e / (2 * width), rem = e % (2 * width);
    const int x = rem >> 1, half = (rem & 1) ^ ((x >> 2) & 1);
    cbase[j] = to_global(arr == 0 ? lp.abase_hi(t) : arr == 1 ? lp.abase_lo(t)
                         : arr == 2 ? lp.bbase_hi(t) : lp.bbase_lo(t));
    cisb[j] = isb;
    cpair[j] = __builtin_amdgcn_readfirstlane(pair);         // one pair per copy (2 * width % 64 == 0)
    chalf[j] = half != 0;
    const int hoff = HS ? 0 : 8 * half;
    ccell[j] = (arr == 0 ? 0 : arr == 1 ? AC : arr == 2 ? 2 * AC : 2 * AC + BC) + cc * 64;
    if (isb) clane[j] = (uint32_t)(bcs * (x < t.cols ? x : t.cols - 1) + hoff);
    else clane[j] = (uint32_t)lp.arow(t, x < t.rows ? x : t.rows - 1) + (uint32_t)hoff;
  }

  // every wave issues CPW copies per chunk (a wave with fewer repeats the
  // last copy: the same cells, the same data), chunks past the end copy the
  // last pair, so that the code has no branches and the compiler can count
  // the copies in flight
  auto issue = [&](int ch, u32x4_t* dst) {
    // the table entries of the chunk's NP pairs first (one wait for all of
    // them), then the copies, each taking its pair's (and its lane's) entry
    constexpr int NE = HS ? 2 : 1;                           // entries per pair
    int up[NP], tv[NP][NE];
    int64_t tb[NP][NE];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int u = __builtin_amdgcn_readfirstlane(ch * NP + q < pmax ? ch * NP + q : pmax);
      up[q] = u;
#pragma unroll
      for (int h = 0; h < NE; ++h) {
        const int e = __builtin_amdgcn_readfirstlane(NE * u + h < emax ? NE * u + h : emax);
        tv[q][h] = atab[e];
        if constexpr (BTAB) tb[q][h] = btab[e];
      }
    }
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const gmem<const uint16_t>* g;
      int u = up[0], v0 = tv[0][0], v1 = tv[0][NE - 1];
      int64_t b0 = 0, b1 = 0;
      if constexpr (BTAB) b0 = tb[0][0], b1 = tb[0][NE - 1];
#pragma unroll
      for (int q = 1; q < NP; ++q) {                         // wave-uniform selects
        const bool m = cpair[j] == q;
        u = m ? up[q] : u;
        v0 = m ? tv[q][0] : v0;
        v1 = m ? tv[q][NE - 1] : v1;
        if constexpr (BTAB) b0 = m ? tb[q][0] : b0, b1 = m ? tb[q][NE - 1] : b1;
      }
      const bool h = HS && chalf[j];                         // this lane's entry
      const int v = h ? v1 : v0;
      if constexpr (BTAB) {      // brick offsets need 64 bits
        const int64_t po = cisb[j] ? (h ? b1 : b0) * bmul : (int64_t)((uint32_t)v * amul);
        g = cbase[j] + (po + (int64_t)clane[j]);
      } else {                   // offsets within one tau slab below 2^32 (host check)
        const uint32_t po = cisb[j] ? lp.b_pairoff(u) : (uint32_t)v * amul;
        g = cbase[j] + (po + clane[j]);
      }
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)g,
                                       (void __attribute__((address_space(3)))*)(dst + ccell[j]),
                                       16, 0, 0);
    }
  };

  f32x4_t acc[RB][NB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  // this lane's cells: group g = 4 kk + lk of the chunk is half (lk & 1) of
  // pair 2 kk + (lk >> 1); row / column x sits in cell 2 x + (half ^ bit 2 of x)
  const int lr = lane & 15, lk = lane >> 4, lh = lk & 1, lpr = lk >> 1;
  int ao[RB], bo[NB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int r = (wm * RB + rb) * 16 + lr;
    ao[rb] = (lpr * ROWS + r) * 2 + (lh ^ ((r >> 2) & 1));
  }
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int c = (wn * NB + cb) * 16 + lr;
    bo[cb] = 2 * AC + (lpr * COLS + c) * 2 + (lh ^ ((c >> 2) & 1));
  }

  const int ngroups = t.K / 8;
  const int nch = (npairs + NP - 1) / NP;
  // One chunk: wait for its copies, barrier, the copies of chunk ch + S - 1
  // into stage dst, then the matrix-core steps on stage ls.
  auto chunk = [&](int ch, u32x4_t* dst, const u32x4_t* ls) {
    wait_vm<CPW * (S - 2)>();        // this wave's copies of chunk ch have landed
    stage_barrier();                 // everyone's have; stage dst is free
    issue(ch + S - 1, dst);
    // groups past the end (last chunk only) read as zero in A
    const bool ok = ch * 4 + lk < ngroups;
    bf16x8_t ah[RB], al[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const u32x4_t z = {0u, 0u, 0u, 0u};
      const u32x4_t h = ls[ao[rb]], l = ls[ao[rb] + AC];
      ah[rb] = __builtin_bit_cast(bf16x8_t, ok ? h : z);
      al[rb] = __builtin_bit_cast(bf16x8_t, ok ? l : z);
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const bf16x8_t bh = __builtin_bit_cast(bf16x8_t, ls[bo[cb]]);
      const bf16x8_t bl = __builtin_bit_cast(bf16x8_t, ls[bo[cb] + BC]);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bh, acc[rb][cb], 0, 0, 0);
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bl, acc[rb][cb], 0, 0, 0);
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rb], bh, acc[rb][cb], 0, 0, 0);
      }
    }
  };
  // The stages are distinct LDS arrays and every access below names one of
  // them (the chunk loop is unrolled by S): the compiler then knows that
  // the copies in flight write other stages than the one read, and does not
  // wait for them before each LDS read (the waits the pipeline needs are the
  // explicit wait_vm + barrier of each chunk).
  int c0 = 0;
  issue(0, L0);
  if constexpr (S == 2) {
    for (; c0 + 2 <= nch; c0 += 2) {
      chunk(c0, L1, L0);
      chunk(c0 + 1, L0, L1);
    }
    if (c0 < nch) chunk(c0, L1, L0);
  } else {
    issue(1, L1);
    for (; c0 + 3 <= nch; c0 += 3) {
      chunk(c0, L2, L0);
      chunk(c0 + 1, L0, L1);
      chunk(c0 + 2, L1, L2);
    }
    if (c0 < nch) chunk(c0, L2, L0);
    if (c0 + 1 < nch) chunk(c0 + 1, L0, L1);
  }
  wait_vm<0>();                      // no copy of a past-the-end chunk outlives the tile

  // f32 16x16 MFMA output: lane l, element i -> row 4*(l/16) + i, col l%16
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int c = (wn * NB + cb) * 16 + lr;
    const bool cv = c < t.cols;
    const int64_t co = cv ? lp.coloff(t, c) : 0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if constexpr (P::kOut == 0) {
        // added with factor kSign to the FP64 output
        gmem<double>* __restrict__ ob = to_global(lp.obase(t));
        double old[4];
        int64_t off[4];
        bool okr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = (wm * RB + rb) * 16 + 4 * lk + i;
          okr[i] = cv && r < t.rows;
          off[i] = okr[i] ? lp.rowoff(t, r) + co : 0;
          old[i] = ob[off[i]];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (okr[i]) ob[off[i]] = old[i] + P::kSign * (double)acc[rb][cb][i];
      } else {
        // stored split into bf16 hi and lo
        gmem<uint16_t>* __restrict__ oh = to_global(lp.obase_hi(t));
        gmem<uint16_t>* __restrict__ ol = to_global(lp.obase_lo(t));
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = (wm * RB + rb) * 16 + 4 * lk + i;
          if (cv && r < t.rows) {
            const int64_t o = out_offset(lp, t, r, c, co);
            const float v = acc[rb][cb][i];
            const uint16_t h = f32_to_bf16_bits(v);
            oh[o] = h;
            ol[o] = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
          }
        }
      }
    }
  }
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_bf3_dma_kernel(P p) {
  int bx, by, bz;
  grid_tile(bx, by, bz);
  tile_bf3_dma_body<WM, WN, RB, NB, S, HS>(p, bx, by, bz);
}

// persistent form (same per-XCD queue protocol as tile_gemm_persistent)
template <int WM, int WN, int RB, int NB, int S, int HS, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_bf3_dma_persistent(P p, int n_work, int* queue) {
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
      tile_bf3_dma_body<WM, WN, RB, NB, S, HS>(p, start + l, 0, 0);
    }
  }
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
inline hipError_t launch_tile_bf3_dma(const P& p, dim3 grid, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_bf3_dma_kernel<WM, WN, RB, NB, S, HS, P>), grid, dim3(64 * WM * WN), 0, st, p);
  return hipGetLastError();
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
inline int persistent_cap_bf3_dma() {
  static int cap = 0;
  if (cap == 0) cap = resident_groups(tile_bf3_dma_persistent<WM, WN, RB, NB, S, HS, P>, 64 * WM * WN);
  return cap;
}

template <int WM, int WN, int RB, int NB, int S, int HS, class P>
inline hipError_t launch_tile_bf3_dma_persistent(const P& p, int n_work, int* queue, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  const int cap = persistent_cap_bf3_dma<WM, WN, RB, NB, S, HS, P>();
  const int grid = cap > 0 ? (n_work < cap ? n_work : cap) : n_work;
  hipLaunchKernelGGL((tile_bf3_dma_persistent<WM, WN, RB, NB, S, HS, P>), dim3(grid), dim3(64 * WM * WN), 0,
                     st, p, n_work, queue);
  return hipGetLastError();
}

}  // namespace gw
