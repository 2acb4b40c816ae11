// Split-precision (BF16 x 3) MFMA tile engine for gfx950.
//
// Every FP64 operand x is carried as two bfloat16 numbers, hi = bf16(x) and
// lo = bf16(x - hi), and a product is formed as
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// with three v_mfma_f32_16x16x32_bf16 and FP32 accumulation (the scheme of
// Henry, Tang and Heinecke, ARITH 2019); the dropped a_lo b_lo term and the
// two roundings leave a relative error of order 2^-16 per product.
//
// A workgroup of WM x WN waves computes a (16*RB*WM) x (16*NB*WN) tile; wave
// (wm, wn) owns RB x NB MFMA blocks (f32 accumulators, four per lane).  The
// contraction index is stored k-contiguous in groups of 8 bf16 (16 bytes):
//   A group (r, g) at abase + aroff(r) + akoff(g)      (offsets in bf16 units)
//   B group (g, c) at bbase + bkoff(g) + bcs() c
// for both the hi and the lo arrays (same offsets).  LDS holds A[r][k] and
// B[c][k] so that each lane reads its 8 k values with one 16-byte access.
// Groups outside rows / cols / K groups read as zero.  Output: kOut == 0 adds
// kSign * C (converted to FP64) to an FP64 array; kOut == 1 stores C split
// into bf16 hi/lo arrays.  Offsets of the output are rowoff(t, r) +
// coloff(t, c), or outoff(t, r, c) when the problem sets kOutOff.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tile_gemm.hpp"

namespace gw {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bf16 bits
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ inline void split_bf16(double x, uint16_t& hi, uint16_t& lo) {
  hi = f32_to_bf16_bits((float)x);
  lo = f32_to_bf16_bits((float)(x - (double)bf16_bits_to_f32(hi)));
}

// Offset of output element (r, c) of a split (kOut == 1) store: rowoff(t, r) +
// coloff(t, c) (co), or outoff(t, r, c) for problems whose layout mixes the
// two (P::kOutOff).
template <class P, class = void>
struct has_outoff : std::false_type {};
template <class P>
struct has_outoff<P, std::void_t<decltype(P::kOutOff)>> : std::bool_constant<P::kOutOff> {};
template <class P, class T>
__device__ __forceinline__ int64_t out_offset(const P& lp, const T& t, int r, int c, int64_t co) {
  if constexpr (has_outoff<P>::value) return lp.outoff(t, r, c);
  else return lp.rowoff(t, r) + co;
}

template <int WM, int WN, int RB, int NB, int KC, class P>
__device__ __forceinline__ void tile_bf16x3_body(const P& p, int bx, int by, int bz) {
  constexpr int ROWS = 16 * RB * WM, COLS = 16 * NB * WN, NT = 64 * WM * WN;
  constexpr int KG = KC / 8;                 // 16-byte groups per row per chunk
  constexpr int LST = KC + 8;                // LDS row stride (bf16), padded
  constexpr int AG = (ROWS * KG + NT - 1) / NT;
  constexpr int BG = (COLS * KG + NT - 1) / NT;
  static_assert(KC % 32 == 0, "KC must be a multiple of the MFMA K (32)");
  __shared__ __attribute__((aligned(16))) uint16_t Ah[ROWS * LST];
  __shared__ __attribute__((aligned(16))) uint16_t Al[ROWS * LST];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[COLS * LST];
  __shared__ __attribute__((aligned(16))) uint16_t Bl[COLS * LST];
  __shared__ int tabA[P::kTabA > 0 ? P::kTabA : 1];
  __shared__ int tabB[P::kTabB > 0 ? P::kTabB : 1];

  typename P::Tile t;
  if (!p.tile(bx, by, bz, t)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const auto lp = resolve(p, t);
  lp.fill(t, tabA, tabB, tid, NT);
  __syncthreads();
  const gmem<const uint16_t>* __restrict__ ahb = to_global(lp.abase_hi(t));
  const gmem<const uint16_t>* __restrict__ alb = to_global(lp.abase_lo(t));
  const gmem<const uint16_t>* __restrict__ bhb = to_global(lp.bbase_hi(t));
  const gmem<const uint16_t>* __restrict__ blb = to_global(lp.bbase_lo(t));
  const int ngroups = t.K / 8;               // K is a multiple of 16
  const int gmax = ngroups - 1;

  u32x4_t rah[AG], ral[AG], rbh[BG], rbl[BG];
  uint32_t amask = 0u, bmask = 0u;
  auto load = [&](int g0) {
    int64_t aoff[AG], boff[BG];
#pragma unroll
    for (int i = 0; i < AG; ++i) {
      const int e = tid + i * NT, r = e % ROWS, g = g0 + e / ROWS;
      const bool ok = e < ROWS * KG && r < t.rows && g < ngroups;
      amask = ok ? (amask | (1u << i)) : (amask & ~(1u << i));
      const int64_t o = lp.aroff(t, r < t.rows ? r : t.rows - 1) + lp.akoff(t, g < gmax ? g : gmax, tabA);
      aoff[i] = ok ? o : 0;
    }
#pragma unroll
    for (int i = 0; i < BG; ++i) {
      const int e = tid + i * NT, c = e % COLS, g = g0 + e / COLS;
      const bool ok = e < COLS * KG && c < t.cols && g < ngroups;
      bmask = ok ? (bmask | (1u << i)) : (bmask & ~(1u << i));
      const int64_t o = lp.bkoff(t, g < gmax ? g : gmax, tabB) + (int64_t)lp.bcs() * c;
      boff[i] = ok ? o : 0;
    }
#pragma unroll
    for (int i = 0; i < AG; ++i) {
      rah[i] = *reinterpret_cast<const gmem<const u32x4_t>*>(ahb + aoff[i]);
      ral[i] = *reinterpret_cast<const gmem<const u32x4_t>*>(alb + aoff[i]);
    }
#pragma unroll
    for (int i = 0; i < BG; ++i) {
      rbh[i] = *reinterpret_cast<const gmem<const u32x4_t>*>(bhb + boff[i]);
      rbl[i] = *reinterpret_cast<const gmem<const u32x4_t>*>(blb + boff[i]);
    }
  };
  auto stash = [&]() {
    const u32x4_t z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < AG; ++i) {
      const int e = tid + i * NT, r = e % ROWS, gl = e / ROWS;
      if (e < ROWS * KG) {
        const bool ok = (amask >> i) & 1u;
        *reinterpret_cast<u32x4_t*>(&Ah[r * LST + 8 * gl]) = ok ? rah[i] : z;
        *reinterpret_cast<u32x4_t*>(&Al[r * LST + 8 * gl]) = ok ? ral[i] : z;
      }
    }
#pragma unroll
    for (int i = 0; i < BG; ++i) {
      const int e = tid + i * NT, c = e % COLS, gl = e / COLS;
      if (e < COLS * KG) {
        const bool ok = (bmask >> i) & 1u;
        *reinterpret_cast<u32x4_t*>(&Bh[c * LST + 8 * gl]) = ok ? rbh[i] : z;
        *reinterpret_cast<u32x4_t*>(&Bl[c * LST + 8 * gl]) = ok ? rbl[i] : z;
      }
    }
  };

  f32x4_t acc[RB][NB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  const int nch = (ngroups + KG - 1) / KG;
  load(0);
  stash();
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) load((ch + 1) * KG);
#pragma unroll
    for (int kk = 0; kk < KC / 32; ++kk) {
      const int ko = kk * 32 + 8 * lk;
      bf16x8_t ah[RB], al[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int r = (wm * RB + rb) * 16 + lr;
        ah[rb] = *reinterpret_cast<const bf16x8_t*>(&Ah[r * LST + ko]);
        al[rb] = *reinterpret_cast<const bf16x8_t*>(&Al[r * LST + ko]);
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int c = (wn * NB + cb) * 16 + lr;
        const bf16x8_t bh = *reinterpret_cast<const bf16x8_t*>(&Bh[c * LST + ko]);
        const bf16x8_t bl = *reinterpret_cast<const bf16x8_t*>(&Bl[c * LST + ko]);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bh, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bl, acc[rb][cb], 0, 0, 0);
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rb], bh, acc[rb][cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (ch + 1 < nch) {
      stash();
      __syncthreads();
    }
  }

  // f32 16x16 MFMA output on gfx950 (measured): lane l, element i -> row 4*(l/16) + i, col l%16
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int c = (wn * NB + cb) * 16 + lr;
    const bool cv = c < t.cols;
    const int64_t co = cv ? lp.coloff(t, c) : 0;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if constexpr (P::kOut == 0) {
        gmem<double>* __restrict__ ob = to_global(lp.obase(t));
        double old[4];
        int64_t off[4];
        bool ok[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = (wm * RB + rb) * 16 + 4 * lk + i;
          ok[i] = cv && r < t.rows;
          off[i] = ok[i] ? lp.rowoff(t, r) + co : 0;
          old[i] = ob[off[i]];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (ok[i]) ob[off[i]] = old[i] + P::kSign * (double)acc[rb][cb][i];
      } else {
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

template <int WM, int WN, int RB, int NB, int KC, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_bf16x3_kernel(P p) {
  int bx, by, bz;
  grid_tile(bx, by, bz);
  tile_bf16x3_body<WM, WN, RB, NB, KC>(p, bx, by, bz);
}

// persistent form (same per-XCD queue protocol as tile_gemm_persistent)
template <int WM, int WN, int RB, int NB, int KC, class P>
__global__ __launch_bounds__(64 * WM * WN) void tile_bf16x3_persistent(P p, int n_work, int* queue) {
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
      tile_bf16x3_body<WM, WN, RB, NB, KC>(p, start + l, 0, 0);
    }
  }
}

template <int WM, int WN, int RB, int NB, int KC, class P>
inline hipError_t launch_tile_bf16x3(const P& p, dim3 grid, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_bf16x3_kernel<WM, WN, RB, NB, KC, P>), grid, dim3(64 * WM * WN), 0, st, p);
  return hipGetLastError();
}

template <int WM, int WN, int RB, int NB, int KC, class P>
inline int persistent_cap_bf16x3() {
  static int cap = 0;
  if (cap == 0) cap = resident_groups(tile_bf16x3_persistent<WM, WN, RB, NB, KC, P>, 64 * WM * WN);
  return cap;
}

template <int WM, int WN, int RB, int NB, int KC, class P>
inline hipError_t launch_tile_bf16x3_persistent(const P& p, int n_work, int* queue, hipStream_t st) {
  if (n_work <= 0) return hipSuccess;
  const int cap = persistent_cap_bf16x3<WM, WN, RB, NB, KC, P>();
  const int grid = cap > 0 ? (n_work < cap ? n_work : cap) : n_work;
  hipLaunchKernelGGL((tile_bf16x3_persistent<WM, WN, RB, NB, KC, P>), dim3(grid), dim3(64 * WM * WN), 0,
                     st, p, n_work, queue);
  return hipGetLastError();
}

}  // namespace gw
