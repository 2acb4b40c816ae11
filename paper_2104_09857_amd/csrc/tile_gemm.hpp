// FP64 MFMA tile engine for gfx950 (CDNA4), shared by every contraction.
//
// A workgroup of WM waves computes a (32*WM) x (16*NB) output tile
//   C[r][c] = sum_k A(r, k) * B(k, c)
// with v_mfma_f64_16x16x4f64.  Wave w owns rows [32w, 32w + 32) (two 16-row
// MFMA blocks) and all NB 16-column blocks, i.e. 2*NB accumulators of four
// doubles per lane.  K is staged through LDS in chunks of KC = 16: A as
// As[k][r], B as Bs[k][c] (both with a pad that puts consecutive k rows in
// opposite LDS bank halves).  The next chunk is prefetched into registers
// while the current one feeds the matrix cores.
//
// A problem type P supplies the index maps (all offsets in doubles):
//   bool   tile(bx, by, bz, Tile&)   fills rows/cols/K; false = skip tile
//   const double* abase(t), int64_t aroff(t, r), int64_t akoff(t, k)
//   const double* bbase(t), int64_t bkoff(t, k)
//   double ascale(t, k)             (only if P::kAScale)
//   void   store(t, r, c, v)        (kDot == false) or
//   void dot(t, r, c, v, s0&, s1&), void dot_out(t, s0, s1)   (kDot == true):
//   two weighted sums of the tile instead of a store
// so A(r, k) = abase[aroff(r) + akoff(k)] (* ascale(k)) and
// B(k, c) = bbase[bkoff(k) + c]; entries outside rows/cols/K read as zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gw {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int KC = 16;

__host__ __device__ constexpr int lds_stride(int n) { return n + (16 - n % 32 + 32) % 32; }

struct TileBase {
  int rows, cols, K;
};

template <int WM, int NB, class P>
__global__ __launch_bounds__(64 * WM) void tile_gemm_kernel(P p) {
  constexpr int ROWS = 32 * WM, COLS = 16 * NB, NT = 64 * WM;
  constexpr int AST = lds_stride(ROWS), BST = lds_stride(COLS);
  constexpr int APT = KC * ROWS / NT;                 // = 8
  constexpr int BPT = (KC * COLS + NT - 1) / NT;
  __shared__ double As[KC * AST];
  __shared__ double Bs[KC * BST];

  typename P::Tile t;
  if (!p.tile(blockIdx.x, blockIdx.y, blockIdx.z, t)) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const double* __restrict__ abase = p.abase(t);
  const double* __restrict__ bbase = p.bbase(t);

  // this thread's A row is fixed: r = tid % ROWS, k = tid / ROWS + 2 i
  const int ar = tid % ROWS;
  const bool arow_ok = ar < t.rows;
  const int64_t aro = arow_ok ? p.aroff(t, ar) : 0;
  const int ak0 = tid / ROWS;

  double ra[APT], rbv[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int k = k0 + ak0 + 2 * i;
      double v = 0.0;
      if (arow_ok && k < t.K) {
        v = abase[aro + p.akoff(t, k)];
        if constexpr (P::kAScale) v *= p.ascale(t, k);
      }
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int e = tid + i * NT;
      const int c = e % COLS, kl = e / COLS;
      const int k = k0 + kl;
      double v = 0.0;
      if (kl < KC && c < t.cols && k < t.K) v = bbase[p.bkoff(t, k) + c];
      rbv[i] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < APT; ++i) As[(ak0 + 2 * i) * AST + ar] = ra[i];
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
      const int e = tid + i * NT;
      const int c = e % COLS, kl = e / COLS;
      if (kl < KC) Bs[kl * BST + c] = rbv[i];
    }
  };

  dbl4 acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

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
      const double a0 = As[krow * AST + wave * 32 + lr];
      const double a1 = As[krow * AST + wave * 32 + 16 + lr];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const double b = Bs[krow * BST + cb * 16 + lr];
        acc[0][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc[0][cb], 0, 0, 0);
        acc[1][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc[1][cb], 0, 0, 0);
      }
    }
    __syncthreads();
    if (ch + 1 < nch) {
      stash();
      __syncthreads();
    }
  }

  // D layout of the 16x16x4 f64 MFMA on gfx950 (measured): lane l, element i
  // -> row 4*i + l/16, col l%16
  if constexpr (!P::kDot) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = wave * 32 + rb * 16 + 4 * i + lk;
          const int c = cb * 16 + lr;
          if (r < t.rows && c < t.cols) p.store(t, r, c, acc[rb][cb][i]);
        }
  } else {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = wave * 32 + rb * 16 + 4 * i + lk;
          const int c = cb * 16 + lr;
          if (r < t.rows && c < t.cols) p.dot(t, r, c, acc[rb][cb][i], s0, s1);
        }
    // fixed-order block reduction (deterministic)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, 64);
      s1 += __shfl_xor(s1, off, 64);
    }
    __shared__ double red[2 * WM];
    if (lane == 0) {
      red[wave] = s0;
      red[WM + wave] = s1;
    }
    __syncthreads();
    if (tid == 0) {
      double t0 = 0.0, t1 = 0.0;
      for (int w = 0; w < WM; ++w) {
        t0 += red[w];
        t1 += red[WM + w];
      }
      p.dot_out(t, t0, t1);
    }
  }
}

template <int WM, int NB, class P>
inline hipError_t launch_tile_gemm(const P& p, dim3 grid, hipStream_t st) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
  hipLaunchKernelGGL((tile_gemm_kernel<WM, NB, P>), grid, dim3(64 * WM), 0, st, p);
  return hipGetLastError();
}

}  // namespace gw
