// Device-side generator of the synthetic three-center bricks.
//
// Same definition as gwinputs/philox.py and gwinputs/system.py: Philox4x32-10
// (Salmon et al., SC'11) keyed by (seed, stream) with the 64-bit element index
// as counter, one Box-Muller normal per counter, value
//   z * exp(-k_t * (d_ab + (d_ac + d_bc)))
// for brick (a, b, c), element [mu][nu][P]; the index of (mu nu|P) uses the
// unordered AO pair so that the tensor is symmetric in mu and nu.
// Input preparation only: none of the GW method's arithmetic is here.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

__device__ __forceinline__ double philox_normal(uint32_t seed, uint32_t stream, uint64_t idx) {
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), 0u, 0u};
  uint32_t k0 = seed, k1 = stream;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    philox_round(c, k0, k1);
  }
  const double two_m32 = 2.3283064365386963e-10;   // 2^-32
  const double u1 = ((double)c[0] + 1.0) * two_m32;
  const double u2 = (double)c[1] * two_m32;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void gen_bricks_kernel(uint32_t seed, uint32_t stream, int64_t n_trip,
                                  const int32_t* __restrict__ trip,
                                  const double* __restrict__ dist, int32_t n_atoms,
                                  int32_t na, int32_t nr, int64_t n_ri_total,
                                  double k_t, double* __restrict__ out) {
  const int64_t bs = (int64_t)na * na * nr;
  const int64_t total = n_trip * bs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / bs;
    const int64_t r = e - t * bs;
    const int32_t i = (int32_t)(r / ((int64_t)na * nr));
    const int32_t j = (int32_t)((r / nr) % na);
    const int32_t p = (int32_t)(r % nr);
    const int32_t a = trip[3 * t], b = trip[3 * t + 1], c = trip[3 * t + 2];
    const uint64_t mu = (uint64_t)a * na + i, nu = (uint64_t)b * na + j;
    const uint64_t lo = mu < nu ? mu : nu, hi = mu < nu ? nu : mu;
    const uint64_t tri = hi * (hi + 1) / 2 + lo;
    const uint64_t idx = tri * (uint64_t)n_ri_total + (uint64_t)c * nr + p;
    const double s = dist[(int64_t)a * n_atoms + b] +
                     (dist[(int64_t)a * n_atoms + c] + dist[(int64_t)b * n_atoms + c]);
    out[e] = philox_normal(seed, stream, idx) * exp(-k_t * s);
  }
}

__global__ void gen_normal_kernel(uint32_t seed, uint32_t stream, const uint64_t* __restrict__ idx,
                                  int64_t n, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = philox_normal(seed, stream, idx[e]);
}

}  // namespace

extern "C" {

// Bricks of the listed triples (device int32 [n_trip][3]), uniform atom sizes
// na (AO) and nr (RI), atom distances dist (device [n_atoms][n_atoms]),
// written to out (device [n_trip][na][na][nr]).  Returns 0 or a hipError_t.
int gwgen_bricks(uint32_t seed, uint32_t stream, int64_t n_trip, const int32_t* trip,
                 const double* dist, int32_t n_atoms, int32_t na, int32_t nr,
                 int64_t n_ri_total, double k_t, double* out, hipStream_t st) {
  if (n_trip <= 0) return 0;
  const int64_t total = n_trip * (int64_t)na * na * nr;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gen_bricks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream,
                     n_trip, trip, dist, n_atoms, na, nr, n_ri_total, k_t, out);
  return (int)hipGetLastError();
}

// Normal deviates for an explicit list of counter indices.
int gwgen_normal(uint32_t seed, uint32_t stream, const uint64_t* idx, int64_t n, double* out,
                 hipStream_t st) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gen_normal_kernel, dim3((unsigned)blocks), dim3(256), 0, st, seed, stream,
                     idx, n, out);
  return (int)hipGetLastError();
}

}  // extern "C"
