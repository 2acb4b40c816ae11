// Status handling, system validation and the HBM-bound helper kernels:
// block Frobenius norms (wavefront reductions), the atom-block filter and
// the mirror of symmetric block matrices.
#include <cmath>
#include <cstring>

#include "gw_internal.hpp"

namespace gw {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// per-atom function offsets: monotone from 0, 1 .. per functions per atom
static gw_status check_offsets(const int32_t* off, int n_atoms, int per, const char* what) {
  if (!off) return GW_OK;
  if (off[0] != 0) {
    set_error(std::string(what) + "[0] must be 0");
    return GW_ERR_ARG;
  }
  for (int a = 0; a < n_atoms; ++a) {
    const int64_t k = (int64_t)off[a + 1] - off[a];
    if (k < 1 || k > per) {
      set_error(std::string(what) + ": atom " + std::to_string(a) + " carries " + std::to_string(k) +
                " functions, outside [1, " + std::to_string(per) + "]");
      return GW_ERR_ARG;
    }
  }
  return GW_OK;
}

int64_t sys_n_ao(const gw_system* s) {
  return s->ao_off ? (int64_t)s->ao_off[s->n_atoms] : (int64_t)s->n_atoms * s->ao_per_atom;
}
int64_t sys_n_ri(const gw_system* s) {
  return s->ri_off ? (int64_t)s->ri_off[s->n_atoms] : (int64_t)s->n_atoms * s->ri_per_atom;
}

gw_status check_system_sizes(const gw_system* s) {
  GW_CHECK_ARG(s != nullptr, "system is null");
  GW_CHECK_ARG(s->n_atoms > 0, "n_atoms must be positive");
  GW_CHECK_ARG(s->ao_per_atom > 0 && s->ri_per_atom > 0, "atom sizes must be positive");
  GW_CHECK_ARG((int64_t)s->n_atoms * s->ao_per_atom < (1 << 30) &&
                   (int64_t)s->n_atoms * s->ri_per_atom < (1 << 30),
               "system too large");
  gw_status rc;
  if ((rc = check_offsets(s->ao_off, s->n_atoms, s->ao_per_atom, "ao_off")) != GW_OK) return rc;
  if ((rc = check_offsets(s->ri_off, s->n_atoms, s->ri_per_atom, "ri_off")) != GW_OK) return rc;
  const int64_t n_ao = sys_n_ao(s);
  GW_CHECK_ARG(s->n_occ >= 1 && s->n_occ < n_ao, "n_occ must be in [1, n_ao)");
  return GW_OK;
}

gw_status check_system(const gw_system* s) {
  gw_status rc = check_system_sizes(s);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(s->n_trip >= 0, "n_trip must be >= 0");
  GW_CHECK_ARG(s->n_trip == 0 || (s->trip != nullptr && s->t3c != nullptr),
               "trip and t3c must be given when n_trip > 0");
  for (int64_t i = 0; i < s->n_trip; ++i) {
    for (int j = 0; j < 3; ++j) {
      const int32_t v = s->trip[3 * i + j];
      GW_CHECK_ARG(v >= 0 && v < s->n_atoms, "triple atom index out of range");
    }
  }
  return GW_OK;
}

// ---------------------------------------------------------------------------
// Systems with per-atom sizes run on their padded form: atom a's functions
// occupy the first n_a of its ao_per_atom (ri_per_atom) slots, the other
// slots are zero functions.  map[i] = padded index of compact function i.
gw_status pad_maps(const gw_system* s, Scratch& sc, PadMaps& m) {
  m.n_ao = (int)sys_n_ao(s);
  m.n_ri = (int)sys_n_ri(s);
  m.N = s->n_atoms * s->ao_per_atom;
  m.NRI = s->n_atoms * s->ri_per_atom;
  auto build = [&](const int32_t* off, int per, int n) {
    std::vector<int32_t> v(n);
    for (int a = 0, i = 0; a < s->n_atoms; ++a) {
      const int k = off ? off[a + 1] - off[a] : per;
      for (int j = 0; j < k; ++j) v[i++] = a * per + j;
    }
    return v;
  };
  gw_status rc = sc.upload(&m.ao, build(s->ao_off, s->ao_per_atom, m.n_ao));
  if (rc != GW_OK) return rc;
  return sc.upload(&m.ri, build(s->ri_off, s->ri_per_atom, m.n_ri));
}

gw_system padded_view(const gw_system* s) {
  gw_system p = *s;
  p.ao_off = nullptr;
  p.ri_off = nullptr;
  return p;
}

// out[m][map[i]][map[j]] = in[m][i][j] (rows of cols_in doubles, cols map)
__global__ void scatter_square_kernel(const double* __restrict__ in, int n_rows, int n, int ld_in,
                                      double* __restrict__ out, int np, const int32_t* __restrict__ rmap,
                                      const int32_t* __restrict__ cmap, int64_t n_mat) {
  const int64_t per = (int64_t)n_rows * n, total = n_mat * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / per;
    const int r = (int)((e - m * per) / n), c = (int)(e - m * per - (int64_t)r * n);
    const int rp = rmap ? rmap[r] : r;
    out[m * (int64_t)(rmap ? np : n_rows) * np + (int64_t)rp * np + cmap[c]] =
        in[m * (int64_t)n_rows * ld_in + (int64_t)r * ld_in + c];
  }
}

// out[m][i][j] = in[m][map[i]][map[j]]
__global__ void gather_square_kernel(const double* __restrict__ in, int np, double* __restrict__ out,
                                     int n, const int32_t* __restrict__ map, int64_t n_mat) {
  const int64_t per = (int64_t)n * n, total = n_mat * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / per;
    const int i = (int)((e - m * per) / n), j = (int)(e - m * per - (int64_t)i * n);
    out[e] = in[m * (int64_t)np * np + (int64_t)map[i] * np + map[j]];
  }
}

static unsigned blocks_for(int64_t total) {
  return (unsigned)std::min<int64_t>(std::max<int64_t>((total + 255) / 256, 1), 1 << 20);
}

hipError_t scatter_square(const double* in, int n, double* out, int np, const int32_t* map,
                          int64_t n_mat, hipStream_t st) {
  hipError_t e = fill_zero(out, 2 * n_mat * (int64_t)np * np, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_square_kernel, dim3(blocks_for(n_mat * n * n)), dim3(256), 0, st, in, n,
                     n, n, out, np, map, map, n_mat);
  return hipGetLastError();
}

hipError_t scatter_cols(const double* in, int rows, int n, double* out, int np, const int32_t* map,
                        hipStream_t st) {
  hipError_t e = fill_zero(out, 2 * (int64_t)rows * np, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_square_kernel, dim3(blocks_for((int64_t)rows * n)), dim3(256), 0, st, in,
                     rows, n, n, out, np, (const int32_t*)nullptr, map, (int64_t)1);
  return hipGetLastError();
}

hipError_t gather_square(const double* in, int np, double* out, int n, const int32_t* map,
                         int64_t n_mat, hipStream_t st) {
  hipLaunchKernelGGL(gather_square_kernel, dim3(blocks_for(n_mat * n * n)), dim3(256), 0, st, in, np,
                     out, n, map, n_mat);
  return hipGetLastError();
}

gw_status build_groups(const gw_system* s, double eps, hipStream_t st, Scratch& sc,
                       BrickGroups& out) {
  const int na = s->n_atoms;
  const int64_t bs = (int64_t)s->ao_per_atom * s->ao_per_atom * s->ri_per_atom;
  out = BrickGroups{};
  out.gb_start.assign(na + 1, 0);
  out.goff.push_back(0);
  if (s->n_trip == 0) return GW_OK;
  double* d_norm = nullptr;
  gw_status rc = sc.alloc(&d_norm, (size_t)s->n_trip);
  if (rc != GW_OK) return rc;
  GW_HIP(brick_norms(s->t3c, s->n_trip, bs, d_norm, st));
  std::vector<double> norm(s->n_trip);
  GW_HIP(hipMemcpyAsync(norm.data(), d_norm, sizeof(double) * s->n_trip, hipMemcpyDeviceToHost, st));
  GW_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> kept;
  kept.reserve(s->n_trip);
  for (int64_t i = 0; i < s->n_trip; ++i) {
    if (!std::isfinite(norm[i])) {
      set_error("three-center tensor contains NaN or Inf");
      return GW_ERR_ARG;
    }
    if (!(norm[i] < eps)) kept.push_back(i);
  }
  std::sort(kept.begin(), kept.end(), [&](int64_t x, int64_t y) {
    const int32_t* a = s->trip + 3 * x;
    const int32_t* b = s->trip + 3 * y;
    const int64_t kx = (int64_t)a[1] * na + a[2], ky = (int64_t)b[1] * na + b[2];
    if (kx != ky) return kx < ky;
    if (a[0] != b[0]) return a[0] < b[0];
    return x < y;
  });
  out.goff.clear();
  for (size_t i = 0; i < kept.size(); ++i) {
    const int32_t* t = s->trip + 3 * kept[i];
    if (i > 0) {
      const int32_t* u = s->trip + 3 * kept[i - 1];
      if (u[0] == t[0] && u[1] == t[1] && u[2] == t[2]) {
        set_error("duplicate triple in trip");
        return GW_ERR_ARG;
      }
    }
    if (out.gs.empty() || out.gs.back() != t[1] || out.gc.back() != t[2]) {
      out.gs.push_back(t[1]);
      out.gc.push_back(t[2]);
      out.goff.push_back((int32_t)out.seg_atom.size());
    }
    out.seg_atom.push_back(t[0]);
    out.seg_brick.push_back(kept[i]);
  }
  out.goff.push_back((int32_t)out.seg_atom.size());
  out.n_kept = (int64_t)kept.size();
  for (int g = 0; g < out.n_groups(); ++g) out.gb_start[out.gs[g] + 1]++;
  for (int b = 0; b < na; ++b) out.gb_start[b + 1] += out.gb_start[b];
  return GW_OK;
}

Panels build_panels(int n_atoms, int PG, int PC, const std::vector<int32_t>& col_atom,
                    const std::vector<int32_t>& k_atom, int per, int rows_factor) {
  Panels P;
  P.PG = PG;
  P.PC = PC;
  P.n_pan = (n_atoms + PG - 1) / PG;
  std::vector<std::vector<int32_t>> U(P.n_pan);
  for (size_t g = 0; g < col_atom.size(); ++g) U[col_atom[g] / PG].push_back(k_atom[g]);
  P.ulen.assign(P.n_pan, 0);
  P.km_off.assign(P.n_pan + 1, 0);
  P.off.assign(P.n_pan + 1, 0);
  for (int p = 0; p < P.n_pan; ++p) {
    auto& u = U[p];
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    P.ulen[p] = (int32_t)u.size();
    for (int32_t a : u)
      for (int i = 0; i < per; ++i) P.kmap.push_back(a * per + i);
    P.km_off[p + 1] = (int32_t)P.kmap.size();
    P.off[p + 1] = P.off[p] + (int64_t)rows_factor * per * P.ulen[p] * PC;
  }
  P.gslot.resize(col_atom.size());
  for (size_t g = 0; g < col_atom.size(); ++g) {
    const auto& u = U[col_atom[g] / PG];
    P.gslot[g] = (int32_t)(std::lower_bound(u.begin(), u.end(), k_atom[g]) - u.begin());
  }
  return P;
}

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void brick_norms_kernel(const double* __restrict__ t3c, int64_t n, int64_t bs,
                                   double* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (b >= n) return;
  const double* p = t3c + b * bs;
  double s = 0.0;
  for (int64_t i = lane; i < bs; i += 64) s += p[i] * p[i];
  s = wave_sum(s);
  if (lane == 0) out[b] = sqrt(s);
}

// one wave per (matrix, block row atom, block col atom)
// in may equal out (in-place filter): no __restrict__ here
__global__ void filter_blocks_kernel(const double* in, double* out,
                                     int n_atoms, int na, double eps, uint8_t* dropped,
                                     int64_t n_blocks) {
  const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blk >= n_blocks) return;
  const int64_t per = (int64_t)n_atoms * n_atoms;
  const int64_t m = blk / per;
  const int a = (int)((blk % per) / n_atoms), b = (int)(blk % n_atoms);
  const int64_t n = (int64_t)n_atoms * na;
  const double* src = in + m * n * n + (int64_t)a * na * n + (int64_t)b * na;
  double* dst = out + m * n * n + (int64_t)a * na * n + (int64_t)b * na;
  const int cnt = na * na;
  double s = 0.0;
  for (int i = lane; i < cnt; i += 64) {
    const double v = src[(i / na) * n + i % na];
    s += v * v;
  }
  s = wave_sum(s);
  const bool drop = sqrt(s) < eps;
  for (int i = lane; i < cnt; i += 64) dst[(i / na) * n + i % na] = drop ? 0.0 : src[(i / na) * n + i % na];
  if (dropped && lane == 0) dropped[blk] = drop ? 1 : 0;
}

__global__ void block_norms_f32_kernel(const double* __restrict__ x, int n_atoms, int nb,
                                       int log10_out, float* __restrict__ out, int64_t n_blocks) {
  const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blk >= n_blocks) return;
  const int64_t per = (int64_t)n_atoms * n_atoms;
  const int64_t m = blk / per;
  const int a = (int)((blk % per) / n_atoms), b = (int)(blk % n_atoms);
  const int64_t n = (int64_t)n_atoms * nb;
  const double* src = x + m * n * n + (int64_t)a * nb * n + (int64_t)b * nb;
  double s = 0.0;
  for (int i = lane; i < nb * nb; i += 64) {
    const double v = src[(i / nb) * n + i % nb];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[blk] = log10_out ? (float)log10(sqrt(s) + 1e-30) : (float)sqrt(s);
}

__global__ void zero_unkept_kernel(double* __restrict__ x, int n_atoms, int nb,
                                   const uint8_t* __restrict__ keep, int64_t n_blocks) {
  const int64_t blk = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (blk >= n_blocks) return;
  const int64_t per = (int64_t)n_atoms * n_atoms;
  const int64_t m = blk / per;
  const int a = (int)((blk % per) / n_atoms), b = (int)(blk % n_atoms);
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  if (keep[m * per + (int64_t)lo * n_atoms + hi]) return;
  const int64_t n = (int64_t)n_atoms * nb;
  double* dst = x + m * n * n + (int64_t)a * nb * n + (int64_t)b * nb;
  for (int i = lane; i < nb * nb; i += 64) dst[(i / nb) * n + i % nb] = 0.0;
}

// 32x32 tiles through LDS; only tiles touching a lower atom block do work
__global__ void mirror_kernel(double* __restrict__ x, int n, int nb) {
  __shared__ double tile[32][33];
  const int64_t m = blockIdx.z;
  double* a = x + m * (int64_t)n * n;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;   // destination tile (rows r0.., cols c0..)
  const int rlast = (r0 + 31 < n ? r0 + 31 : n - 1);
  if (rlast / nb <= c0 / nb) return;                       // no element below the block diagonal
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int sr = c0 + j, sc = r0 + tx;                    // source element (c0 + j, r0 + tx)
    tile[j][tx] = (sr < n && sc < n) ? a[(int64_t)sr * n + sc] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int dr = r0 + j, dc = c0 + tx;
    if (dr < n && dc < n && (dr / nb) > (dc / nb)) a[(int64_t)dr * n + dc] = tile[tx][j];
  }
}

}  // namespace

hipError_t brick_norms(const double* t3c, int64_t n, int64_t bs, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int wpb = 4;
  hipLaunchKernelGGL(brick_norms_kernel, dim3((unsigned)((n + wpb - 1) / wpb)), dim3(64 * wpb), 0,
                     st, t3c, n, bs, out);
  return hipGetLastError();
}

hipError_t filter_square_blocks(const double* in, double* out, int n_mat, int n_atoms, int na,
                                double eps, uint8_t* dropped, hipStream_t st) {
  const int64_t nblk = (int64_t)n_mat * n_atoms * n_atoms;
  if (nblk <= 0) return hipSuccess;
  const int wpb = 4;
  hipLaunchKernelGGL(filter_blocks_kernel, dim3((unsigned)((nblk + wpb - 1) / wpb)),
                     dim3(64 * wpb), 0, st, in, out, n_atoms, na, eps, dropped, nblk);
  return hipGetLastError();
}

hipError_t block_norms_f32(const double* x, int n_mat, int n_atoms, int nb, int log10_out,
                           float* out, hipStream_t st) {
  const int64_t nblk = (int64_t)n_mat * n_atoms * n_atoms;
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(block_norms_f32_kernel, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, st, x,
                     n_atoms, nb, log10_out, out, nblk);
  return hipGetLastError();
}

hipError_t zero_unkept_blocks(double* x, int n_mat, int n_atoms, int nb, const uint8_t* keep,
                              hipStream_t st) {
  const int64_t nblk = (int64_t)n_mat * n_atoms * n_atoms;
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_unkept_kernel, dim3((unsigned)((nblk + 3) / 4)), dim3(256), 0, st, x,
                     n_atoms, nb, keep, nblk);
  return hipGetLastError();
}

hipError_t mirror_lower_blocks(double* x, int n_mat, int n, int nb, hipStream_t st) {
  if (n_mat <= 0 || n <= 0) return hipSuccess;
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(mirror_kernel, dim3(t, t, n_mat), dim3(256), 0, st, x, n, nb);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(uint32_t* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0u;
}

hipError_t fill_zero(void* x, int64_t n_words32, hipStream_t st) {
  if (n_words32 <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n_words32 + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, st, static_cast<uint32_t*>(x),
                     n_words32);
  return hipGetLastError();
}

}  // namespace gw

extern "C" const char* gw_last_error(void) { return gw::g_last_error.c_str(); }
extern "C" const char* gw_version(void) { return "libgw 0.1 (gfx950, FP64 MFMA)"; }
