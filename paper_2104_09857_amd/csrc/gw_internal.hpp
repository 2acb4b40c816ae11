// Internal helpers of libgw: status handling, scratch memory, shared kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gw.h"

namespace gw {

void set_error(const std::string& msg);
void clear_error();

#define GW_CHECK_ARG(cond, msg)      \
  do {                               \
    if (!(cond)) {                   \
      ::gw::set_error(msg);          \
      return GW_ERR_ARG;             \
    }                                \
  } while (0)

#define GW_HIP(call)                                                           \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::gw::set_error(std::string("HIP error in ") + #call + ": " +            \
                      hipGetErrorString(e_));                                  \
      return GW_ERR_HIP;                                                       \
    }                                                                          \
  } while (0)

// Device allocations released when the owner goes out of scope: stream
// ordered (hipMallocAsync / hipFreeAsync on `st`) for the scratch of one
// call, or plain hipMalloc / hipFree (ordered = false) for objects that
// outlive the stream they were created on (plans).
class Scratch {
 public:
  explicit Scratch(hipStream_t st, bool ordered = true) : st_(st), ordered_(ordered) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() {
    for (void* p : ptrs_) (void)(ordered_ ? hipFreeAsync(p, st_) : hipFree(p));
  }
  template <class T>
  gw_status alloc(T** out, size_t count) {
    void* p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    hipError_t e = ordered_ ? hipMallocAsync(&p, bytes, st_) : hipMalloc(&p, bytes);
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      set_error("scratch allocation of " + std::to_string(bytes) + " bytes failed");
      return GW_ERR_NOMEM;
    }
    ptrs_.push_back(p);
    *out = static_cast<T*>(p);
    return GW_OK;
  }
  template <class T>
  gw_status upload(T** out, const std::vector<T>& host) {
    gw_status s = alloc(out, host.size());
    if (s != GW_OK) return s;
    if (!host.empty()) {
      hipError_t e = hipMemcpyAsync(*out, host.data(), host.size() * sizeof(T),
                                    hipMemcpyHostToDevice, st_);
      if (e != hipSuccess) {
        set_error(std::string("upload failed: ") + hipGetErrorString(e));
        return GW_ERR_HIP;
      }
    }
    return GW_OK;
  }
  hipStream_t stream() const { return st_; }

 private:
  hipStream_t st_;
  bool ordered_;
  std::vector<void*> ptrs_;
};

// x[0 .. n_words) = 0 with a kernel (usable inside a captured graph, unlike
// hipMemsetAsync)
hipError_t fill_zero(void* x, int64_t n_words32, hipStream_t st);

// Validates the system description (host side, before any launch).
gw_status check_system(const gw_system* s);
// The same without the triple list (sizes, offsets, occupation).
gw_status check_system_sizes(const gw_system* s);
// AO / RI function counts (the offsets' totals, or atoms x per-atom size).
int64_t sys_n_ao(const gw_system* s);
int64_t sys_n_ri(const gw_system* s);

// Systems with per-atom sizes (ao_off / ri_off) run on their padded form:
// atom a's functions take the first of its ao_per_atom (ri_per_atom) slots.
// ao / ri: device maps compact function index -> padded index.
struct PadMaps {
  int n_ao = 0, n_ri = 0, N = 0, NRI = 0;
  int32_t *ao = nullptr, *ri = nullptr;
};
gw_status pad_maps(const gw_system* s, Scratch& sc, PadMaps& m);
// the same system without offsets (its padded form; bricks are already padded)
gw_system padded_view(const gw_system* s);
// out[m] (np x np, zeroed first) with out[m][map[i]][map[j]] = in[m][i][j]
hipError_t scatter_square(const double* in, int n, double* out, int np, const int32_t* map,
                          int64_t n_mat, hipStream_t st);
// out (rows x np, zeroed first) with out[r][map[j]] = in[r][j]
hipError_t scatter_cols(const double* in, int rows, int n, double* out, int np, const int32_t* map,
                        hipStream_t st);
// out[m][i][j] = in[m][map[i]][map[j]] (in: np x np per matrix)
hipError_t gather_square(const double* in, int np, double* out, int n, const int32_t* map,
                         int64_t n_mat, hipStream_t st);

// Kept bricks grouped by (second atom s, RI atom c); each group lists the
// bricks (f, s, c) in ascending first atom f.  Groups are ordered by (s, c).
struct BrickGroups {
  int64_t n_kept = 0;
  std::vector<int32_t> gs, gc, goff, seg_atom;   // goff: [n_groups + 1] into seg_*
  std::vector<int64_t> seg_brick;
  std::vector<int32_t> gb_start;                 // [n_atoms + 1] first group of each s
  int n_groups() const { return (int)gs.size(); }
};

// Brick norms on the device, filter (norm < eps dropped), grouping on the host.
// Synchronizes the stream once.
gw_status build_groups(const gw_system* s, double eps, hipStream_t st, Scratch& sc,
                       BrickGroups& out);

// Column panels of PG consecutive atoms for a block-sparse GEMM whose K range
// is the union U_p of the atoms coupled to the panel's columns.  Each group g
// couples column atom col_atom[g] to K atom k_atom[g]; K atom a contributes
// `per` consecutive functions (a * per + i) to kmap.  Panel p holds
// rows_factor * per * |U_p| rows of PC columns starting at off[p].
struct Panels {
  int PG = 1, PC = 0, n_pan = 0;
  std::vector<int32_t> ulen, km_off, kmap, gslot;
  std::vector<int64_t> off;
};
Panels build_panels(int n_atoms, int PG, int PC, const std::vector<int32_t>& col_atom,
                    const std::vector<int32_t>& k_atom, int per, int rows_factor);

// Frobenius norms of `n` consecutive bricks of `bs` doubles (one wave each).
hipError_t brick_norms(const double* t3c, int64_t n, int64_t bs, double* out, hipStream_t st);

// Copy of a stack of n_mat square matrices (n_atoms*na) with every na x na atom
// block of Frobenius norm < eps set to zero; dropped[m*n_atoms^2 + a*n_atoms + b]
// = 1 for dropped blocks (may be null).
hipError_t filter_square_blocks(const double* in, double* out, int n_mat, int n_atoms, int na,
                                double eps, uint8_t* dropped, hipStream_t st);

// out[m][a][b] = Frobenius norm (or its log10 after adding 1e-30) of the
// nb x nb atom blocks of a stack of n_mat square matrices (n_atoms * nb).
hipError_t block_norms_f32(const double* x, int n_mat, int n_atoms, int nb, int log10_out,
                           float* out, hipStream_t st);

// zero every atom block (a, b) of x[m] with keep[m][min(a,b)][max(a,b)] == 0
hipError_t zero_unkept_blocks(double* x, int n_mat, int n_atoms, int nb, const uint8_t* keep,
                              hipStream_t st);

// x[m] lower atom blocks (row atom > col atom) <- transpose of the upper ones.
hipError_t mirror_lower_blocks(double* x, int n_mat, int n, int nb, hipStream_t st);

}  // namespace gw
