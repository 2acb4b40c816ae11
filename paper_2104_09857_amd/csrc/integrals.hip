// Three-center overlap integrals (Eq. 4) of s-type Gaussian basis functions,
// in the brick layout of gw_system.  Every function is a normalized s-type
// Gaussian g(r) = (2a/pi)^(3/4) exp(-a |r - R|^2); the product of three of
// them (exponents a, b, c at A, B, C) is one Gaussian of exponent s = a+b+c
// scaled by exp(-(ab|A-B|^2 + ac|A-C|^2 + bc|B-C|^2)/s), whose integral is
// (pi/s)^(3/2) (Gaussian product theorem).  Elementwise and bound by the
// output writes: one lane per brick element, the atom triple and the three
// centres looked up per lane.
#include <cmath>

#include "gw_internal.hpp"

namespace gw {
namespace {

struct Fn {
  double ox, oy, oz;   // offset of the centre from its atom
  double a;            // exponent
  double n;            // normalization (2a/pi)^(3/4)
};

__global__ void t3c_gaussian_kernel(const double* __restrict__ xyz, const int32_t* __restrict__ trip,
                                    const Fn* __restrict__ ao, const Fn* __restrict__ ri, int NA,
                                    int NR, int64_t n_trip, double pi15, double* __restrict__ out) {
  const int64_t bs = (int64_t)NA * NA * NR, total = n_trip * bs;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e / bs;
    const int r = (int)(e - t * bs);
    const int mu = r / (NA * NR), rem = r - mu * NA * NR, nu = rem / NR, P = rem - nu * NR;
    const int ia = trip[3 * t], ib = trip[3 * t + 1], ic = trip[3 * t + 2];
    const Fn fa = ao[mu], fb = ao[nu], fc = ri[P];
    const double ax = xyz[3 * ia] + fa.ox, ay = xyz[3 * ia + 1] + fa.oy, az = xyz[3 * ia + 2] + fa.oz;
    const double bx = xyz[3 * ib] + fb.ox, by = xyz[3 * ib + 1] + fb.oy, bz = xyz[3 * ib + 2] + fb.oz;
    const double cx = xyz[3 * ic] + fc.ox, cy = xyz[3 * ic + 1] + fc.oy, cz = xyz[3 * ic + 2] + fc.oz;
    const double dab = (ax - bx) * (ax - bx) + (ay - by) * (ay - by) + (az - bz) * (az - bz);
    const double dac = (ax - cx) * (ax - cx) + (ay - cy) * (ay - cy) + (az - cz) * (az - cz);
    const double dbc = (bx - cx) * (bx - cx) + (by - cy) * (by - cy) + (bz - cz) * (bz - cz);
    const double s = fa.a + fb.a + fc.a;
    const double ex = (fa.a * fb.a * dab + fa.a * fc.a * dac + fb.a * fc.a * dbc) / s;
    out[e] = fa.n * fb.n * fc.n * pi15 / (s * sqrt(s)) * exp(-ex);
  }
}

gw_status fns(int n, const double* expo, const double* off, std::vector<Fn>& out) {
  out.resize(n);
  for (int i = 0; i < n; ++i) {
    GW_CHECK_ARG(std::isfinite(expo[i]) && expo[i] > 0.0, "Gaussian exponents must be finite and > 0");
    const double ox = off ? off[3 * i] : 0.0, oy = off ? off[3 * i + 1] : 0.0,
                 oz = off ? off[3 * i + 2] : 0.0;
    GW_CHECK_ARG(std::isfinite(ox) && std::isfinite(oy) && std::isfinite(oz), "offsets must be finite");
    out[i] = Fn{ox, oy, oz, expo[i], std::pow(2.0 * expo[i] / M_PI, 0.75)};
  }
  return GW_OK;
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" gw_status gw_t3c_gaussian(const gw_system* s, const double* ao_exp,
                                     const double* ao_offset, const double* ri_exp,
                                     const double* ri_offset, double* t3c, hipStream_t st) {
  clear_error();
  // the system's own t3c is not read: its sizes and triple list are
  gw_status rc = check_system_sizes(s);
  if (rc != GW_OK) return rc;
  GW_CHECK_ARG(s->n_trip >= 0 && (s->n_trip == 0 || s->trip), "trip must be given when n_trip > 0");
  for (int64_t i = 0; i < 3 * s->n_trip; ++i)
    GW_CHECK_ARG(s->trip[i] >= 0 && s->trip[i] < s->n_atoms, "triple atom index out of range");
  GW_CHECK_ARG(!s->ao_off && !s->ri_off, "gw_t3c_gaussian takes systems without per-atom offsets");
  GW_CHECK_ARG(s->xyz != nullptr, "the atom coordinates (xyz) are required");
  GW_CHECK_ARG(ao_exp && ri_exp, "ao_exp and ri_exp must be non-null");
  GW_CHECK_ARG(s->n_trip == 0 || t3c != nullptr, "t3c must be non-null");
  for (int i = 0; i < 3 * s->n_atoms; ++i) GW_CHECK_ARG(std::isfinite(s->xyz[i]), "xyz must be finite");
  const int NA = s->ao_per_atom, NR = s->ri_per_atom;
  std::vector<Fn> ao, ri;
  if ((rc = fns(NA, ao_exp, ao_offset, ao)) != GW_OK) return rc;
  if ((rc = fns(NR, ri_exp, ri_offset, ri)) != GW_OK) return rc;
  if (s->n_trip == 0) return GW_OK;
  Scratch sc(st);
  double* d_xyz;
  int32_t* d_trip;
  Fn *d_ao, *d_ri;
  if ((rc = sc.upload(&d_xyz, std::vector<double>(s->xyz, s->xyz + 3 * s->n_atoms))) != GW_OK) return rc;
  if ((rc = sc.upload(&d_trip, std::vector<int32_t>(s->trip, s->trip + 3 * s->n_trip))) != GW_OK) return rc;
  if ((rc = sc.upload(&d_ao, ao)) != GW_OK) return rc;
  if ((rc = sc.upload(&d_ri, ri)) != GW_OK) return rc;
  const int64_t total = s->n_trip * (int64_t)NA * NA * NR;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(t3c_gaussian_kernel, dim3(blocks), dim3(256), 0, st, d_xyz, d_trip, d_ao, d_ri,
                     NA, NR, s->n_trip, std::pow(M_PI, 1.5), t3c);
  GW_HIP(hipGetLastError());
  return GW_OK;
}
