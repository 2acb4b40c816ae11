// Quasiparticle energies (Eq. 12), host FP64.
//   Sigma^c_n(i w_k) = sum_j c_kj (vir - occ)(tau_j) + i sum_j s_kj (vir + occ)(tau_j)
// Pade interpolant as a Thiele continued fraction (Vidberg & Serene, J. Low
// Temp. Phys. 29, 179 (1977)):
//   C(z) = a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))
// with a_p = g_p(z_p), g_1(z_i) = f_i and
//   g_p(z_i) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_i)) / ((z_i - z_{p-1}) g_{p-1}(z_i)),
// evaluated with the three-term recurrence for numerator and denominator
// (and their z derivatives).  Virtual states use nodes +i w_k, occupied
// states -i w_k with conjugated values, w_k within the window (the paper's
// 10 eV without options).  Newton-Raphson from E = eps_n on
//   f(E) = E - eps_n + vxc_n - sig_x_n - Re Sigma^c_n(E - mu_F).
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "gw.h"

namespace gw {
void set_error(const std::string& msg);
void clear_error();
}

namespace {

using cplx = std::complex<double>;

std::vector<cplx> thiele_coeffs(const std::vector<cplx>& z, std::vector<cplx> g) {
  const size_t n = z.size();
  std::vector<cplx> a(n);
  if (n == 0) return a;
  a[0] = g[0];
  for (size_t p = 1; p < n; ++p) {
    for (size_t i = p; i < n; ++i) g[i] = (g[p - 1] - g[i]) / ((z[i] - z[p - 1]) * g[i]);
    a[p] = g[p];
  }
  return a;
}

void thiele_eval(const std::vector<cplx>& zn, const std::vector<cplx>& a, cplx z, cplx* val,
                 cplx* der) {
  cplx ap = 0.0, ac = a[0], bp = 1.0, bc = 1.0;
  cplx dap = 0.0, dac = 0.0, dbp = 0.0, dbc = 0.0;
  for (size_t n = 1; n < a.size(); ++n) {
    const cplx fac = (z - zn[n - 1]) * a[n];
    const cplx an = ac + fac * ap, bn = bc + fac * bp;
    const cplx dan = dac + a[n] * ap + fac * dap, dbn = dbc + a[n] * bp + fac * dbp;
    ap = ac; ac = an; bp = bc; bc = bn;
    dap = dac; dac = dan; dbp = dbc; dbc = dbn;
  }
  *val = ac / bc;
  *der = (dac * bc - ac * dbc) / (bc * bc);
}

}  // namespace

extern "C" gw_status gw_continue_qp(int32_t n_gw, const double* sig_occ, const double* sig_vir,
                                    const double* sig_x, const double* eps_n, const double* vxc_n,
                                    const int32_t* is_occ, double mu_f, int32_t n_tau, int32_t n_w,
                                    const double* omega, const double* cos_w, const double* sin_w,
                                    const gw_qp_opts* opts, double* e_qp, int32_t* state_status) {
  gw::clear_error();
  if (n_gw < 1 || n_tau < 1 || n_w < 1 || !sig_occ || !sig_vir || !sig_x || !eps_n || !is_occ ||
      !omega || !cos_w || !sin_w || !e_qp || !state_status || !std::isfinite(mu_f)) {
    gw::set_error("gw_continue_qp: invalid argument");
    return GW_ERR_ARG;
  }
  // without options: the analytic continuation window of the paper's
  // computational details, i[0, +-10 eV] (10 eV in hartree, CODATA 2018)
  const double window = opts ? opts->pade_window : 10.0 / 27.211386245988;
  const double tol = (opts && opts->newton_tol > 0) ? opts->newton_tol : 1e-10;
  const int max_iter = (opts && opts->max_iter > 0) ? opts->max_iter : 100;
  for (int k = 0; k < n_w; ++k)
    if (!(omega[k] > 0) || !std::isfinite(omega[k])) {
      gw::set_error("gw_continue_qp: omega must be positive and finite");
      return GW_ERR_ARG;
    }
  gw_status ret = GW_OK;
  for (int n = 0; n < n_gw; ++n) {
    // transforms to the imaginary axis
    std::vector<cplx> zn, fv;
    for (int k = 0; k < n_w; ++k) {
      if (window > 0 && omega[k] > window) continue;
      double re = 0.0, im = 0.0;
      for (int j = 0; j < n_tau; ++j) {
        const double so = sig_occ[(size_t)n * n_tau + j], sv = sig_vir[(size_t)n * n_tau + j];
        re += cos_w[(size_t)k * n_tau + j] * (sv - so);
        im += sin_w[(size_t)k * n_tau + j] * (sv + so);
      }
      if (is_occ[n]) {
        zn.push_back(cplx(0.0, -omega[k]));
        fv.push_back(cplx(re, -im));
      } else {
        zn.push_back(cplx(0.0, omega[k]));
        fv.push_back(cplx(re, im));
      }
    }
    state_status[n] = GW_ERR_NO_CONVERGE;
    e_qp[n] = std::nan("");
    if (zn.empty()) {
      ret = GW_ERR_NO_CONVERGE;
      continue;
    }
    const std::vector<cplx> a = thiele_coeffs(zn, fv);
    const double vxc = vxc_n ? vxc_n[n] : 0.0;
    double e = eps_n[n];
    for (int it = 0; it < max_iter; ++it) {
      cplx val, der;
      thiele_eval(zn, a, cplx(e - mu_f, 0.0), &val, &der);
      const double f = e - eps_n[n] + vxc - sig_x[n] - val.real();
      const double fp = 1.0 - der.real();
      const double de = -f / fp;
      e += de;
      if (!std::isfinite(e)) break;
      if (std::fabs(de) < tol) {
        state_status[n] = GW_OK;
        e_qp[n] = e;
        break;
      }
    }
    if (state_status[n] != GW_OK) ret = GW_ERR_NO_CONVERGE;
  }
  if (ret != GW_OK) gw::set_error("Newton did not converge for at least one state");
  return ret;
}

extern "C" gw_status gw_evgw_update(int32_t n_mo, int32_t n_occ, const double* eps0, int32_t n_gw,
                                    const int32_t* states, const double* e_qp, double* eps_out,
                                    double* mu_out) {
  gw::clear_error();
  if (n_mo < 2 || n_occ < 1 || n_occ >= n_mo || n_gw < 1 || n_gw > n_mo || !eps0 || !states ||
      !e_qp || !eps_out || !mu_out) {
    gw::set_error("gw_evgw_update: invalid argument");
    return GW_ERR_ARG;
  }
  std::vector<char> seen((size_t)n_mo, 0);
  double d_occ = 0.0, d_vir = 0.0;
  int n_o = 0, n_v = 0;
  for (int n = 0; n < n_gw; ++n) {
    const int i = states[n];
    if (i < 0 || i >= n_mo || seen[i] || !std::isfinite(e_qp[n]) || !std::isfinite(eps0[i])) {
      gw::set_error("gw_evgw_update: states must be distinct indices in [0, n_mo) with finite energies");
      return GW_ERR_ARG;
    }
    seen[i] = 1;
    if (i < n_occ) {
      d_occ += e_qp[n] - eps0[i];
      ++n_o;
    } else {
      d_vir += e_qp[n] - eps0[i];
      ++n_v;
    }
  }
  d_occ = n_o ? d_occ / n_o : 0.0;
  d_vir = n_v ? d_vir / n_v : 0.0;
  for (int i = 0; i < n_mo; ++i) eps_out[i] = eps0[i] + (i < n_occ ? d_occ : d_vir);
  for (int n = 0; n < n_gw; ++n) eps_out[states[n]] = e_qp[n];
  double homo = eps_out[0], lumo = eps_out[n_occ];
  for (int i = 1; i < n_occ; ++i) homo = std::max(homo, eps_out[i]);
  for (int i = n_occ + 1; i < n_mo; ++i) lumo = std::min(lumo, eps_out[i]);
  *mu_out = 0.5 * (homo + lumo);
  if (!(homo < lumo)) {
    gw::set_error("gw_evgw_update: an occupied level ends at or above a virtual one");
    return GW_ERR_NO_CONVERGE;
  }
  return GW_OK;
}

// Energy zero of the Green's function (Eq. 2 decays in tau only when every
// occupied level lies below it and every virtual level above): the midpoint
// of the highest occupied and the lowest virtual level over all channels.
extern "C" gw_status gw_fermi_level(int32_t n_chan, const int32_t* n_mo, const int32_t* n_occ,
                                    const double* const* eps, double* mu_out) {
  gw::clear_error();
  if (n_chan < 1 || n_chan > 16 || !n_mo || !n_occ || !eps || !mu_out) {
    gw::set_error("gw_fermi_level: n_chan in [1, 16] and non-null arrays required");
    return GW_ERR_ARG;
  }
  double homo = -INFINITY, lumo = INFINITY;
  for (int c = 0; c < n_chan; ++c) {
    if (!eps[c] || n_mo[c] < 2 || n_occ[c] < 0 || n_occ[c] > n_mo[c]) {
      gw::set_error("gw_fermi_level: channel " + std::to_string(c) +
                    " needs eps and 0 <= n_occ <= n_mo, n_mo >= 2");
      return GW_ERR_ARG;
    }
    for (int i = 0; i < n_mo[c]; ++i) {
      const double e = eps[c][i];
      if (!std::isfinite(e)) {
        gw::set_error("gw_fermi_level: non-finite energy");
        return GW_ERR_ARG;
      }
      if (i < n_occ[c]) homo = std::max(homo, e);
      else lumo = std::min(lumo, e);
    }
  }
  if (!(homo < lumo)) {
    gw::set_error("gw_fermi_level: an occupied level lies at or above a virtual level "
                  "(no energy zero between them; the Green's function would not decay)");
    return GW_ERR_ARG;
  }
  *mu_out = 0.5 * (homo + lumo);
  return GW_OK;
}
