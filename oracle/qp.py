"""From Sigma(tau) to quasiparticle energies (transforms, Pade, Eq. 12), FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

* ``sigma_iw``: Sigma^c_n(i w_k) = sum_j c_kj (S^vir - S^occ)(tau_j)
                                  + i sum_j s_kj (S^vir + S^occ)(tau_j).
* ``thiele_coeffs`` / ``thiele_eval``: Pade interpolant as a Thiele continued
  fraction (Vidberg & Serene, J. Low Temp. Phys. 29, 179 (1977)):
      C(z) = a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))
  with a_i = g_i(z_i), g_1(z_i) = f_i,
       g_p(z) = (g_{p-1}(z_{p-1}) - g_{p-1}(z)) / ((z - z_{p-1}) g_{p-1}(z)).
  Virtual states use the nodes +i w_k with Sigma^c(i w_k), occupied states the
  nodes -i w_k with conj(Sigma^c(i w_k)), with |w_k| <= window: by default the
  paper's window of 10 eV on the imaginary axis (computational details);
  window=None takes every node.
* ``solve_qp``: Newton-Raphson on
      f(E) = E - eps_n + vxc_n - Sigma^x_n - Re Sigma^c_n(E - mu_F) = 0
  from E = eps_n, derivative from the continued fraction, |dE| < tol.

Pinned by: exact reproduction of rational data by the continued fraction,
Sigma^c = 0 giving eps - vxc + Sigma^x, and the polynomial root of a one-pole
Sigma^c (tests/test_oracle_screen_sigma_qp.py).
"""
from __future__ import annotations

import numpy as np

# the analytic continuation window of the computational details: i[0, +10 eV]
# for virtual and i[0, -10 eV] for occupied states (CODATA 2018 hartree)
PADE_WINDOW_HA = 10.0 / 27.211386245988


def sigma_iw(sig_occ, sig_vir, cos_w, sin_w):
    """[n_gw][n_w] complex from [n_gw][n_tau] real pieces."""
    re = (sig_vir - sig_occ) @ cos_w.T
    im = (sig_vir + sig_occ) @ sin_w.T
    return re + 1j * im


def thiele_coeffs(z, f):
    z = np.asarray(z, dtype=np.complex128)
    g = np.array(f, dtype=np.complex128)
    n = len(z)
    a = np.empty(n, dtype=np.complex128)
    a[0] = g[0]
    for p in range(1, n):
        # g_{p+1}(z_i) for i >= p from g_p
        g[p:] = (g[p - 1] - g[p:]) / ((z[p:] - z[p - 1]) * g[p:])
        a[p] = g[p]
    return a


def thiele_eval(z_nodes, a, z):
    """Value and derivative of the continued fraction at z (complex)."""
    z = complex(z)
    a_prev, a_cur = 0.0 + 0j, a[0]          # A_{0}, A_{1}
    b_prev, b_cur = 1.0 + 0j, 1.0 + 0j      # B_{0}, B_{1}
    da_prev, da_cur = 0j, 0j
    db_prev, db_cur = 0j, 0j
    for n in range(1, len(a)):
        fac = (z - z_nodes[n - 1]) * a[n]
        a_new = a_cur + fac * a_prev
        b_new = b_cur + fac * b_prev
        da_new = da_cur + a[n] * a_prev + fac * da_prev
        db_new = db_cur + a[n] * b_prev + fac * db_prev
        a_prev, a_cur = a_cur, a_new
        b_prev, b_cur = b_cur, b_new
        da_prev, da_cur = da_cur, da_new
        db_prev, db_cur = db_cur, db_new
    val = a_cur / b_cur
    der = (da_cur * b_cur - a_cur * db_cur) / (b_cur * b_cur)
    return val, der


def pade_nodes(omega, sig_iw_n, occupied, window=None):
    omega = np.asarray(omega)
    sel = np.ones(len(omega), dtype=bool) if window is None else (np.abs(omega) <= window)
    if occupied:
        return -1j * omega[sel], np.conj(sig_iw_n[sel])
    return 1j * omega[sel], sig_iw_n[sel]


class NoConvergence(RuntimeError):
    pass


def solve_qp(eps_n, vxc_n, sigx_n, mu_f, z_nodes, a, tol=1e-10, max_iter=100):
    e = float(eps_n)
    for _ in range(max_iter):
        val, der = thiele_eval(z_nodes, a, e - mu_f)
        f = e - eps_n + vxc_n - sigx_n - val.real
        fp = 1.0 - der.real
        de = -f / fp
        e += de
        if not np.isfinite(e):
            break
        if abs(de) < tol:
            return e
    raise NoConvergence(f"Newton did not converge from {eps_n}")


def qp_energies(sig_occ, sig_vir, sig_x, eps_n, vxc_n, is_occ, mu_f, omega,
                cos_w, sin_w, window=PADE_WINDOW_HA, tol=1e-10, max_iter=100):
    """eps^QP for every state (NaN where Newton fails) and a status array
    (0 ok, 1 no convergence)."""
    siw = sigma_iw(sig_occ, sig_vir, cos_w, sin_w)
    out = np.empty(len(eps_n))
    status = np.zeros(len(eps_n), dtype=np.int32)
    for k in range(len(eps_n)):
        zn, fv = pade_nodes(omega, siw[k], bool(is_occ[k]), window)
        a = thiele_coeffs(zn, fv)
        try:
            out[k] = solve_qp(eps_n[k], vxc_n[k], sig_x[k], mu_f, zn, a, tol, max_iter)
        except NoConvergence:
            out[k] = np.nan
            status[k] = 1
    return out, status
