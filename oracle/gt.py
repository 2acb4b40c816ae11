"""Imaginary-time density matrices (Eq. 2), FP64, plain sums over MOs.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

Pinned by (tests/test_oracle_gt_chi.py): idempotency and trace of D^occ(0),
D^occ(0) + D^vir(0) = 1 (S = 1), the semigroup law D(t1) D(t2) = D(t1 + t2),
symmetry and positivity; with a non-orthogonal AO basis the metric forms
D S D = D, tr(D S) = n_occ and (D^occ + D^vir)(0) S = 1
(tests/test_oracle_metric.py).
"""
from __future__ import annotations

import numpy as np


def density_matrices(C, eps, n_occ, mu_f, tau):
    """D^occ(tau_j) and D^vir(tau_j), each [n_tau][n_ao][n_ao].

    C is [n_mo][n_ao] (row n = MO n), eps ascending.  The occupied part uses
    exp(+(eps_i - mu_f) tau) over i < n_occ, the virtual part
    exp(-(eps_a - mu_f) tau) over a >= n_occ (Eq. 2 with the energy zero at
    mu_f so that both branches decay).
    """
    C = np.asarray(C, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64) - mu_f
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    co, cv = C[:n_occ], C[n_occ:]
    eo, ev = eps[:n_occ], eps[n_occ:]
    d_occ = np.empty((len(tau), C.shape[1], C.shape[1]))
    d_vir = np.empty_like(d_occ)
    for j, t in enumerate(tau):
        d_occ[j] = co.T @ (np.exp(eo * t)[:, None] * co)
        d_vir[j] = cv.T @ (np.exp(-ev * t)[:, None] * cv)
    return d_occ, d_vir
