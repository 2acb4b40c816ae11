"""Screening: chi(i w), dielectric matrix, W^c(i w) and W^c(tau) (Eqs. 5-9), FP64.

Test infrastructure (the oracle): used only by tests/, __graft_entry__.smoke()
and the CPU baseline of bench.py, never by the product path.

RI overlap metric S = 1 (the synthetic tensor plays the role of (mu nu P)),
so chi~ = chi and W~ = W (Eqs. 5-6).  Step by step:

  chi(i w_k) = 2 s sum_j c_kj chi(tau_j)       cosine transform, s = spin factor
  V = L L^T                                    Cholesky (Eq. 8)
  eps(i w_k) = 1 - L^T chi(i w_k) L            (Eq. 7)
  W^c(i w_k) = L [eps^-1 - 1] L^T              (Eq. 9), eps^-1 via Cholesky
  W^c(tau_j) = 1/2 sum_k d_jk W^c(i w_k)       inverse cosine transform

Pinned by: eig(eps) >= 1, W^c negative semidefinite, the Cholesky route equal
to the V^{1/2} route, chi = 0 giving W^c = 0, and the single-pole closed form
of the self-energy built on top (tests/test_oracle_screen_sigma_qp.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotSPD(ValueError):
    pass


def chi_omega(chi_tau, cos_w, spin):
    """[n_w][n_ri][n_ri] from [n_tau][n_ri][n_ri]."""
    return np.ascontiguousarray(2.0 * spin * np.einsum("kj,jpq->kpq", cos_w, chi_tau, optimize=True))


def cholesky_lower(a):
    try:
        return sla.cholesky(a, lower=True)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e)) from e


def dielectric(chi_w, L):
    n = L.shape[0]
    return np.eye(n) - L.T @ chi_w @ L


def wc_omega(chi_w, L):
    eps = dielectric(chi_w, L)
    r = cholesky_lower(eps)                       # eps = R R^T
    eps_inv = sla.cho_solve((r, True), np.eye(eps.shape[0]))
    return L @ (eps_inv - np.eye(eps.shape[0])) @ L.T


def screen_w(chi_tau, V, cos_w, icos_w, spin):
    """W^c(tau_j) stack from the chi(tau_j) stack."""
    L = cholesky_lower(V)
    chi_w = chi_omega(chi_tau, cos_w, spin)
    wcw = np.stack([wc_omega(chi_w[k], L) for k in range(chi_w.shape[0])])
    return np.ascontiguousarray(0.5 * np.einsum("jk,kpq->jpq", icos_w, wcw, optimize=True))


def wc_omega_sqrt(chi_w, V):
    """The V^{1/2} form: W^c = V^{1/2} [(1 - V^{1/2} chi V^{1/2})^-1 - 1] V^{1/2}."""
    w, u = np.linalg.eigh(V)
    vh = (u * np.sqrt(w)) @ u.T
    n = V.shape[0]
    eps = np.eye(n) - vh @ chi_w @ vh
    return vh @ (np.linalg.inv(eps) - np.eye(n)) @ vh
